"""Nodal DG right-hand side for the 3D compressible Euler equations (FP64, NumPy).  Test infrastructure only.

A nonlinear conservation law in the form of Section 2, du/dt + div F(u) = 0,
with u = (rho, rho u, rho v, rho w, E) and, for gamma = 1.4,
    p = (gamma - 1) (E - |m|^2 / (2 rho)),   m = rho (u, v, w),
    F_d(u) = (m_d, m m_d / rho + p e_d, (E + p) m_d / rho).
The semi-discrete scheme is the strong nodal DG form with the flux
collocated at the nodes (D_d applied to the nodal values of F_d(u)):
    du/dt = - sum_d D_d F_d(u) + L Fscale [ n.F(u-) - F* ],
with the local Lax-Friedrichs flux
    F* = 1/2 n.(F(u-) + F(u+)) + alpha/2 lambda (u- - u+),
    lambda = max(|n.m-| / rho- + c-, |n.m+| / rho+ + c+),  c = sqrt(gamma p / rho),
so n.F(u-) - F* = 1/2 n.(F(u-) - F(u+)) - alpha/2 lambda (u- - u+).
Boundary codes: 0 slip wall (rho+ = rho-, m+ = m- - 2 n (n.m-), E+ = E-),
1 and 2 transmissive (u+ = u-).

Parity: pinned by tests/test_oracle_euler.py -- uniform flow and a resting
density perturbation at uniform pressure are exact steady states (rhs = 0 to
roundoff); the discrete conservation identity (every conserved quantity
changes only through boundary fluxes, computed from traces); and the
linearisation about a resting state equals the linear oracle with the Euler
flux Jacobians and the Rusanov penalty at the sound speed.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def pressure(u, gamma=GAMMA):
    rho, m, E = u[0], u[1:4], u[4]
    return (gamma - 1.0) * (E - 0.5 * np.sum(m * m, axis=0) / rho)


def flux(u, gamma=GAMMA):
    """F_d(u) for d = x, y, z: (3, 5, ...)."""
    rho, m, E = u[0], u[1:4], u[4]
    p = pressure(u, gamma)
    vel = m / rho
    F = np.empty((3, 5) + u.shape[1:])
    for d in range(3):
        F[d, 0] = m[d]
        for j in range(3):
            F[d, 1 + j] = m[j] * vel[d] + (p if j == d else 0.0)
        F[d, 4] = (E + p) * vel[d]
    return F


def sound_speed(u, gamma=GAMMA):
    return np.sqrt(gamma * pressure(u, gamma) / u[0])


def exterior(mesh, uM):
    """Exterior traces of boundary faces: (5, K, 4, Nfp) with interior faces untouched."""
    uP = uM.copy()
    n = np.stack([mesh.nx, mesh.ny, mesh.nz])[:, :, :, None]        # (3, K, 4, 1)
    wall = (mesh.EToE < 0) & (mesh.bc == 0)
    nm = np.sum(n * uM[1:4], axis=0)
    refl = uM[1:4] - 2.0 * n * nm
    uP[1:4] = np.where(wall[None, :, :, None], refl, uM[1:4])
    return uP


def traces(mesh, u):
    K, Np = mesh.K, mesh.Np
    uM = u[:, :, mesh.re.Fmask]
    bnd = mesh.EToE < 0
    uP = u.reshape(5, K * Np)[:, np.where(mesh.vmapP >= 0, mesh.vmapP, 0)]
    ext = exterior(mesh, uM)
    uP = np.where(bnd[None, :, :, None], ext, uP)
    return uM, uP


def numerical_flux_difference(mesh, uM, uP, gamma=GAMMA, alpha=1.0):
    """n.F(u-) - F* at every face node: (5, K, 4, Nfp)."""
    n = np.stack([mesh.nx, mesh.ny, mesh.nz])[:, None, :, :, None]  # (3, 1, K, 4, 1)
    FM = np.sum(n * flux(uM, gamma), axis=0)
    FP = np.sum(n * flux(uP, gamma), axis=0)
    nn = n[:, 0]
    lam = np.maximum(np.abs(np.sum(nn * uM[1:4], axis=0)) / uM[0] + sound_speed(uM, gamma),
                     np.abs(np.sum(nn * uP[1:4], axis=0)) / uP[0] + sound_speed(uP, gamma))
    return 0.5 * (FM - FP) - 0.5 * alpha * lam[None] * (uM - uP)


def rhs(mesh, u, gamma=GAMMA, alpha=1.0):
    u = np.asarray(u, dtype=np.float64)
    K, Nfp = mesh.K, mesh.Nfp
    re = mesh.re
    F = flux(u, gamma)                                    # (3, 5, K, Np)
    out = np.zeros_like(u)
    met = {0: (mesh.rx, mesh.sx, mesh.tx), 1: (mesh.ry, mesh.sy, mesh.ty), 2: (mesh.rz, mesh.sz, mesh.tz)}
    for d in range(3):
        a, b, c = met[d]
        for q in range(5):
            f = F[d, q]
            out[q] -= a[:, None] * (f @ re.Dr.T) + b[:, None] * (f @ re.Ds.T) + c[:, None] * (f @ re.Dt.T)
    uM, uP = traces(mesh, u)
    g = numerical_flux_difference(mesh, uM, uP, gamma, alpha) * mesh.Fscale[None, :, :, None]
    out += g.reshape(5, K, 4 * Nfp) @ re.LIFT.T
    return out


def total_rate(mesh, r):
    """sum_k J_k 1^T M r_q for each conserved quantity q: (5,)."""
    w = mesh.J[:, None] * np.sum(mesh.re.M, axis=0)[None, :]   # (K, Np): J_k (1^T M)_i
    return np.einsum("kn,qkn->q", w, r)


def boundary_flux_rate(mesh, u, gamma=GAMMA, alpha=1.0):
    """- sum over boundary faces of the integral of F*: (5,), from traces only."""
    uM, uP = traces(mesh, u)
    n = np.stack([mesh.nx, mesh.ny, mesh.nz])[:, None, :, :, None]
    FM = np.sum(n * flux(uM, gamma), axis=0)
    Fstar = FM - numerical_flux_difference(mesh, uM, uP, gamma, alpha)
    Mf1 = np.sum(mesh.re.Mf, axis=1)                              # (4, Nfp): 1^T M_f per face
    per = np.einsum("fj,qkfj->qkf", Mf1, Fstar) * mesh.sJ[None]
    bnd = mesh.EToE < 0
    return -np.sum(np.where(bnd[None], per, 0.0), axis=(1, 2))


def jacobians_at_rest(rho0, p0, gamma=GAMMA):
    """Flux Jacobians A_d = dF_d/du at the resting state (rho0, 0, p0): (3, 5, 5)."""
    H0 = (p0 / (gamma - 1.0) + p0) / rho0
    A = np.zeros((3, 5, 5))
    for d in range(3):
        A[d, 0, 1 + d] = 1.0
        A[d, 1 + d, 4] = gamma - 1.0
        A[d, 4, 1 + d] = H0
    return A
