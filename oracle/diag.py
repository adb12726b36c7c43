"""Diagnostics for the DG oracle: energy, its exact dissipation, errors, the
assembled operator and the time-step rule.  Test infrastructure only.

Energy: E(u) = 1/2 sum_k J_k (eps_k E_k^T M E_k + mu_k H_k^T M H_k), the
M^k-norm of the global-matrix definitions (Section 2) with M^k = J_k M
(Section 2.1), weighted by the material (1/2 sum J u^T M u for eps = mu = 1).

Dissipation: for the scheme and flux of ``oracle.maxwell`` the discrete
energy rate is exactly
    sum_k J_k (eps E^T M rhs_E + mu H^T M rhs_H)
      = - alpha sum_{interior faces} [ |n x dE|^2 / (Z- + Z+) + |n x dH|^2 / (Y- + Y+) ]_f
        + sum_{boundary faces} ( - (a_E + a_H)/2 [ H- . (n x E-) ]_f
             - alpha/2 [ (1 - a_E) |n x E-|^2 / Z + (1 - a_H) Z |n x H-|^2 ]_f ),
where [g]_f = sJ_f sum g^T M_f g integrates over the face with the face mass
matrix and (a_E, a_H) are the boundary face's exterior-state factors
(E+ = a_E E-, H+ = a_H H-).  It follows from the divergence of E x H (the
volume term integrates to -[n . (E- x H-)]_f per face), the central part of
the flux cancelling between the two sides of every interior face.  Perfectly
conducting walls give - alpha [ |n x E-|^2 ]_f.
``dissipation`` evaluates the right side from traces only.

Parity: ``energy``/``dissipation`` are pinned against each other through the
oracle RHS (tests/test_oracle_rhs.py) and by alpha = 0 giving exactly 0;
``assemble`` is a column-by-column application of the RHS.
"""
from __future__ import annotations

import numpy as np

from .maxwell import MIRROR, rhs, traces


def _material(mesh):
    """(6, K, 1) weights eps (E fields) and mu (H fields) of the energy."""
    return np.concatenate([np.repeat(mesh.eps[None, :], 3, axis=0),
                           np.repeat(mesh.mu[None, :], 3, axis=0)])[:, :, None]


def energy(mesh, u):
    u = np.asarray(u, dtype=np.float64)
    Mu = u @ mesh.re.M.T                               # (6, K, Np)
    return 0.5 * float(np.sum(mesh.J[None, :, None] * _material(mesh) * u * Mu))


def energy_rate(mesh, u, alpha: float = 1.0):
    """sum_k J_k (eps E^T M rhs_E + mu H^T M rhs_H) computed through the oracle RHS."""
    r = rhs(mesh, u, alpha)
    Mr = r @ mesh.re.M.T
    return float(np.sum(mesh.J[None, :, None] * _material(mesh) * u * Mr))


def dissipation(mesh, u, alpha: float = 1.0):
    """Right side of the energy identity, from face traces only."""
    uM, uP, bnd = traces(mesh, u)
    n = np.stack([mesh.nx, mesh.ny, mesh.nz])[:, :, :, None]
    Mf = mesh.re.Mf                                      # (4, Nfp, Nfp)

    def face_form(g, h):
        # g, h: (3, K, 4, Nfp) -> (K, 4) sum_c g_c^T M_f h_c
        Mh = np.einsum("fij,ckfj->ckfi", Mf, h)
        return np.sum(g * Mh, axis=(0, 3))

    ncdE = np.cross(n, uM[0:3] - uP[0:3], axis=0)
    ncdH = np.cross(n, uM[3:6] - uP[3:6], axis=0)
    ncE = np.cross(n, uM[0:3], axis=0)
    ncH = np.cross(n, uM[3:6], axis=0)
    interior = ~bnd
    Zm = np.repeat(mesh.Z[:, None], 4, axis=1)
    Zp = np.where(bnd, Zm, mesh.Z[np.where(bnd, 0, mesh.EToE)])
    fi = face_form(ncdE, ncdE) / (Zm + Zp) + face_form(ncdH, ncdH) / (1.0 / Zm + 1.0 / Zp)
    total = -alpha * np.sum((mesh.sJ * fi)[interior]) * 0.5  # each interior face seen twice
    for code, (aE, aH) in MIRROR.items():
        sel = mesh.bc == code
        if not np.any(sel):
            continue
        fb = (-0.5 * (aE + aH) * face_form(uM[3:6], ncE)
              - 0.5 * alpha * ((1.0 - aE) * face_form(ncE, ncE) / Zm + (1.0 - aH) * Zm * face_form(ncH, ncH)))
        total += np.sum((mesh.sJ * fb)[sel])
    return float(total)


def mass_norm(mesh, u):
    return float(np.sqrt(2.0 * energy(mesh, u)))


def assemble(mesh, alpha: float = 1.0):
    """Dense operator matrix A with rhs(u).ravel() = A @ u.ravel() (tiny meshes only)."""
    n = 6 * mesh.K * mesh.Np
    Amat = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        Amat[:, j] = rhs(mesh, e.reshape(6, mesh.K, mesh.Np), alpha).ravel()
        e[j] = 0.0
    return Amat


def block_mass(mesh):
    """Diagonal-block global mass matrix (M^k (x) I_6) matching u.ravel() order."""
    n = 6 * mesh.K * mesh.Np
    W = np.zeros((n, n))
    for c in range(6):
        for k in range(mesh.K):
            o = (c * mesh.K + k) * mesh.Np
            W[o:o + mesh.Np, o:o + mesh.Np] = mesh.J[k] * mesh.re.M
    return W


def dt_cfl(mesh, cfl: float = 0.5):
    """Time step reading dt = CFL * 2 / ((N+1)^2 * max Fscale)  (dt ~ dx / N^2)."""
    return cfl * 2.0 / ((mesh.N + 1) ** 2 * float(np.max(mesh.Fscale)))
