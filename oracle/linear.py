"""Nodal DG right-hand side for a general linear hyperbolic system (FP64, NumPy).  Test infrastructure only.

The conservation law of Section 2, du/dt + div F(u) = 0, with the linear flux
F_d(u) = A_d u (A_d constant m x m matrices, d = x, y, z), discretised by the
same semi-discrete scheme as the Maxwell oracle:
    du/dt = - sum_d A_d D_d u + L [ n.F - (n.F)* ]
on every element (D_d the physical derivative built from Dr, Ds, Dt and the
constant metric, Section 2.1).  The numerical flux is the central average
plus an upwind penalty,
    (n.F)* = 1/2 A_n (u- + u+) + alpha/2 |A_n| (u- - u+),  A_n = sum_d n_d A_d,
so n.F - (n.F)* = 1/2 (A_n - alpha |A_n|)(u- - u+), with |A_n| the matrix
absolute value (eigendecomposition; the A_d of the systems here are
symmetric).  alpha = 1 is upwind, alpha = 0 central.  For Maxwell's
equations in conservation form this is exactly the flux of the Maxwell
oracle (tests/test_oracle_linear.py checks it element by element).

A boundary face takes the exterior state u+ = B_b(n) u- of its condition
code b, given per system as a function of the outward normal.

Parity: pinned by tests/test_oracle_linear.py -- identity with the Maxwell
oracle for the Maxwell matrices (all alpha, all boundary codes), the exact
discrete energy identity for symmetric systems computed from face traces
alone, exact differentiation of linear fields, and the closed-form acoustic
cavity mode converging at the method's rate.
"""
from __future__ import annotations

import numpy as np



class LinearSystem:
    """m fields, A (3, m, m) flux matrices and boundary states {code: B(n)}.

    The upwind penalty uses |A_n| (symmetric A_d); with ``speed`` given it is
    the local Lax-Friedrichs (Rusanov) penalty speed * I instead, for any A_d."""

    def __init__(self, names, A, boundary, speed=None):
        self.names = tuple(names)
        self.m = len(self.names)
        self.A = np.asarray(A, dtype=np.float64)
        if self.A.shape != (3, self.m, self.m):
            raise ValueError("A must have shape (3, m, m)")
        self.boundary = dict(boundary)
        self.speed = speed

    def A_n(self, n):
        """A_n for normals n (..., 3): (..., m, m)."""
        return np.einsum("...d,dij->...ij", n, self.A)

    def abs_A_n(self, n):
        if self.speed is not None:
            return np.broadcast_to(self.speed * np.eye(self.m), n.shape[:-1] + (self.m, self.m))
        w, V = np.linalg.eigh(self.A_n(n))
        return np.einsum("...ik,...k,...jk->...ij", V, np.abs(w), V)


def maxwell_system():
    """(Ex, Ey, Ez, Hx, Hy, Hz): dE/dt - curl H = 0, dH/dt + curl E = 0, so
    (A_n u)_E = -n x H and (A_n u)_H = n x E; walls: conducting (E+ = -E-,
    H+ = H-), magnetic-conducting (the dual), absorbing (zero exterior)."""
    A = np.zeros((3, 6, 6))
    for d in range(3):
        e = np.zeros(3)
        e[d] = 1.0
        for j in range(3):
            h = np.zeros(3)
            h[j] = 1.0
            A[d, 0:3, 3 + j] = -np.cross(e, h)
            A[d, 3:6, j] = np.cross(e, h)
    ident = np.eye(6)
    bc = {0: lambda n: np.broadcast_to(np.diag([-1.0, -1, -1, 1, 1, 1]), n.shape[:-1] + (6, 6)),
          1: lambda n: np.broadcast_to(np.diag([1.0, 1, 1, -1, -1, -1]), n.shape[:-1] + (6, 6)),
          2: lambda n: np.zeros(n.shape[:-1] + (6, 6))}
    del ident
    return LinearSystem(("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"), A, bc)


def acoustics_system():
    """(p, vx, vy, vz): dp/dt + div v = 0, dv/dt + grad p = 0 (unit density and
    sound speed).  Boundary codes: 0 rigid wall (v+ = v- - 2 n (n.v-),
    p+ = p-), 1 pressure release (p+ = -p-, v+ = v-), 2 absorbing (zero
    exterior)."""
    A = np.zeros((3, 4, 4))
    for d in range(3):
        A[d, 0, 1 + d] = 1.0
        A[d, 1 + d, 0] = 1.0

    def rigid(n):
        B = np.zeros(n.shape[:-1] + (4, 4))
        B[..., 0, 0] = 1.0
        B[..., 1:, 1:] = np.eye(3) - 2.0 * n[..., :, None] * n[..., None, :]
        return B

    def release(n):
        return np.broadcast_to(np.diag([-1.0, 1, 1, 1]), n.shape[:-1] + (4, 4))

    return LinearSystem(("p", "vx", "vy", "vz"), A,
                        {0: rigid, 1: release, 2: lambda n: np.zeros(n.shape[:-1] + (4, 4))})


def acoustic_cavity_mode(x, y, z, t: float = 0.0):
    """Closed-form (1,1,0) mode of the unit cube with rigid walls:
    p = cos(pi x) cos(pi y) cos(w t), v = (pi / w) (sin(pi x) cos(pi y),
    cos(pi x) sin(pi y), 0) sin(w t), w = pi sqrt(2); it satisfies both
    equations and v.n = 0 on all six walls.  Shape (4,) + x.shape."""
    w = np.pi * np.sqrt(2.0)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    p = np.cos(np.pi * x) * np.cos(np.pi * y) * np.cos(w * t)
    vx = (np.pi / w) * np.sin(np.pi * x) * np.cos(np.pi * y) * np.sin(w * t)
    vy = (np.pi / w) * np.cos(np.pi * x) * np.sin(np.pi * y) * np.sin(w * t)
    return np.stack([p, vx, vy, np.zeros_like(x)])


def _grad(mesh, f):
    re = mesh.re
    fr, fs, ft = f @ re.Dr.T, f @ re.Ds.T, f @ re.Dt.T
    dx = mesh.rx[:, None] * fr + mesh.sx[:, None] * fs + mesh.tx[:, None] * ft
    dy = mesh.ry[:, None] * fr + mesh.sy[:, None] * fs + mesh.ty[:, None] * ft
    dz = mesh.rz[:, None] * fr + mesh.sz[:, None] * fs + mesh.tz[:, None] * ft
    return np.stack([dx, dy, dz])                      # (3, K, Np)


def exterior_traces(mesh, sys, u):
    """Interior and exterior traces (m, K, 4, Nfp), boundary states applied."""
    m, K, Np = u.shape
    uM = u[:, :, mesh.re.Fmask]                           # (m, K, 4, Nfp)
    bnd = mesh.EToE < 0
    uP = u.reshape(m, K * Np)[:, np.where(mesh.vmapP >= 0, mesh.vmapP, 0)]
    n = np.stack([mesh.nx, mesh.ny, mesh.nz], axis=-1)   # (K, 4, 3)
    for code, Bfun in sys.boundary.items():
        sel = bnd & (mesh.bc == code)
        if np.any(sel):
            B = Bfun(n[sel])                                # (nsel, m, m)
            uP[:, sel, :] = np.einsum("sij,jsk->isk", B, uM[:, sel, :])
    return uM, uP, n


def rhs(mesh, sys, u, alpha: float = 1.0):
    """du/dt for u of shape (m, K, Np)."""
    u = np.asarray(u, dtype=np.float64)
    m, K, Nfp = sys.m, mesh.K, mesh.Nfp
    g = np.stack([_grad(mesh, u[c]) for c in range(m)])  # (m, 3, K, Np)
    out = -np.einsum("dij,jdkn->ikn", sys.A, g)
    uM, uP, n = exterior_traces(mesh, sys, u)
    P = 0.5 * (sys.A_n(n) - alpha * sys.abs_A_n(n))      # (K, 4, m, m)
    f = np.einsum("kfij,jkfn->ikfn", P, uM - uP) * mesh.Fscale[None, :, :, None]
    out += f.reshape(m, K, 4 * Nfp) @ mesh.re.LIFT.T
    return out


def energy(mesh, u):
    u = np.asarray(u, dtype=np.float64)
    return 0.5 * float(np.sum(mesh.J[None, :, None] * u * (u @ mesh.re.M.T)))


def energy_rate(mesh, sys, u, alpha: float = 1.0):
    """sum_k J_k u^T M rhs through the RHS."""
    r = rhs(mesh, sys, u, alpha)
    return float(np.sum(mesh.J[None, :, None] * u * (r @ mesh.re.M.T)))


def energy_rate_from_traces(mesh, sys, u, alpha: float = 1.0):
    """The same rate from face traces only: for symmetric A_d the volume term
    integrates to -1/2 of u^T A_n u over the element boundary (the discrete
    divergence theorem of the operators), so per face and side
        [ -1/2 u-^T A_n u- + u-^T 1/2 (A_n - alpha |A_n|)(u- - u+) ]_f,
    [g]_f = sJ sum over face-node pairs with the face mass matrix."""
    uM, uP, n = exterior_traces(mesh, sys, u)
    An = sys.A_n(n)
    P = 0.5 * (An - alpha * sys.abs_A_n(n))
    a = np.einsum("kfij,jkfn->ikfn", An, uM)
    b = np.einsum("kfij,jkfn->ikfn", P, uM - uP)
    Mf = mesh.re.Mf                                      # (4, Nfp, Nfp)
    g = -0.5 * a + b                                     # (m, K, 4, Nfp)
    Mg = np.einsum("fij,ckfj->ckfi", Mf, g)
    per_face = np.sum(uM * Mg, axis=(0, 3))              # (K, 4)
    return float(np.sum(mesh.sJ * per_face))
