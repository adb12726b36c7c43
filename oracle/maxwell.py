"""Semi-discrete nodal DG right-hand side for 3D Maxwell (FP64, NumPy).  Test infrastructure only.

The operator is the paper's semi-discrete scheme (Section 2):
    du/dt = - sum_nu D^nu F(u) + L [ n.F - (n.F)* ]   on every element,
for the linear Maxwell flux, split as in Section 2.1 into F(u), local
differentiation, flux gather and flux lifting.  With u = (E, H) and a
permittivity eps and permeability mu constant per element (the conservation
law of Section 2 with the material matrix on the time derivative):
eps dE/dt = curl H, mu dH/dt = -curl E, so -D F(u) is the discrete curl built
from the reference Dr, Ds, Dt and the element's constant metric, divided by
eps or mu.

Flux (results section, Maxwell upwind flux of the flux figure, part a; the
H part by the E -> H, H -> -E duality), with jumps dE = E- - E+,
dH = H- - H+, impedances Z = sqrt(mu / eps) and admittances Y = 1 / Z of the
own (-) and neighbour (+) element:
    fE = [ -Z+ n x dH + alpha (n (n . dE) - dE) ] / (Z- + Z+)
    fH = [  Y+ n x dE + alpha (n (n . dH) - dH) ] / (Y- + Y+)
and rhs += LIFT (Fscale * f) before the division by eps or mu.  With
eps = mu = 1 this is 1/2 [ -n x dH + alpha (n (n.dE) - dE) ] and
1/2 [ n x dE + alpha (n (n.dH) - dH) ].  alpha = 1 is upwind, alpha = 0
central.  The weights are those of the Riemann solution between two media
(the reading taken for the paper's generic flux); they are pinned by exact
energy conservation of the central flux, which fails for any other
weighting.

Boundary faces take an exterior state built from the interior trace,
E+ = a_E E-, H+ = a_H H-, so dE = (1 - a_E) E-, dH = (1 - a_H) H-, with
(a_E, a_H) per condition code of the mesh:
    0  perfectly conducting wall (n x E = 0):          (-1,  1)
    1  perfectly magnetic-conducting wall (n x H = 0): ( 1, -1)
    2  absorbing face (no incoming wave):              ( 0,  0)
Code 1 is code 0 seen through the E -> H, H -> -E duality of the equations;
code 2 makes the upwind flux that of a zero exterior, so an outgoing wave
leaves without reflection.  A boundary face's exterior has the material of
its element (Z+ = Z-).

The sign reading (the printed flux is the term subtracted, i.e. the
n.F - (n.F)* of the scheme equals the expression above) is the one under which
the discrete energy is non-increasing; tests/test_oracle_rhs.py pins it by
the exact discrete energy identity.

Layout: u is (6, K, Np) FP64 in the field order (Ex, Ey, Ez, Hx, Hy, Hz).
"""
from __future__ import annotations

import numpy as np


def curl(mesh, fx, fy, fz):
    """Discrete curl of a nodal vector field (each (K, Np))."""
    re = mesh.re

    def grads(f):
        fr = f @ re.Dr.T
        fs = f @ re.Ds.T
        ft = f @ re.Dt.T
        dx = mesh.rx[:, None] * fr + mesh.sx[:, None] * fs + mesh.tx[:, None] * ft
        dy = mesh.ry[:, None] * fr + mesh.sy[:, None] * fs + mesh.ty[:, None] * ft
        dz = mesh.rz[:, None] * fr + mesh.sz[:, None] * fs + mesh.tz[:, None] * ft
        return dx, dy, dz

    xx, xy, xz = grads(fx)
    yx, yy, yz = grads(fy)
    zx, zy, zz = grads(fz)
    return zy - yz, xz - zx, yx - xy


def traces(mesh, u):
    """Interior and exterior traces at face nodes, each (6, K, 4, Nfp), and the
    boundary mask (K, 4)."""
    K, Np, Nfp = mesh.K, mesh.Np, mesh.Nfp
    uM = u[:, :, mesh.re.Fmask]                       # (6, K, 4, Nfp)
    flat = u.reshape(6, K * Np)
    bnd = mesh.EToE < 0
    idx = np.where(mesh.vmapP >= 0, mesh.vmapP, 0)
    uP = flat[:, idx]                                  # (6, K, 4, Nfp)
    return uM, uP, bnd


#: exterior-state factors (a_E, a_H) per boundary condition code
MIRROR = {0: (-1.0, 1.0), 1: (1.0, -1.0), 2: (0.0, 0.0)}


def surface_flux(mesh, u, alpha: float = 1.0):
    """Fscale * [n.F - (n.F)*] at every face node: (6, K, 4, Nfp)."""
    uM, uP, bnd = traces(mesh, u)
    dE = uM[0:3] - uP[0:3]
    dH = uM[3:6] - uP[3:6]
    aE = np.zeros(bnd.shape)
    aH = np.zeros(bnd.shape)
    for code, (ae, ah) in MIRROR.items():
        aE[mesh.bc == code] = ae
        aH[mesh.bc == code] = ah
    b = bnd[None, :, :, None]
    dE = np.where(b, (1.0 - aE[None, :, :, None]) * uM[0:3], dE)
    dH = np.where(b, (1.0 - aH[None, :, :, None]) * uM[3:6], dH)
    n = np.stack([mesh.nx, mesh.ny, mesh.nz])[:, :, :, None]  # (3, K, 4, 1)
    ndE = np.sum(n * dE, axis=0)
    ndH = np.sum(n * dH, axis=0)
    Zm = np.repeat(mesh.Z[:, None], 4, axis=1)
    Zp = np.where(bnd, Zm, mesh.Z[np.where(bnd, 0, mesh.EToE)])
    Zm, Zp = Zm[None, :, :, None], Zp[None, :, :, None]
    Ym, Yp = 1.0 / Zm, 1.0 / Zp
    fE = (-Zp * np.cross(n, dH, axis=0) + alpha * (n * ndE - dE)) / (Zm + Zp)
    fH = (Yp * np.cross(n, dE, axis=0) + alpha * (n * ndH - dH)) / (Ym + Yp)
    f = np.concatenate([fE, fH], axis=0)
    return f * mesh.Fscale[None, :, :, None]


def rhs(mesh, u, alpha: float = 1.0):
    """du/dt for u of shape (6, K, Np)."""
    u = np.asarray(u, dtype=np.float64)
    K, Np, Nfp = mesh.K, mesh.Np, mesh.Nfp
    out = np.empty_like(u)
    cx, cy, cz = curl(mesh, u[3], u[4], u[5])
    out[0], out[1], out[2] = cx, cy, cz
    cx, cy, cz = curl(mesh, u[0], u[1], u[2])
    out[3], out[4], out[5] = -cx, -cy, -cz
    f = surface_flux(mesh, u, alpha).reshape(6, K, 4 * Nfp)
    out += f @ mesh.re.LIFT.T
    out[0:3] /= mesh.eps[None, :, None]
    out[3:6] /= mesh.mu[None, :, None]
    return out
