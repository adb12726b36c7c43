"""Pins of the general linear-hyperbolic oracle (oracle/linear.py), CPU only.

Each check is fixed by something other than the oracle's own formula:
  * for Maxwell's equations in conservation form, the generic flux
    1/2 (A_n - alpha |A_n|)(u- - u+) with |A_n| from an eigendecomposition is
    the closed-form Maxwell flux of oracle/maxwell.py, element by element,
    for every alpha and boundary code;
  * for symmetric systems the energy rate equals a sum of face integrals of
    the traces (discrete divergence theorem); central fluxes with reflecting
    boundaries conserve energy exactly, upwind fluxes dissipate it;
  * linear fields are differentiated exactly (interior elements);
  * the closed-form acoustic cavity mode is reached at the method's rate.
"""
import numpy as np
import pytest

import dg_inputs as I
from oracle import diag as D
from oracle import linear as Li
from oracle import lserk as L
from oracle import maxwell as Mx
from oracle import mesh as Me


@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("N", [1, 3, 4])
def test_generic_flux_is_the_maxwell_flux(N, alpha):
    VX, EToV = I.kuhn_cube(2, 0.1, 3)
    bc = I.random_face_bc(EToV.shape[0], 5)
    m = Me.Mesh(N, VX, EToV, face_bc=bc)
    u = I.field_noise((6, m.K, m.Np), 1.0, 2)
    r1 = Mx.rhs(m, u, alpha)
    r2 = Li.rhs(m, Li.maxwell_system(), u, alpha)
    assert np.abs(r1 - r2).max() <= 1e-13 * np.abs(r1).max()


def test_maxwell_matrices_are_symmetric_with_unit_speeds():
    s = Li.maxwell_system()
    for d in range(3):
        assert np.array_equal(s.A[d], s.A[d].T)
    n = np.array([0.36, 0.48, 0.8])
    w = np.linalg.eigvalsh(s.A_n(n))
    assert np.allclose(np.sort(w), [-1, -1, 0, 0, 1, 1])


@pytest.mark.parametrize("system", ["acoustics", "maxwell"])
@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_energy_rate_from_traces(system, alpha):
    s = Li.acoustics_system() if system == "acoustics" else Li.maxwell_system()
    VX, EToV = I.kuhn_cube(2, 0.1, 7)
    bc = I.random_face_bc(EToV.shape[0], 8)
    m = Me.Mesh(3, VX, EToV, face_bc=bc)
    u = I.field_noise((s.m, m.K, m.Np), 1.0, 9)
    a = Li.energy_rate(m, s, u, alpha)
    b = Li.energy_rate_from_traces(m, s, u, alpha)
    scale = float(np.sum(m.J[None, :, None] * np.abs(u) * np.abs(Li.rhs(m, s, u, alpha) @ m.re.M.T)))
    assert abs(a - b) <= 1e-12 * scale
    if system == "maxwell":
        assert abs(a - D.dissipation(m, u, alpha)) <= 1e-12 * scale


def test_acoustics_central_flux_with_reflecting_walls_conserves_energy():
    s = Li.acoustics_system()
    VX, EToV = I.kuhn_cube(2, 0.1, 1)
    bc = I.random_face_bc(EToV.shape[0], 2, codes=(0, 1))
    m = Me.Mesh(4, VX, EToV, face_bc=bc)
    u = I.field_noise((4, m.K, m.Np), 1.0, 3)
    scale = float(np.sum(m.J[None, :, None] * np.abs(u) * np.abs(Li.rhs(m, s, u, 0.0) @ m.re.M.T)))
    assert abs(Li.energy_rate(m, s, u, 0.0)) <= 1e-13 * scale
    assert Li.energy_rate(m, s, u, 1.0) < 0


def test_linear_fields_are_differentiated_exactly():
    """p = a.x + c, v = b (constant): dp/dt = -div v = 0, dv/dt = -grad p = -a
    on elements with no boundary face."""
    s = Li.acoustics_system()
    VX, EToV = I.kuhn_cube(3, 0.1, 4)
    m = Me.Mesh(2, VX, EToV)
    a = np.array([0.3, -1.2, 0.7])
    u = np.zeros((4, m.K, m.Np))
    u[0] = a[0] * m.x + a[1] * m.y + a[2] * m.z + 0.4
    u[1:] = np.array([0.5, -0.25, 2.0])[:, None, None]
    r = Li.rhs(m, s, u, 1.0)
    inner = np.all(m.EToE >= 0, axis=1)
    assert inner.any()
    assert np.abs(r[0, inner]).max() < 1e-11
    for d in range(3):
        assert np.abs(r[1 + d, inner] + a[d]).max() < 1e-11


def test_acoustic_cavity_mode_converges():
    s = Li.acoustics_system()
    N, T = 3, 0.25
    errs = []
    for k in (2, 4):
        VX, EToV = I.kuhn_cube(k, 0.1, k)
        m = Me.Mesh(N, VX, EToV)
        u0 = Li.acoustic_cavity_mode(m.x, m.y, m.z, 0.0)
        ns = int(np.ceil(T / D.dt_cfl(m, 0.5)))
        u = L.integrate(lambda v, t: Li.rhs(m, s, v), u0, 0.0, T / ns, ns)
        ex = Li.acoustic_cavity_mode(m.x, m.y, m.z, T)
        errs.append(np.sqrt(2 * Li.energy(m, u - ex)) / np.sqrt(2 * Li.energy(m, u0)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > N + 0.5, (errs, rate)
