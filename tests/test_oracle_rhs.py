"""Pins for the oracle's right-hand side (CPU only).

* polynomial exactness: a degree-4 field in the space gives the exact
  -curl E at every node, including wall elements;
* the exact discrete energy identity (both sides computed independently), and
  exactly zero rate for the central flux -- this fixes the sign reading of the
  printed flux and the consistency of the neighbour map;
* linearity; invariance under element renumbering;
* brute force on tiny meshes: the assembled operator is M-dissipative
  (M-skew for alpha = 0) and its least-damped eigenvalues approximate the
  cube-cavity frequencies pi*sqrt(l^2+m^2+n^2);
* a wrong sign anywhere in the flux or the curl fails the energy pins.
"""
import numpy as np
import pytest

import dg_inputs as I
from oracle import diag as D
from oracle import maxwell as Mx
from oracle import mesh as Me


def _mesh(N, k, seed=0, jitter=0.1):
    VX, EToV = I.kuhn_cube(k, jitter, seed)
    return Me.Mesh(N, VX, EToV)


def _fields(m, seed=1):
    return I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, seed)


@pytest.mark.parametrize("N,k", [(4, 2), (5, 2), (6, 1)])
def test_polynomial_exactness_including_walls(N, k):
    m = _mesh(N, k)
    x, y = m.x, m.y
    u = np.zeros((6, m.K, m.Np))
    u[2] = x * (1 - x) * y * (1 - y)
    r = Mx.rhs(m, u)
    ex = np.zeros_like(u)
    ex[3] = -x * (1 - x) * (1 - 2 * y)
    ex[4] = (1 - 2 * x) * y * (1 - y)
    assert np.abs(r - ex).max() < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3])
def test_constant_and_linear_fields_on_interior_elements(N):
    m = _mesh(N, 3)
    interior = np.all(m.EToE >= 0, axis=1)
    u = np.zeros((6, m.K, m.Np))
    u[0] = 1.0
    u[4] = 2.0 * m.z - m.x          # H = (0, 2z - x, 0): curl H = (-2, 0, -1)
    r = Mx.rhs(m, u)
    assert np.abs(r[:, interior][[1, 3, 4, 5]]).max() < 1e-12
    assert np.allclose(r[0][interior], -2.0, atol=1e-12)
    assert np.allclose(r[2][interior], -1.0, atol=1e-12)


@pytest.mark.parametrize("N,k,alpha", [(3, 4, 1.0), (3, 4, 0.0), (4, 2, 1.0), (2, 3, 1.0), (6, 1, 1.0), (1, 3, 0.5)])
def test_energy_identity(N, k, alpha):
    m = _mesh(N, k)
    u = _fields(m)
    rate = D.energy_rate(m, u, alpha)
    diss = D.dissipation(m, u, alpha)
    scale = D.energy(m, u) * max(1.0, np.max(m.Fscale)) * (N + 1) ** 2
    assert abs(rate - diss) < 1e-13 * scale
    if alpha == 0.0:
        assert abs(rate) < 1e-13 * scale
    else:
        assert rate < 0.0


def test_linearity():
    m = _mesh(3, 2)
    a = _fields(m, 1)
    b = I.field_noise((6, m.K, m.Np), 1.0, 9)
    lhs = Mx.rhs(m, 2.0 * a - 3.0 * b)
    rhs = 2.0 * Mx.rhs(m, a) - 3.0 * Mx.rhs(m, b)
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(lhs).max()


def test_element_renumbering_invariance():
    VX, EToV = I.kuhn_cube(2, 0.1, 4)
    m = Me.Mesh(3, VX, EToV)
    u = _fields(m)
    perm = np.random.default_rng(3).permutation(m.K)
    m2 = Me.Mesh(3, VX, EToV[perm])
    r1 = Mx.rhs(m, u)
    r2 = Mx.rhs(m2, u[:, perm])
    assert np.abs(r1[:, perm] - r2).max() < 1e-12 * np.abs(r1).max()


def test_sign_error_breaks_energy_identity(monkeypatch):
    """Planted mistake on the CPU: flipping the central E-flux sign must be caught."""
    m = _mesh(3, 2)
    u = _fields(m)
    good = abs(D.energy_rate(m, u, 0.0))
    orig = Mx.surface_flux

    def flipped(mesh, uu, alpha=1.0):
        f = orig(mesh, uu, alpha)
        f[0:3] *= -1.0
        return f

    monkeypatch.setattr(Mx, "surface_flux", flipped)
    bad = abs(D.energy_rate(m, u, 0.0))
    assert good < 1e-15 and bad > 1e-6


@pytest.fixture(scope="module")
def tiny_operator():
    m = _mesh(5, 1, jitter=0.0)
    return m, D.assemble(m, 1.0), D.assemble(m, 0.0), D.block_mass(m)


def test_operator_is_mass_dissipative_and_central_is_skew(tiny_operator):
    m, A, A0, W = tiny_operator
    S = W @ A
    assert np.linalg.eigvalsh(S + S.T).max() < 1e-12
    S0 = W @ A0
    assert np.abs(S0 + S0.T).max() < 1e-12


def test_least_damped_eigenvalues_are_cavity_frequencies(tiny_operator):
    m, A, _, _ = tiny_operator
    lam = np.linalg.eigvals(A)
    assert lam.real.max() < 1e-10
    up = lam[lam.imag > 0.5]
    up = up[np.argsort(np.abs(up.real) / np.abs(up))][:12]
    up = np.sort(up.imag)
    assert np.allclose(up[:3], np.pi * np.sqrt(2.0), atol=2e-3)       # (1,1,0) triplet
    assert np.allclose(up[3:5], np.pi * np.sqrt(3.0), atol=3e-3)      # (1,1,1) pair
