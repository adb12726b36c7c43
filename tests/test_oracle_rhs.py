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


# ---------------------------------------------------------------------------
# Boundary conditions other than the perfectly conducting wall.
# ---------------------------------------------------------------------------
def _dual(u):
    """E -> H, H -> -E: a symmetry of the Maxwell equations."""
    return np.concatenate([u[3:6], -u[0:3]])


@pytest.mark.parametrize("N,alpha", [(3, 1.0), (2, 0.5), (4, 0.0)])
def test_magnetic_wall_is_the_dual_of_the_conducting_wall(N, alpha):
    """A perfectly magnetic-conducting wall is a conducting wall seen through
    the duality of the equations: rhs_PMC(dual u) = dual rhs_PEC(u)."""
    VX, EToV = I.kuhn_cube(2, 0.1, 5)
    pec = Me.Mesh(N, VX, EToV)
    pmc = Me.Mesh(N, VX, EToV, np.ones((EToV.shape[0], 4), dtype=np.int8))
    u = _fields(pec)
    lhs = Mx.rhs(pmc, _dual(u), alpha)
    rhs = _dual(Mx.rhs(pec, u, alpha))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()
    # and the two walls really differ
    assert np.abs(Mx.rhs(pmc, u, alpha) - Mx.rhs(pec, u, alpha)).max() > 1e-3 * np.abs(rhs).max()


@pytest.mark.parametrize("N", [2, 3, 5])
def test_outgoing_plane_wave_with_mixed_walls_is_exact(N):
    """E = (0, x^2, 0), H = (0, 0, x^2) is a wave moving in +x with
    dE/dt = (0, -2x, 0), dH/dt = (0, 0, -2x).  With an absorbing face at
    x = 1 (the wave leaves there), conducting walls at y = 0, 1 (E normal to
    them), magnetic walls at z = 0, 1 (H normal to them) and the fields zero
    at x = 0, every jump and every boundary penalty vanishes, so the upwind
    scheme reproduces the exact time derivative at every node."""
    VX, EToV = I.kuhn_cube(2, 0.1, 3)
    bc = I.cube_face_bc(VX, EToV, {"x1": 2, "y0": 0, "y1": 0, "z0": 1, "z1": 1})
    m = Me.Mesh(N, VX, EToV, bc)
    u = np.zeros((6, m.K, m.Np))
    u[1] = m.x ** 2
    u[5] = m.x ** 2
    ex = np.zeros_like(u)
    ex[1] = -2 * m.x
    ex[5] = -2 * m.x
    assert np.abs(Mx.rhs(m, u) - ex).max() < 1e-11
    # a conducting wall at x = 1 reflects the wave: no longer exact there
    m0 = Me.Mesh(N, VX, EToV, I.cube_face_bc(VX, EToV, {"z0": 1, "z1": 1}))
    assert np.abs(Mx.rhs(m0, u) - ex).max() > 0.1


@pytest.mark.parametrize("N,alpha,seed", [(3, 1.0, 1), (2, 0.5, 2), (4, 0.0, 3), (1, 1.0, 4)])
def test_energy_identity_with_mixed_boundary_codes(N, alpha, seed):
    VX, EToV = I.kuhn_cube(2, 0.1, seed)
    m = Me.Mesh(N, VX, EToV, I.random_face_bc(EToV.shape[0], seed))
    assert set(np.unique(m.bc[m.EToE < 0])) == {0, 1, 2}
    u = _fields(m)
    rate = D.energy_rate(m, u, alpha)
    diss = D.dissipation(m, u, alpha)
    scale = D.energy(m, u) * max(1.0, np.max(m.Fscale)) * (N + 1) ** 2
    assert abs(rate - diss) < 1e-13 * scale
    if alpha == 0.0:
        assert abs(rate) < 1e-13 * scale
    else:
        assert rate < 0.0


def test_boundary_codes_are_checked_and_ignored_on_interior_faces():
    VX, EToV = I.kuhn_cube(1, 0.0, 0)
    with pytest.raises(ValueError):
        Me.Mesh(2, VX, EToV, np.full((6, 4), 3, dtype=np.int8))
    VX, EToV = I.kuhn_cube(2, 0.1, 0)
    m0 = Me.Mesh(2, VX, EToV)
    codes = np.zeros((m0.K, 4), dtype=np.int8)
    codes[m0.EToE >= 0] = 7                      # interior entries are not read
    m1 = Me.Mesh(2, VX, EToV, codes)
    u = _fields(m0)
    assert np.array_equal(Mx.rhs(m0, u), Mx.rhs(m1, u))


# ---------------------------------------------------------------------------
# Materials: permittivity eps and permeability mu constant per element.
# ---------------------------------------------------------------------------
def _materials(K, seed):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(-1.0, 1.5, K)), np.exp(rng.uniform(-1.0, 1.0, K))


@pytest.mark.parametrize("N,alpha,seed", [(3, 1.0, 1), (2, 0.5, 2), (4, 0.0, 3), (3, 0.0, 4)])
def test_energy_identity_with_materials(N, alpha, seed):
    """eps- and mu-weighted energy: the rate equals the derived dissipation
    exactly, and the central flux conserves it exactly -- which holds only
    for the impedance weights of the flux."""
    VX, EToV = I.kuhn_cube(2, 0.1, seed)
    eps, mu = _materials(EToV.shape[0], seed)
    m = Me.Mesh(N, VX, EToV, I.random_face_bc(EToV.shape[0], seed), eps, mu)
    u = _fields(m)
    rate = D.energy_rate(m, u, alpha)
    diss = D.dissipation(m, u, alpha)
    scale = D.energy(m, u) * max(1.0, np.max(m.Fscale)) * (N + 1) ** 2 * np.max(1.0 / np.minimum(eps, mu))
    assert abs(rate - diss) < 1e-13 * scale
    if alpha == 0.0:
        assert abs(rate) < 1e-13 * scale
    else:
        assert rate < 0.0


def test_swapped_impedance_weights_break_conservation(monkeypatch):
    """Planted mistake on the CPU: weighting the jump by the own impedance
    instead of the neighbour's makes the central flux gain or lose energy."""
    VX, EToV = I.kuhn_cube(2, 0.1, 5)
    eps, mu = _materials(EToV.shape[0], 5)
    m = Me.Mesh(3, VX, EToV, None, eps, mu)
    u = _fields(m)
    good = abs(D.energy_rate(m, u, 0.0))
    orig = Mx.surface_flux

    def swapped(mesh, uu, alpha=1.0):
        # recompute fE with Z- in place of Z+ (alpha = 0 part only)
        uM, uP, bnd = Mx.traces(mesh, uu)
        f = orig(mesh, uu, alpha)
        Zm = np.repeat(mesh.Z[:, None], 4, axis=1)
        Zp = np.where(bnd, Zm, mesh.Z[np.where(bnd, 0, mesh.EToE)])
        f[0:3] *= (Zm / Zp)[None, :, :, None]
        return f

    monkeypatch.setattr(Mx, "surface_flux", swapped)
    bad = abs(D.energy_rate(m, u, 0.0))
    assert good < 1e-13 * D.energy(m, u) and bad > 1e-6 * D.energy(m, u)


@pytest.mark.parametrize("N", [4, 5])
def test_polynomial_exactness_with_piecewise_materials(N):
    """E = (0, 0, x(1-x)y(1-y)), H = 0 has no jumps and satisfies the
    conducting walls, so in every element dH/dt = -curl E / mu exactly and
    dE/dt = 0, whatever the materials."""
    VX, EToV = I.kuhn_cube(2, 0.1, 6)
    eps, mu = _materials(EToV.shape[0], 6)
    m = Me.Mesh(N, VX, EToV, None, eps, mu)
    x, y = m.x, m.y
    u = np.zeros((6, m.K, m.Np))
    u[2] = x * (1 - x) * y * (1 - y)
    ex = np.zeros_like(u)
    ex[3] = -x * (1 - x) * (1 - 2 * y) / mu[:, None]
    ex[4] = (1 - 2 * x) * y * (1 - y) / mu[:, None]
    assert np.abs(Mx.rhs(m, u) - ex).max() < 1e-11


def test_homogeneous_material_scales_time():
    """eps = mu = c everywhere: same impedance as vacuum, light speed 1/c,
    so the right-hand side is the vacuum one divided by c."""
    VX, EToV = I.kuhn_cube(2, 0.1, 7)
    K = EToV.shape[0]
    m0 = Me.Mesh(3, VX, EToV)
    mc = Me.Mesh(3, VX, EToV, None, np.full(K, 2.5), np.full(K, 2.5))
    u = _fields(m0)
    assert np.abs(Mx.rhs(mc, u) - Mx.rhs(m0, u) / 2.5).max() < 1e-13 * np.abs(Mx.rhs(m0, u)).max()
    with pytest.raises(ValueError):
        Me.Mesh(3, VX, EToV, None, np.full(K, -1.0), None)
