"""Pins for the oracle's reference element (CPU only).

Each check ties the oracle to something other than itself: library GLL points,
Gauss-Jacobi quadrature, exact derivatives of monomials, the discrete
divergence theorem, symmetry of the node set under the 24 vertex
permutations, and the lattice structure of the face nodes.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.special import roots_jacobi

from oracle import refelem as R

ORDERS = list(range(1, 10))


@pytest.mark.parametrize("N", ORDERS)
def test_gll_points_match_legendre_derivative_roots(N):
    x = R.gll_points(N)
    ref = np.sort(np.concatenate([[-1.0, 1.0], np.polynomial.legendre.Legendre.basis(N).deriv().roots().real]))
    assert np.allclose(x, ref, atol=1e-13)


@pytest.mark.parametrize("a,b", [(0, 0), (1, 0), (2, 0), (5, 0), (1, 1), (3, 2)])
def test_jacobi_orthonormal_by_gauss_quadrature(a, b):
    n = 8
    x, w = roots_jacobi(n + 2, a, b)
    P = np.stack([R.jacobi_p(x, a, b, i) for i in range(n + 1)])
    G = (P * w) @ P.T
    assert np.allclose(G, np.eye(n + 1), atol=1e-13)


@pytest.mark.parametrize("a,b", [(0, 0), (2, 0), (1, 1)])
def test_jacobi_derivative_against_finite_difference(a, b):
    x = np.linspace(-0.9, 0.9, 7)
    h = 1e-6
    for n in range(6):
        fd = (R.jacobi_p(x + h, a, b, n) - R.jacobi_p(x - h, a, b, n)) / (2 * h)
        assert np.allclose(R.grad_jacobi_p(x, a, b, n), fd, atol=1e-6)


@pytest.mark.parametrize("N", ORDERS)
def test_node_counts_and_faces(N):
    re = R.ref_element(N)
    assert len(re.r) == (N + 1) * (N + 2) * (N + 3) // 6
    assert re.Fmask.shape == (4, (N + 1) * (N + 2) // 2)
    # all nodes inside the closed reference tetrahedron
    assert np.all(re.r >= -1 - 1e-13) and np.all(re.s >= -1 - 1e-13) and np.all(re.t >= -1 - 1e-13)
    assert np.all(re.r + re.s + re.t <= -1 + 1e-13)


@pytest.mark.parametrize("N", ORDERS)
def test_edge_nodes_are_gll_points(N):
    re = R.ref_element(N)
    sel = (np.abs(1 + re.s) < 1e-12) & (np.abs(1 + re.t) < 1e-12)   # edge v0 -> v1
    assert np.allclose(np.sort(re.r[sel]), R.gll_points(N), atol=1e-13)
    sel = (np.abs(1 + re.r) < 1e-12) & (np.abs(1 + re.s) < 1e-12)   # edge v0 -> v3
    assert np.allclose(np.sort(re.t[sel]), R.gll_points(N), atol=1e-13)


@pytest.mark.parametrize("N", ORDERS)
def test_node_set_invariant_under_vertex_permutations(N):
    re = R.ref_element(N)
    lam = np.stack([-(1 + re.r + re.s + re.t) / 2, (1 + re.r) / 2, (1 + re.s) / 2, (1 + re.t) / 2], axis=1)
    for p in itertools.permutations(range(4)):
        lp = lam[:, p]
        d = np.linalg.norm(lam[:, None, :] - lp[None, :, :], axis=2)
        assert d.min(axis=1).max() < 1e-13


def _monomials(N):
    return [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]


@pytest.mark.parametrize("N", ORDERS)
def test_exact_differentiation_of_monomials(N):
    re = R.ref_element(N)
    r, s, t = re.r, re.s, re.t
    scale = 1.0
    for (a, b, c) in _monomials(N):
        p = r ** a * s ** b * t ** c
        dr = a * r ** max(a - 1, 0) * s ** b * t ** c if a else 0 * r
        ds = b * r ** a * s ** max(b - 1, 0) * t ** c if b else 0 * r
        dt = c * r ** a * s ** b * t ** max(c - 1, 0) if c else 0 * r
        tol = 1e-12 * max(1.0, N * N) * scale
        assert np.abs(re.Dr @ p - dr).max() < tol
        assert np.abs(re.Ds @ p - ds).max() < tol
        assert np.abs(re.Dt @ p - dt).max() < tol
    for D in (re.Dr, re.Ds, re.Dt):
        assert np.abs(D.sum(axis=1)).max() < 1e-12 * N * N


@pytest.mark.parametrize("N", ORDERS)
def test_mass_and_stiffness_match_quadrature_definitions(N):
    re = R.ref_element(N)
    M, S = R.quadrature_mass_stiffness(N)
    assert np.allclose(M, re.M, atol=1e-13, rtol=0)
    assert abs(M.sum() - 4.0 / 3.0) < 1e-13
    for Sq, D in zip(S, (re.Dr, re.Ds, re.Dt)):
        assert np.allclose(np.linalg.solve(M, Sq), D, atol=1e-11 * N * N, rtol=0)


@pytest.mark.parametrize("N", ORDERS)
def test_face_mass_is_reference_triangle_mass(N):
    re = R.ref_element(N)
    for f in range(4):
        assert abs(re.Mf[f].sum() - 2.0) < 1e-13
        # integrates degree <= 2N products on the face exactly: int x^2 over the triangle
        p, q = R.FACE_PARAM[f]
        x = (re.r, re.s, re.t)[p][re.Fmask[f]]
        # int_{ref tri} x^2 dA = 2/3
        assert abs(x @ re.Mf[f] @ x - 2.0 / 3.0) < 1e-13


def _embed(re, f):
    E = np.zeros((re.Np, re.Np))
    idx = re.Fmask[f]
    E[np.ix_(idx, idx)] = re.Mf[f]
    return E


@pytest.mark.parametrize("N", ORDERS)
def test_sbp_discrete_divergence_theorem(N):
    """M D_nu + (M D_nu)^T equals the boundary term int n_nu l_i l_j dS."""
    re = R.ref_element(N)
    M, _ = R.quadrature_mass_stiffness(N)
    E = [_embed(re, f) for f in range(4)]
    Q = [M @ re.Dr, M @ re.Ds, M @ re.Dt]
    # reference normals (scaled by face area / param area): r: +f2 -f3, s: +f2 -f1, t: +f2 -f0
    targets = [E[2] - E[3], E[2] - E[1], E[2] - E[0]]
    for Qn, T in zip(Q, targets):
        assert np.abs(Qn + Qn.T - T).max() < 1e-12 * N * N


@pytest.mark.parametrize("N", ORDERS)
def test_lift_is_inverse_mass_times_embedded_face_mass(N):
    re = R.ref_element(N)
    M, _ = R.quadrature_mass_stiffness(N)
    assert np.abs(M @ re.LIFT - re.Emat).max() < 1e-12 * N


@pytest.mark.parametrize("N", ORDERS)
def test_face_nodes_lattice_and_mass_consistent_across_faces(N):
    """Every face carries the same lattice points and the same face mass matrix
    (up to the node permutation that the lattice fixes)."""
    re = R.ref_element(N)
    L = R.lattice(N)
    key0 = None
    for f, fv in enumerate(R.FACE_VERTS):
        sub = L[re.Fmask[f]][:, list(fv)]
        keys = [tuple(x) for x in sub]
        assert len(set(keys)) == re.Nfp
        if key0 is None:
            key0, M0 = keys, re.Mf[f]
            continue
        perm = [keys.index(k) for k in key0]
        assert np.allclose(re.Mf[f][np.ix_(perm, perm)], M0, atol=1e-13)


def test_alpha_table_and_sizes():
    assert R.alpha_opt(4) == pytest.approx(0.1002)
    assert R.n_p(4) == 35 and R.n_fp(4) == 15 and R.n_p(9) == 220


def test_warp_vanishes_for_linear_and_is_odd():
    x = np.linspace(-0.99, 0.99, 11)
    assert np.all(R.warp_over_bubble(1, x) == 0.0)
    for N in (3, 4, 7):
        assert np.allclose(R.warp_over_bubble(N, -x), -R.warp_over_bubble(N, x), atol=1e-15)
        # warp(e_i) = GLL_i - e_i at the equispaced points
        e = -1.0 + 2.0 * np.arange(N + 1) / N
        w = R.warp_over_bubble(N, e[1:-1]) * (1 - e[1:-1] ** 2)
        assert np.allclose(w, R.gll_points(N)[1:-1] - e[1:-1], atol=1e-14)
