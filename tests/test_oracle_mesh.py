"""Pins for the oracle's geometry and connectivity (CPU only)."""
import numpy as np
import pytest

import dg_inputs as I
from oracle import mesh as Me
from oracle import refelem as R


@pytest.fixture(scope="module", params=[(3, 4, 0), (2, 3, 7), (5, 2, 3)])
def mesh(request):
    N, k, seed = request.param
    VX, EToV = I.kuhn_cube(k, 0.1, seed)
    return Me.Mesh(N, VX, EToV), k


def test_cube_volume_and_boundary_area(mesh):
    m, k = mesh
    assert abs(np.sum(m.J) * 4.0 / 3.0 - 1.0) < 1e-13
    assert abs(np.sum(2.0 * m.sJ[m.EToE < 0]) - 6.0) < 1e-12
    assert m.n_boundary_faces == 12 * k * k


def test_unjittered_jacobian_closed_form():
    k = 3
    VX, EToV = I.kuhn_cube(k, 0.0, 0)
    m = Me.Mesh(2, VX, EToV)
    assert np.allclose(m.J, (1.0 / k) ** 3 / 8.0, rtol=1e-13)


def test_normals_unit_orthogonal_and_closed_surface(mesh):
    m, _ = mesh
    n = np.stack([m.nx, m.ny, m.nz], axis=2)
    assert np.allclose(np.linalg.norm(n, axis=2), 1.0, atol=1e-14)
    v = m.VX[m.EToV]
    for f, (a, b, c) in enumerate(R.FACE_VERTS):
        for e in (v[:, b] - v[:, a], v[:, c] - v[:, a]):
            assert np.abs(np.einsum("kd,kd->k", n[:, f], e)).max() < 1e-13
        # outward: points away from the opposite vertex
        opp = ({0, 1, 2, 3} - {a, b, c}).pop()
        assert np.all(np.einsum("kd,kd->k", n[:, f], v[:, a] - v[:, opp]) > 0)
    # divergence theorem for a constant field: sum_f area_f n_f = 0
    closure = np.einsum("kf,kfd->kd", 2.0 * m.sJ, n)
    assert np.abs(closure).max() < 1e-14


def test_metric_inverts_the_affine_map(mesh):
    m, _ = mesh
    re = m.re
    # x_r computed by differentiating node coordinates must invert (rx .. tz)
    for X in (m.x, m.y, m.z):
        assert np.all(np.isfinite(X))
    xr, xs, xt = m.x @ re.Dr.T, m.x @ re.Ds.T, m.x @ re.Dt.T
    # d x / d x = rx x_r + sx x_s + tx x_t = 1
    assert np.allclose(m.rx[:, None] * xr + m.sx[:, None] * xs + m.tx[:, None] * xt, 1.0, atol=1e-12)
    yr, ys, yt = m.y @ re.Dr.T, m.y @ re.Ds.T, m.y @ re.Dt.T
    assert np.allclose(m.rx[:, None] * yr + m.sx[:, None] * ys + m.tx[:, None] * yt, 0.0, atol=1e-12)


def test_matched_traces_coincide_and_are_reciprocal(mesh):
    m, _ = mesh
    X = np.stack([m.x.ravel(), m.y.ravel(), m.z.ravel()], axis=1)
    own = (np.arange(m.K)[:, None, None] * m.Np + m.re.Fmask[None, :, :])
    inner = m.vmapP >= 0
    d = np.linalg.norm(X[own[inner]] - X[m.vmapP[inner]], axis=1)
    assert d.max() < 1e-14
    # reciprocity per face slot: the partner face maps back onto our own nodes
    for k in range(m.K):
        for f in range(4):
            k2, f2 = m.EToE[k, f], m.EToF[k, f]
            if k2 < 0:
                continue
            assert m.EToE[k2, f2] == k and m.EToF[k2, f2] == f
            assert set(m.vmapP[k2, f2].tolist()) == set(own[k, f].tolist())
            assert set(m.vmapP[k, f].tolist()) == set(own[k2, f2].tolist())
    # every face appears at most twice
    assert np.all((m.EToE >= 0) == (m.EToF >= 0))


def test_fscale_definition(mesh):
    m, _ = mesh
    v = m.VX[m.EToV]
    for f, (a, b, c) in enumerate(R.FACE_VERTS):
        area = 0.5 * np.linalg.norm(np.cross(v[:, b] - v[:, a], v[:, c] - v[:, a]), axis=1)
        vol = np.abs(np.linalg.det(np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2))) / 6
        # Fscale = (area/2) / (vol / (4/3))
        assert np.allclose(m.Fscale[:, f], (area / 2) / (vol * 0.75), rtol=1e-13)


def test_inputs_are_seeded_and_conforming():
    VX1, E1 = I.kuhn_cube(3, 0.1, 5)
    VX2, E2 = I.kuhn_cube(3, 0.1, 5)
    assert np.array_equal(VX1, VX2) and np.array_equal(E1, E2)
    VX3, _ = I.kuhn_cube(3, 0.1, 6)
    assert not np.array_equal(VX1, VX3)
    # boundary vertices stay on the cube surface
    onb = np.any((np.abs(VX1) < 1e-15) | (np.abs(VX1 - 1) < 1e-15), axis=1)
    assert onb.sum() == 4 ** 3 - 2 ** 3
    draws = I.batch_draws()
    assert len(draws) == 64 and all(4 <= k <= 20 and 2 <= n <= 7 for k, n, _ in draws)
