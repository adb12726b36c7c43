"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (max-norm, relative to the largest oracle value, padding
excluded):
  FP64 right-hand side    1e-12  (the stated bar)
  FP64 100 LSERK steps    1e-10  (accumulated roundoff)
  FP32 right-hand side    5e-5   (binary32 rounding of O(Np) dot products
                                   with |D| ~ N^2; the measured number is
                                   printed)
"""
import sys

import numpy as np
import pytest

import dg_inputs as I
from oracle import diag as D
from oracle import lserk as L
from oracle import maxwell as Mx
from oracle import mesh as Me

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dg():
    import torch
    assert torch.cuda.is_available()
    from paper_1211_0582_amd import dg as mod
    return mod


def _case(N, k, seed=0, noise_seed=1, jitter=0.1):
    VX, EToV = I.kuhn_cube(k, jitter, seed)
    m = Me.Mesh(N, VX, EToV)
    u = I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, noise_seed)
    return VX, EToV, m, u


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _gpu_rhs(dg, N, VX, EToV, u, precision="fp64", alpha=1.0):
    import torch
    p = dg.Problem(N, VX, EToV, precision, alpha)
    du = p.pack(u)
    out = p.zeros_state()
    p.rhs(du, out)
    torch.cuda.synchronize()
    r = p.unpack(out)
    p.close()
    return r


@pytest.mark.parametrize("N", range(1, 10))
def test_fp64_rhs_all_orders(dg, N):
    k = 3 if N <= 6 else 2
    _say(f"[gpu] fp64 rhs N={N} k={k}")
    VX, EToV, m, u = _case(N, k)
    ref = Mx.rhs(m, u)
    got = _gpu_rhs(dg, N, VX, EToV, u)
    err = _rel(got, ref)
    _say(f"  rel err {err:.3e}")
    assert err < 1e-12
    for c in range(6):
        assert np.abs(got[c] - ref[c]).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_fp64_rhs_flux_parameter(dg, alpha):
    _say(f"[gpu] fp64 rhs alpha={alpha}")
    VX, EToV, m, u = _case(3, 3, seed=4)
    ref = Mx.rhs(m, u, alpha)
    got = _gpu_rhs(dg, 3, VX, EToV, u, alpha=alpha)
    assert _rel(got, ref) < 1e-12


def test_single_element_all_walls(dg):
    _say("[gpu] single element")
    VX = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    EToV = np.array([[0, 1, 2, 3]], dtype=np.int32)
    m = Me.Mesh(4, VX, EToV)
    u = I.field_noise((6, 1, m.Np), 1.0, 3)
    assert _rel(_gpu_rhs(dg, 4, VX, EToV, u), Mx.rhs(m, u)) < 1e-12


@pytest.mark.parametrize("N,k", [(4, 5), (2, 7), (5, 4)])
def test_ragged_tail_tiles(dg, N, k):
    """K not a multiple of the workgroup tile: the last tile is partial."""
    _say(f"[gpu] ragged N={N} k={k}")
    VX, EToV, m, u = _case(N, k, seed=9)
    info_tile = None
    p = dg.Problem(N, VX, EToV, "fp64")
    info_tile = p.info.tile_elems
    p.close()
    assert m.K % info_tile != 0 or m.K < info_tile
    assert _rel(_gpu_rhs(dg, N, VX, EToV, u), Mx.rhs(m, u)) < 1e-12


def test_config1_fp64_100_lserk_steps(dg):
    """K = 384, N = 3, cavity mode, 100 steps at CFL 0.5."""
    import torch
    _say("[gpu] config-1 100 LSERK steps fp64")
    VX, EToV = I.kuhn_cube(4, 0.1, 0)
    m = Me.Mesh(3, VX, EToV)
    u0 = I.cavity_mode(m.x, m.y, m.z)
    dt = D.dt_cfl(m, 0.5)
    ref = L.integrate(lambda v, t: Mx.rhs(m, v), u0, 0.0, dt, 100)
    p = dg.Problem(3, VX, EToV, "fp64")
    assert abs(p.info.dt_cfl1 * 0.5 - dt) < 1e-15 * dt
    du = p.pack(u0)
    res = p.zeros_state()
    p.rk_step(du, res, 0.0, dt, 100)
    torch.cuda.synchronize()
    got = p.unpack(du)
    p.close()
    err = _rel(got, ref)
    _say(f"  rel err after 100 steps {err:.3e}")
    assert err < 1e-10
    # energy of the GPU state is below the initial energy (upwind dissipation)
    assert D.energy(m, got) < D.energy(m, u0)


def test_fp32_rhs_error_band(dg):
    _say("[gpu] fp32 rhs N=4")
    VX, EToV, m, u = _case(4, 3)
    ref = Mx.rhs(m, u)
    got = _gpu_rhs(dg, 4, VX, EToV, u, "fp32")
    err = _rel(got, ref)
    _say(f"  fp32 rel err {err:.3e}")
    assert err < 5e-5


def test_padding_is_never_read_and_runs_are_deterministic(dg):
    import torch
    _say("[gpu] padding poison + determinism")
    VX, EToV, m, u = _case(4, 2)
    p = dg.Problem(4, VX, EToV, "fp64")
    du = p.pack(u)
    n = m.K * m.Np
    fs = p.info.field_stride
    for c in range(6):
        du[c * fs + n:(c + 1) * fs] = float("nan")
    a, b = p.zeros_state(), p.zeros_state()
    p.rhs(du, a)
    p.rhs(du, b)
    torch.cuda.synchronize()
    ra, rb = p.unpack(a), p.unpack(b)
    p.close()
    assert np.all(np.isfinite(ra))
    assert np.array_equal(ra, rb)
    assert _rel(ra, Mx.rhs(m, u)) < 1e-12


def test_rhs_rejects_aliasing(dg):
    VX, EToV = I.kuhn_cube(1, 0.0, 0)
    p = dg.Problem(2, VX, EToV, "fp64")
    x = p.zeros_state()
    with pytest.raises(dg.DgError) as e:
        p.rhs(x, x)
    assert e.value.status == dg.DG_EINVAL
    p.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 5e-5)])
def test_config2_full_size(dg, precision, tol):
    """K = 82,944 (24^3 x 6), N = 4: the benchmark's launch configuration,
    checked against the oracle on every element."""
    _say(f"[gpu] config-2 full size {precision}")
    VX, EToV, m, u = _case(4, 24)
    ref = Mx.rhs(m, u)
    got = _gpu_rhs(dg, 4, VX, EToV, u, precision)
    err = _rel(got, ref)
    _say(f"  rel err {err:.3e}")
    assert err < tol
