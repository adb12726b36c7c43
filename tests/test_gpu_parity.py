"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Every kernel variant ("valu": vector ALUs; "mfma": matrix cores with the
Runge-Kutta stage fused into the epilogue) is compared with the oracle on the
same seeded inputs.  Tolerances (max-norm, relative to the largest oracle
value, padding excluded):
  FP64 right-hand side    1e-12  (the stated bar)
  FP64 100 LSERK steps    1e-10  (accumulated roundoff)
  FP32 right-hand side    5e-5   (binary32 rounding of O(Np)-term dot
                                   products with |D| ~ N^2; the measured value
                                   is printed)
"""
import functools
import sys

import numpy as np
import pytest

import dg_inputs as I
from oracle import diag as D
from oracle import lserk as L
from oracle import maxwell as Mx
from oracle import mesh as Me

pytestmark = pytest.mark.gpu

VARIANTS = ("valu", "mfma")
TOL = {"fp64": 1e-12, "fp32": 5e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dg():
    import torch
    assert torch.cuda.is_available()
    from paper_1211_0582_amd import dg as mod
    return mod


@functools.lru_cache(maxsize=None)
def _case(N, k, seed=0, noise_seed=1, alpha=1.0):
    VX, EToV = I.kuhn_cube(k, 0.1, seed)
    m = Me.Mesh(N, VX, EToV)
    u = I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, noise_seed)
    return VX, EToV, m, u, Mx.rhs(m, u, alpha)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _problem(dg, N, VX, EToV, precision, variant, alpha=1.0):
    try:
        p = dg.Problem(N, VX, EToV, precision, alpha)
    except dg.DgError as e:
        if e.status == dg.DG_EUNSUPPORTED:
            pytest.skip(f"no kernel at all for N={N} {precision}")
        raise
    try:
        p.set_variant(variant)
    except dg.DgError as e:
        p.close()
        if e.status == dg.DG_EUNSUPPORTED:
            pytest.skip(f"variant {variant} not built for N={N} {precision}")
        raise
    return p


def _gpu_rhs(dg, N, VX, EToV, u, precision, variant, alpha=1.0):
    import torch
    p = _problem(dg, N, VX, EToV, precision, variant, alpha)
    du = p.pack(u)
    out = p.zeros_state()
    p.rhs(du, out)
    torch.cuda.synchronize()
    r = p.unpack(out)
    p.close()
    return r


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N", range(1, 10))
def test_rhs_all_orders(dg, N, precision, variant):
    k = 3 if N <= 6 else 2
    _say(f"[gpu] rhs N={N} k={k} {precision} {variant}")
    VX, EToV, m, u, ref = _case(N, k)
    got = _gpu_rhs(dg, N, VX, EToV, u, precision, variant)
    err = _rel(got, ref)
    _say(f"  rel err {err:.3e}")
    assert err < TOL[precision]
    if precision == "fp64":
        for c in range(6):
            assert np.abs(got[c] - ref[c]).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_fp64_rhs_flux_parameter(dg, alpha, variant):
    _say(f"[gpu] fp64 rhs alpha={alpha} {variant}")
    VX, EToV, m, u, ref = _case(3, 3, seed=4, alpha=alpha)
    got = _gpu_rhs(dg, 3, VX, EToV, u, "fp64", variant, alpha=alpha)
    assert _rel(got, ref) < 1e-12


@pytest.mark.parametrize("variant", VARIANTS)
def test_single_element_all_walls(dg, variant):
    _say(f"[gpu] single element {variant}")
    VX = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    EToV = np.array([[0, 1, 2, 3]], dtype=np.int32)
    m = Me.Mesh(4, VX, EToV)
    u = I.field_noise((6, 1, m.Np), 1.0, 3)
    assert _rel(_gpu_rhs(dg, 4, VX, EToV, u, "fp64", variant), Mx.rhs(m, u)) < 1e-12


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("N,k", [(4, 5), (2, 7), (5, 5), (3, 1)])
def test_ragged_tail_tiles(dg, N, k, variant):
    """K not a multiple of the elements per workgroup: the last tile is partial."""
    _say(f"[gpu] ragged N={N} k={k} {variant}")
    VX, EToV, m, u, ref = _case(N, k, seed=9)
    p = _problem(dg, N, VX, EToV, "fp64", variant)
    tile = p.info.tile_elems
    p.close()
    assert m.K % tile != 0
    assert _rel(_gpu_rhs(dg, N, VX, EToV, u, "fp64", variant), ref) < 1e-12


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("nsteps", [100, 7])
def test_config1_fp64_lserk_steps(dg, variant, nsteps):
    """K = 384, N = 3, cavity mode at CFL 0.5: nsteps steps in one call (an odd
    stage count exercises the fused variant's final buffer copy)."""
    import torch
    _say(f"[gpu] config-1 {nsteps} LSERK steps fp64 {variant}")
    VX, EToV = I.kuhn_cube(4, 0.1, 0)
    m = Me.Mesh(3, VX, EToV)
    u0 = I.cavity_mode(m.x, m.y, m.z)
    dt = D.dt_cfl(m, 0.5)
    ref = L.integrate(lambda v, t: Mx.rhs(m, v), u0, 0.0, dt, nsteps)
    p = _problem(dg, 3, VX, EToV, "fp64", variant)
    assert abs(p.info.dt_cfl1 * 0.5 - dt) < 1e-15 * dt
    du = p.pack(u0)
    res = p.zeros_state()
    p.rk_step(du, res, 0.0, dt, nsteps)
    torch.cuda.synchronize()
    got = p.unpack(du)
    p.close()
    err = _rel(got, ref)
    _say(f"  rel err after {nsteps} steps {err:.3e}")
    assert err < 1e-10
    assert D.energy(m, got) < D.energy(m, u0)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "f16x3"])
def test_residual_is_not_read_at_the_first_stage(dg, precision, variant):
    """The first stage has A_1 = 0 and must not read res: a residual array full
    of NaN on entry gives the same result as a zeroed one, and both match the
    oracle's step."""
    import torch
    _say(f"[gpu] NaN residual on entry {precision} {variant}")
    VX, EToV, m, u, _ = _case(3, 3)
    dt = D.dt_cfl(m, 0.5)
    ref = L.integrate(lambda v, t: Mx.rhs(m, v), u, 0.0, dt, 3)
    outs = []
    for fill in (0.0, float("nan")):
        p = _problem(dg, 3, VX, EToV, precision, variant)
        du = p.pack(u)
        res = p.empty_state()
        res.fill_(fill)
        p.rk_step(du, res, 0.0, dt, 3)
        torch.cuda.synchronize()
        outs.append(p.unpack(du))
        p.close()
    assert np.all(np.isfinite(outs[1]))
    assert np.array_equal(outs[0], outs[1])
    tol = {"fp64": 1e-12, "fp32": 1e-5, "f16x3": 1e-4}[precision]
    assert _rel(outs[1], ref) < tol


@pytest.mark.parametrize("variant", VARIANTS)
def test_fp32_lserk_steps(dg, variant):
    import torch
    _say(f"[gpu] fp32 20 LSERK steps {variant}")
    VX, EToV = I.kuhn_cube(3, 0.1, 0)
    m = Me.Mesh(4, VX, EToV)
    u0 = I.cavity_mode(m.x, m.y, m.z)
    dt = D.dt_cfl(m, 0.5)
    ref = L.integrate(lambda v, t: Mx.rhs(m, v), u0, 0.0, dt, 20)
    p = _problem(dg, 4, VX, EToV, "fp32", variant)
    du = p.pack(u0)
    res = p.zeros_state()
    p.rk_step(du, res, 0.0, dt, 20)
    torch.cuda.synchronize()
    err = _rel(p.unpack(du), ref)
    p.close()
    _say(f"  fp32 rel err after 20 steps {err:.3e}")
    assert err < 1e-5


@pytest.mark.parametrize("variant", VARIANTS)
def test_padding_is_never_read_and_runs_are_deterministic(dg, variant):
    import torch
    _say(f"[gpu] padding poison + determinism {variant}")
    VX, EToV, m, u, ref = _case(4, 2)
    p = _problem(dg, 4, VX, EToV, "fp64", variant)
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
    assert _rel(ra, ref) < 1e-12


TUNING_VARIANTS = ("mfma_waves", "mfma_prefetch", "mfma_occupancy", "mfma_interleave", "mfma_lift", "mfma_tail")


@pytest.mark.parametrize("variant", TUNING_VARIANTS)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "f16x3", "bf16x3"])
@pytest.mark.parametrize("N", range(1, 10))
def test_every_tuning_variant_matches_the_oracle(dg, N, precision, variant):
    """Each tuning configuration of the matrix-core kernel (the autotuner's
    search space) gives the operator to the precision's tolerance, in the
    right-hand side and in a fused LSERK step."""
    import torch
    VX, EToV, m, u, ref = _case(N, 2)
    p = _problem(dg, N, VX, EToV, precision, variant)
    _say(f"[gpu] tuning variant {variant} N={N} {precision}")
    du = p.pack(u)
    out = p.zeros_state()
    p.rhs(du, out)
    torch.cuda.synchronize()
    got = p.unpack(out)
    tol = dict(TOL, **SPLIT_TOL)[precision] * (max(1.0, N / 4) if precision in SPLIT_TOL else 1.0)
    assert _rel(got, ref) < tol
    dt = D.dt_cfl(m, 0.5)
    step_ref = L.integrate(lambda v, t: Mx.rhs(m, v), u, 0.0, dt, 1)
    res = p.zeros_state()
    p.rk_step(du, res, 0.0, dt, 1)
    torch.cuda.synchronize()
    assert _rel(p.unpack(du), step_ref) < {"fp64": 1e-12, "fp32": 1e-5}.get(precision, 1e-3)
    p.close()


def test_variants_agree_and_default(dg):
    import torch
    VX, EToV, m, u, ref = _case(4, 2)
    p = dg.Problem(4, VX, EToV, "fp64")
    from paper_1211_0582_amd import autotune
    assert p.variant == (autotune.lookup(4, "fp64", p.info.K, arch="gfx950") or "mfma")
    with pytest.raises(dg.DgError) as e:
        p.set_variant(dg.dg_variant_count())
    assert e.value.status == dg.DG_EINVAL
    p.close()
    p = dg.Problem(9, VX, EToV, "fp64")       # FP64 at N = 9: only the vector kernel is built
    assert p.variant == "valu"
    with pytest.raises(dg.DgError) as e:
        p.set_variant("mfma")
    assert e.value.status == dg.DG_EUNSUPPORTED
    assert p.variant == "valu"
    p.close()
    assert dg.dg_variant_name(dg.dg_variant_count()) is None
    torch.cuda.synchronize()


def test_rhs_rejects_aliasing(dg):
    VX, EToV = I.kuhn_cube(1, 0.0, 0)
    p = dg.Problem(2, VX, EToV, "fp64")
    x = p.zeros_state()
    with pytest.raises(dg.DgError) as e:
        p.rhs(x, x)
    assert e.value.status == dg.DG_EINVAL
    with pytest.raises(ValueError):
        p.rhs(x, x[:10])
    p.close()


def test_state_arrays_must_be_16_byte_aligned(dg):
    """The kernels write state arrays with 16-byte stores: a state array that
    starts 8 bytes into an allocation is refused before any launch."""
    import torch
    VX, EToV = I.kuhn_cube(1, 0.0, 0)
    p = dg.Problem(2, VX, EToV, "fp64")
    n = p.info.state_elems
    buf = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    good, off = buf[:n], buf[1:]
    res = p.zeros_state()
    for call in (lambda: p.rhs(off, res), lambda: p.rhs(good, off), lambda: p.rk_step(off, res, 0.0, 1e-3, 1)):
        with pytest.raises(dg.DgError) as e:
            call()
        assert e.value.status == dg.DG_EINVAL and "16-byte" in str(e.value)
    p.rhs(good, res)
    torch.cuda.synchronize()
    p.close()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config2_full_size(dg, precision, variant):
    """K = 82,944 (24^3 x 6), N = 4: the benchmark's launch configuration,
    checked against the oracle on every element."""
    _say(f"[gpu] config-2 full size {precision} {variant}")
    VX, EToV, m, u, ref = _case(4, 24)
    got = _gpu_rhs(dg, 4, VX, EToV, u, precision, variant)
    err = _rel(got, ref)
    _say(f"  rel err {err:.3e}")
    assert err < TOL[precision]


@pytest.mark.parametrize("variant", VARIANTS)
def test_config2_fused_stage_matches_rhs_plus_update(dg, variant):
    """One LSERK step at full size against the oracle's step (FP64)."""
    import torch
    _say(f"[gpu] config-2 one LSERK step fp64 {variant}")
    VX, EToV, m, u, _ = _case(4, 24)
    dt = D.dt_cfl(m, 0.5)
    ref = L.integrate(lambda v, t: Mx.rhs(m, v), u, 0.0, dt, 1)
    p = _problem(dg, 4, VX, EToV, "fp64", variant)
    du = p.pack(u)
    res = p.zeros_state()
    p.rk_step(du, res, 0.0, dt, 1)
    torch.cuda.synchronize()
    err = _rel(p.unpack(du), ref)
    p.close()
    _say(f"  rel err {err:.3e}")
    assert err < 1e-12


# Split 16-bit contractions: error against the FP64 oracle, stated per
# precision (relative to max |rhs|).  The volume and lift terms are each
# larger than their sum by about the metric scale times N^2, so a relative
# rounding u of the B operand (fields, fluxes) shows up magnified in the
# result: heads alone (x1) and an operator-only split (x2) leave the operand
# rounding (BF16 u = 2^-9, FP16 u = 2^-12) in place; splitting the operand too
# (x3) leaves u^2-level terms plus FP32 accumulation.  Measured on MI355X at
# k = 2..3, N = 2..7 (worst over N, divided by max(1, N/4)): bf16 0.16,
# bf16x2 0.16, bf16x3 2.8e-4, f16 1.6e-2, f16x2 1.3e-2, f16x3 4.9e-6; at the
# full K = 82,944 mesh bf16x3 9.4e-4, f16x3 2.2e-5.  Bounds: about 3x those.
SPLIT_TOL = {"bf16": 5e-1, "bf16x2": 5e-1, "bf16x3": 1e-3, "f16": 5e-2, "f16x2": 5e-2, "f16x3": 2e-5}
SPLIT_TOL_FULL = {"bf16x3": 3e-3, "f16x3": 7e-5}


@pytest.mark.parametrize("variant", ["mfma"])
@pytest.mark.parametrize("precision", list(SPLIT_TOL))
@pytest.mark.parametrize("N", range(1, 10))
def test_split_precision_rhs(dg, N, precision, variant):
    k = 3 if N <= 5 else 2
    _say(f"[gpu] split rhs N={N} {precision} {variant}")
    VX, EToV, m, u, ref = _case(N, k)
    got = _gpu_rhs(dg, N, VX, EToV, u, precision, variant)
    err = _rel(got, ref)
    _say(f"  {precision} N={N} rel err {err:.3e}")
    assert err < SPLIT_TOL[precision] * max(1.0, N / 4)


@pytest.mark.parametrize("variant", ["mfma"])
@pytest.mark.parametrize("precision", ["bf16x3", "f16x3"])
def test_split_precision_full_size_and_steps(dg, precision, variant):
    import torch
    _say(f"[gpu] split precision full size {precision} {variant}")
    VX, EToV, m, u, ref = _case(4, 24)
    got = _gpu_rhs(dg, 4, VX, EToV, u, precision, variant)
    err = _rel(got, ref)
    _say(f"  {precision} K=82944 rel err {err:.3e}")
    assert err < SPLIT_TOL_FULL[precision]
    VX, EToV = I.kuhn_cube(3, 0.1, 0)
    mm = Me.Mesh(4, VX, EToV)
    u0 = I.cavity_mode(mm.x, mm.y, mm.z)
    dt = D.dt_cfl(mm, 0.5)
    ref = L.integrate(lambda v, t: Mx.rhs(mm, v), u0, 0.0, dt, 20)
    p = _problem(dg, 4, VX, EToV, precision, variant)
    du = p.pack(u0)
    res = p.zeros_state()
    p.rk_step(du, res, 0.0, dt, 20)
    torch.cuda.synchronize()
    err = _rel(p.unpack(du), ref)
    p.close()
    _say(f"  {precision} 20 LSERK steps rel err {err:.3e}")
    assert err < SPLIT_TOL[precision]


# ---------------------------------------------------------------------------
# Batches: many independent problems of different order and size stepped
# together.  The grouped launches (with and without graph replay) run the
# same per-tile code as one launch per problem, so the results are bitwise
# equal; one problem is also checked against the oracle.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_modes_agree_bitwise_and_match_oracle(dg, precision):
    import torch
    _say(f"[gpu] batch modes {precision}")
    specs = [(2, 3, 11), (4, 2, 12), (3, 4, 13), (4, 1, 14), (5, 2, 15), (2, 1, 16)]
    if precision == "fp64":
        specs = [s for s in specs if s[0] <= 4]
    meshes, oracle_meshes, us = [], [], []
    for N, k, seed in specs:
        VX, EToV = I.kuhn_cube(k, 0.1, seed)
        m = Me.Mesh(N, VX, EToV)
        meshes.append((N, VX, EToV))
        oracle_meshes.append(m)
        us.append(I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, seed))
    dts = [D.dt_cfl(m, 0.5) for m in oracle_meshes]
    results = {}
    for mode in ("graph", "grouped", "per_problem"):
        b = dg.Batch(meshes, precision)
        du = [p.pack(u) for p, u in zip(b.problems, us)]
        res = [p.zeros_state() for p in b.problems]
        b.rk_step(du, res, dts, 3, mode)
        b.rk_step(du, res, dts, 2, mode)     # second call: replays the captured graphs
        torch.cuda.synchronize()
        results[mode] = [p.unpack(x) for p, x in zip(b.problems, du)]
        b.close()
    for i in range(len(specs)):
        assert np.array_equal(results["graph"][i], results["per_problem"][i])
        assert np.array_equal(results["grouped"][i], results["per_problem"][i])
    m = oracle_meshes[1]
    ref = L.integrate(lambda v, t: Mx.rhs(m, v), us[1], 0.0, dts[1], 5)
    err = _rel(results["graph"][1], ref)
    _say(f"  batch problem 1 vs oracle after 5 steps: {err:.3e}")
    assert err < (1e-10 if precision == "fp64" else 1e-5)


def test_batch_of_the_64_draws_every_problem_against_the_oracle(dg):
    """The 64-problem mix (orders drawn from 2..7, so the four-wave tiles of
    the batched kernel at N = 6, 7 run) on small meshes (k = 1 or 2) so the
    oracle stays cheap: all three modes agree bitwise and every problem
    matches the oracle after two steps (FP32)."""
    import torch
    draws = I.batch_draws()
    assert {n for _, n, _ in draws} >= {6, 7}
    meshes, oms, us = [], [], []
    for p_, (k, N, seed) in enumerate(draws):
        kk = 1 + p_ % 2
        VX, EToV = I.kuhn_cube(kk, 0.1, seed)
        meshes.append((N, VX, EToV))
        m = Me.Mesh(N, VX, EToV)
        oms.append(m)
        us.append(I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, seed))
    dts = [D.dt_cfl(m, 0.5) for m in oms]
    results = {}
    for mode in ("graph", "grouped", "per_problem"):
        _say(f"[gpu] 64-draw batch {mode}")
        b = dg.Batch(meshes, "fp32")
        du = [p.pack(u) for p, u in zip(b.problems, us)]
        res = [p.zeros_state() for p in b.problems]
        b.rk_step(du, res, dts, 2, mode)
        torch.cuda.synchronize()
        results[mode] = [p.unpack(x) for p, x in zip(b.problems, du)]
        b.close()
    worst = 0.0
    for i, m in enumerate(oms):
        assert np.array_equal(results["graph"][i], results["per_problem"][i])
        assert np.array_equal(results["grouped"][i], results["per_problem"][i])
        ref = L.integrate(lambda v, t: Mx.rhs(m, v), us[i], 0.0, dts[i], 2)
        worst = max(worst, _rel(results["graph"][i], ref))
    _say(f"  worst problem vs oracle after 2 steps: {worst:.3e}")
    assert worst < 1e-5


def test_fp64_batch_past_the_cache_size(dg):
    """FP64 batch whose step touches more than the 256 MB last-level cache
    (K = 82,944 at N = 4: 3 x 139 MB), so its stages write through streaming
    stores: the three modes agree bitwise, and the small problem of the batch
    matches the oracle after two steps."""
    import torch
    _say("[gpu] fp64 batch past the cache size")
    specs = [(4, 24, 0), (3, 2, 21)]
    meshes, oms, us = [], [], []
    for N, k, seed in specs:
        VX, EToV = I.kuhn_cube(k, 0.1, seed)
        meshes.append((N, VX, EToV))
        m = Me.Mesh(N, VX, EToV)
        oms.append(m)
        us.append(I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, seed + 1))
    dts = [D.dt_cfl(m, 0.5) for m in oms]
    results = {}
    for mode in ("graph", "grouped", "per_problem"):
        b = dg.Batch(meshes, "fp64")
        du = [p.pack(u) for p, u in zip(b.problems, us)]
        res = [p.zeros_state() for p in b.problems]
        b.rk_step(du, res, dts, 2, mode)
        torch.cuda.synchronize()
        results[mode] = [p.unpack(x) for p, x in zip(b.problems, du)]
        b.close()
        del du, res
    for i in range(len(specs)):
        assert np.array_equal(results["graph"][i], results["per_problem"][i])
        assert np.array_equal(results["grouped"][i], results["per_problem"][i])
    ref = L.integrate(lambda v, t: Mx.rhs(oms[1], v), us[1], 0.0, dts[1], 2)
    err = _rel(results["graph"][1], ref)
    _say(f"  small problem vs oracle after 2 steps: {err:.3e}")
    assert err < 1e-12


def test_batch_rejects_mixed_precision_and_unsupported(dg):
    VX, EToV = I.kuhn_cube(1, 0.0, 0)
    descs = (dg.MeshDesc * 2)()
    with pytest.raises(dg.DgError):
        dg.Batch([(3, VX, EToV), (9, VX, EToV)], "fp64")   # FP64 N = 9 has no matrix-core kernel


# ---------------------------------------------------------------------------
# Large mesh: 48^3 x 6 tetrahedra (K = 663,552), N = 5, FP32 state (about
# 0.9 GB per state array) -- the oracle on every element, and two properties
# that hold at any size: the exact discrete energy identity and polynomial
# exactness.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def large_case():
    _say("[gpu] building the K=663552 N=5 oracle case")
    VX, EToV = I.kuhn_cube(48, 0.1, 0)
    m = Me.Mesh(5, VX, EToV)
    u = I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, 1)
    ref = Mx.rhs(m, u)
    diss = D.dissipation(m, u, 1.0)
    scale = float(np.sum(m.J[None, :, None] * np.abs(u) * np.abs(ref @ m.re.M.T)))
    return VX, EToV, m, u, ref, diss, scale


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("f16x3", 2e-4), ("bf16x3", 1e-2)])
def test_large_mesh_against_oracle_and_energy_identity(dg, large_case, precision, tol):
    _say(f"[gpu] large mesh K=663552 N=5 {precision}")
    VX, EToV, m, u, ref, diss, scale = large_case
    got = _gpu_rhs(dg, 5, VX, EToV, u, precision, "mfma")
    err = _rel(got, ref)
    _say(f"  {precision} rel err vs oracle {err:.3e}")
    assert err < tol
    # energy identity with the GPU right-hand side: sum_k J_k u^T M rhs
    Mr = got @ m.re.M.T
    rate = float(np.sum(m.J[None, :, None] * u * Mr))
    _say(f"  energy rate {rate:.6e} vs dissipation {diss:.6e} (scale {scale:.3e})")
    assert abs(rate - diss) < 10 * tol * scale


def test_large_mesh_polynomial_exactness(dg, large_case):
    _say("[gpu] large mesh polynomial exactness fp32")
    VX, EToV, m = large_case[:3]
    x, y = m.x, m.y
    u = np.zeros((6, m.K, m.Np))
    u[2] = x * (1 - x) * y * (1 - y)
    got = _gpu_rhs(dg, 5, VX, EToV, u, "fp32", "mfma")
    ex = np.zeros_like(u)
    ex[3] = -x * (1 - x) * (1 - 2 * y)
    ex[4] = (1 - 2 * x) * y * (1 - y)
    err = float(np.abs(got - ex).max())
    _say(f"  max abs err {err:.3e}")
    assert err < 1e-4


# ---------------------------------------------------------------------------
# End to end on the GPU: time integration of the cavity mode against its
# closed form (h-convergence at the rate the method gives, N + 1 in theory,
# N + 1/2 guaranteed), and the discrete energy never increasing under the
# upwind flux.  The errors and energies are measured by the oracle's mass
# norm on the unpacked GPU states.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N,precision,ks,cfl,expect", [
    (2, "fp64", (2, 4, 8), 0.5, 2.5),
    (3, "fp64", (2, 4, 8), 0.5, 3.5),
    (4, "fp64", (2, 4), 0.125, 4.5),
    (3, "fp32", (2, 4), 0.5, 3.3),
    (3, "f16x3", (2, 4), 0.5, 3.3),
])
def test_gpu_cavity_h_convergence(dg, N, precision, ks, cfl, expect):
    import torch
    T = 0.25
    errs = []
    for k in ks:
        _say(f"[gpu] cavity convergence N={N} k={k} {precision}")
        VX, EToV = I.kuhn_cube(k, 0.1, k)
        m = Me.Mesh(N, VX, EToV)
        u0 = I.cavity_mode(m.x, m.y, m.z, 0.0)
        ns = int(np.ceil(T / D.dt_cfl(m, cfl)))
        p = dg.Problem(N, VX, EToV, precision)
        du = p.pack(u0)
        res = p.zeros_state()
        p.rk_step(du, res, 0.0, T / ns, ns)
        torch.cuda.synchronize()
        u = p.unpack(du)
        p.close()
        ex = I.cavity_mode(m.x, m.y, m.z, T)
        errs.append(D.mass_norm(m, u - ex) / D.mass_norm(m, u0))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    _say(f"  errors {['%.3e' % e for e in errs]} rates {['%.2f' % r for r in rates]}")
    assert rates[-1] > expect


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gpu_energy_non_increasing(dg, precision):
    import torch
    _say(f"[gpu] energy over 100 LSERK steps {precision}")
    VX, EToV = I.kuhn_cube(4, 0.1, 0)
    m = Me.Mesh(3, VX, EToV)
    u0 = I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, 1)
    dt = D.dt_cfl(m, 0.5)
    p = dg.Problem(3, VX, EToV, precision)
    du = p.pack(u0)
    res = p.zeros_state()
    energies = [D.energy(m, p.unpack(du))]
    for _ in range(10):
        p.rk_step(du, res, 0.0, dt, 10)
        torch.cuda.synchronize()
        energies.append(D.energy(m, p.unpack(du)))
    p.close()
    tol = 1e-13 if precision == "fp64" else 1e-6
    assert np.all(np.diff(energies) <= tol * energies[0])
    assert energies[-1] < energies[0]


# ---------------------------------------------------------------------------
# The large-mesh workload's time stepping on subsampled meshes of the same
# recipe (N = 5, k = 6, 12, 24; the full mesh is k = 48): FP64 on the GPU
# against the oracle's integration at k = 6 and against the cavity's closed
# form (h-convergence); FP32 and the x3 split precisions over 200 LSERK steps
# with the discrete energy checked every 10 steps and the state compared with
# the FP64 run of the same steps.
# ---------------------------------------------------------------------------
C5_KS = (6, 12, 24)
C5_STEPS = 200


@pytest.fixture(scope="module")
def c5_fp64(dg):
    """FP64 GPU states after C5_STEPS steps at CFL 0.5 per k, and the closed-form
    errors at a common final time (the 200 steps of k = 24)."""
    import torch
    out = {}
    T = None
    for k in sorted(C5_KS, reverse=True):
        _say(f"[gpu] subsampled large-mesh workload fp64 k={k}")
        VX, EToV = I.kuhn_cube(k, 0.1, 0)
        m = Me.Mesh(5, VX, EToV)
        u0 = I.cavity_mode(m.x, m.y, m.z)
        dt = D.dt_cfl(m, 0.5)
        if T is None:
            T = C5_STEPS * dt
        p = dg.Problem(5, VX, EToV, "fp64")
        du = p.pack(u0)
        res = p.zeros_state()
        p.rk_step(du, res, 0.0, dt, C5_STEPS)
        torch.cuda.synchronize()
        u_steps = p.unpack(du)
        ns = int(np.ceil(T / dt))
        du = p.pack(u0)
        p.rk_step(du, res, 0.0, T / ns, ns)
        torch.cuda.synchronize()
        uT = p.unpack(du)
        p.close()
        err = D.mass_norm(m, uT - I.cavity_mode(m.x, m.y, m.z, T)) / D.mass_norm(m, u0)
        out[k] = dict(mesh=(VX, EToV), m=m, u0=u0, dt=dt, u_steps=u_steps, err_T=err, T=T)
    return out


def test_subsampled_large_workload_fp64_against_oracle_and_closed_form(c5_fp64):
    c = c5_fp64[6]
    m = c["m"]
    _say("[gpu] fp64 k=6 N=5 200 steps vs the oracle's integration")
    ref = L.integrate(lambda v, t: Mx.rhs(m, v), c["u0"], 0.0, c["dt"], C5_STEPS)
    err = _rel(c["u_steps"], ref)
    _say(f"  rel err after {C5_STEPS} steps {err:.3e}")
    assert err < 1e-10
    errs = [c5_fp64[k]["err_T"] for k in C5_KS]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    _say(f"  closed-form errors at T={c['T']:.4f}: {['%.3e' % e for e in errs]} rates {['%.2f' % r for r in rates]}")
    assert np.all(rates > 5.5)        # N + 1/2 guaranteed, N + 1 = 6 expected


# Worst relative deviation from the FP64 state after 200 steps (bound), and
# the relative energy rise allowed per 10-step interval: the upwind scheme
# dissipates (the FP64 energy never rises), so a rise can only come from
# rounding, of the order of T x (relative RHS error) x |rhs| / |u|, with
# T = 10 dt = 2.6e-3 at k = 24, |rhs| / |u| about omega = 4.4 and RHS errors
# of about 1e-6 (FP32), 2e-5 (f16x3) and 1e-3 (bf16x3); the bounds are 10x
# those.
C5_DEV = {"fp32": 1e-5, "f16x3": 2e-4, "bf16x3": 3e-3}
C5_ETOL = {"fp32": 1e-6, "f16x3": 1e-5, "bf16x3": 1e-3}


@pytest.mark.parametrize("precision", ["fp32", "f16x3", "bf16x3"])
def test_subsampled_large_workload_200_steps(dg, c5_fp64, precision):
    import torch
    for k in C5_KS:
        c = c5_fp64[k]
        VX, EToV = c["mesh"]
        m = c["m"]
        _say(f"[gpu] subsampled large-mesh workload {precision} k={k} {C5_STEPS} steps")
        p = dg.Problem(5, VX, EToV, precision)
        du = p.pack(c["u0"])
        res = p.zeros_state()
        energies = [D.energy(m, p.unpack(du))]
        for _ in range(C5_STEPS // 10):
            p.rk_step(du, res, 0.0, c["dt"], 10)
            torch.cuda.synchronize()
            energies.append(D.energy(m, p.unpack(du)))
        u = p.unpack(du)
        p.close()
        dev = _rel(u, c["u_steps"])
        rise = float(np.max(np.diff(energies)) / energies[0])
        _say(f"  deviation from fp64 {dev:.3e}, largest energy rise per 10 steps {rise:.3e}")
        assert dev < C5_DEV[precision]
        assert rise <= C5_ETOL[precision]
        assert energies[-1] <= energies[0] * (1 + C5_ETOL[precision])
