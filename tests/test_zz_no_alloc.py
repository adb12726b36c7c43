"""dg_rk_step_noalloc (the stepping entry point that allocates nothing)
against dg_rk_step, through the C ABI.

Same kernels, same arithmetic: the result must equal dg_rk_step's bit for
bit, on two calls in a row (the second on a smaller problem, so the static
scratch holds the first call's leftovers), for the fused matrix-core stages
(an odd stage count exercises the final copy out of the scratch) and the
unfused vector-ALU path.  Problems whose state exceeds the static scratch are
refused before any launch.
"""
import ctypes as C

import numpy as np
import pytest

import dg_inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    assert torch.cuda.is_available()
    from paper_1211_0582_amd import dg as mod
    return mod


def _steps(dg, N, k, precision, variant, nsteps, noalloc):
    import torch
    VX, EToV = I.kuhn_cube(k, 0.1, 3)
    p = dg.Problem(N, VX, EToV, precision)
    p.set_variant(variant)
    xyz = p.nodes()
    u0 = I.cavity_mode(xyz[..., 0], xyz[..., 1], xyz[..., 2]) + I.field_noise((6, p.info.K, p.info.Np), 1e-3, 7)
    du = p.pack(u0)
    res = p.zeros_state()
    dt = 0.5 * p.info.dt_cfl1
    fn = dg.lib.dg_rk_step_noalloc if noalloc else dg.lib.dg_rk_step
    st = fn(p.handle, du.data_ptr(), res.data_ptr(), C.c_double(0.0), C.c_double(dt), nsteps,
            torch.cuda.current_stream().cuda_stream)
    dg._check(st)
    torch.cuda.synchronize()
    out = p.unpack(du)
    p.close()
    return out


@pytest.mark.parametrize("precision,variant", [("fp64", "mfma"), ("fp32", "mfma"), ("fp64", "valu"),
                                               ("f16x3", "mfma")])
def test_noalloc_matches_rk_step_on_two_calls(dg, precision, variant):
    for N, k, nsteps in ((4, 4, 3), (3, 2, 2)):     # second call: smaller problem
        print(f"[gpu] noalloc vs rk_step N={N} k={k} {precision} {variant} steps={nsteps}", flush=True)
        ref = _steps(dg, N, k, precision, variant, nsteps, False)
        got = _steps(dg, N, k, precision, variant, nsteps, True)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref)


def test_noalloc_refuses_states_beyond_the_static_scratch(dg):
    import torch
    VX, EToV = I.kuhn_cube(40, 0.0, 0)            # K = 384,000, N = 3: 369 MB per FP64 state array
    p = dg.Problem(3, VX, EToV, "fp64")
    assert p.info.state_elems * p.info.elem_bytes > (256 << 20)
    u, res = p.zeros_state(), p.zeros_state()
    st = dg.lib.dg_rk_step_noalloc(p.handle, u.data_ptr(), res.data_ptr(), C.c_double(0.0), C.c_double(1e-4), 1,
                                   torch.cuda.current_stream().cuda_stream)
    assert st == dg.DG_EUNSUPPORTED
    assert "static scratch" in dg.lib.dg_last_error().decode()
    p.close()


def test_noalloc_leaves_device_memory_unchanged(dg):
    import torch
    VX, EToV = I.kuhn_cube(3, 0.1, 1)
    p = dg.Problem(4, VX, EToV, "fp32")
    u, res = p.zeros_state(), p.zeros_state()
    s = torch.cuda.current_stream().cuda_stream
    dg._check(dg.lib.dg_rk_step_noalloc(p.handle, u.data_ptr(), res.data_ptr(), C.c_double(0.0), C.c_double(1e-3),
                                        2, s))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        dg._check(dg.lib.dg_rk_step_noalloc(p.handle, u.data_ptr(), res.data_ptr(), C.c_double(0.0),
                                            C.c_double(1e-3), 3, s))
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    p.close()
