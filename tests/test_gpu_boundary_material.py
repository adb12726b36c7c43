"""GPU parity for the boundary-condition codes and per-element materials.

The HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs: per-face condition codes (conducting, magnetic-conducting,
absorbing) drawn at random on every boundary face, and per-element
permittivity and permeability drawn at random (the material form of the
flux, with impedance weights).  Tolerances as for the vacuum operator:
FP64 1e-12, FP32 5e-5 relative to max |rhs|.
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


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _materials(K, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(1.0, 4.0, K), rng.uniform(0.5, 2.0, K)


def _run_rhs(dg, N, VX, EToV, u, precision, variant, **kw):
    import torch
    p = dg.Problem(N, VX, EToV, precision, **kw)
    try:
        p.set_variant(variant)
    except dg.DgError as e:
        p.close()
        if e.status == dg.DG_EUNSUPPORTED:
            pytest.skip(f"{variant} not built for N={N} {precision}")
        raise
    du = p.pack(u)
    out = p.zeros_state()
    p.rhs(du, out)
    torch.cuda.synchronize()
    r = p.unpack(out)
    p.close()
    return r


@pytest.mark.parametrize("variant", ["valu", "mfma"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [1, 3, 4, 6])
def test_boundary_codes_rhs(dg, N, precision, variant):
    _say(f"[gpu] boundary codes N={N} {precision} {variant}")
    VX, EToV = I.kuhn_cube(3, 0.1, 5)
    bc = I.random_face_bc(EToV.shape[0], 17)
    m = Me.Mesh(N, VX, EToV, face_bc=bc)
    u = I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-1, 2)
    ref = Mx.rhs(m, u)
    got = _run_rhs(dg, N, VX, EToV, u, precision, variant, face_bc=bc)
    err = _rel(got, ref)
    _say(f"  rel err {err:.3e}")
    assert err < TOL[precision]


@pytest.mark.parametrize("variant", ["valu", "mfma"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [2, 4, 5])
def test_materials_rhs(dg, N, precision, variant):
    _say(f"[gpu] materials N={N} {precision} {variant}")
    VX, EToV = I.kuhn_cube(3, 0.1, 6)
    K = EToV.shape[0]
    eps, mu = _materials(K, 8)
    bc = I.random_face_bc(K, 9)
    m = Me.Mesh(N, VX, EToV, face_bc=bc, eps=eps, mu=mu)
    u = I.field_noise((6, m.K, m.Np), 1.0, 4)
    ref = Mx.rhs(m, u, 0.7)
    got = _run_rhs(dg, N, VX, EToV, u, precision, variant, alpha=0.7, face_bc=bc, eps=eps, mu=mu)
    err = _rel(got, ref)
    _say(f"  rel err {err:.3e}")
    assert err < TOL[precision]


def test_unit_materials_take_the_vacuum_kernels_bitwise(dg):
    """eps = mu = 1 given explicitly selects the vacuum kernels, and the material
    kernels with all-one materials give the same bits (their record reproduces
    the vacuum flux exactly)."""
    import torch
    N = 4
    VX, EToV = I.kuhn_cube(2, 0.1, 1)
    K = EToV.shape[0]
    m = Me.Mesh(N, VX, EToV)
    u = I.field_noise((6, m.K, m.Np), 1.0, 5)
    a = _run_rhs(dg, N, VX, EToV, u, "fp64", "mfma")
    b = _run_rhs(dg, N, VX, EToV, u, "fp64", "mfma", eps=np.ones(K), mu=np.ones(K))
    assert np.array_equal(a, b)
    eps = np.ones(K)
    eps[0] = 1.0 + 2.0 ** -40           # forces the material form; differs at roundoff only
    c = _run_rhs(dg, N, VX, EToV, u, "fp64", "mfma", eps=eps)
    assert _rel(c, a) < 1e-11
    torch.cuda.synchronize()


@pytest.mark.parametrize("variant", ["valu", "mfma"])
def test_materials_and_codes_lserk_steps(dg, variant):
    """20 LSERK steps with materials and mixed boundary codes against the
    oracle's integration, FP64; the oracle's energy (material-weighted)
    does not increase."""
    import torch
    _say(f"[gpu] materials + codes 20 steps {variant}")
    N = 3
    VX, EToV = I.kuhn_cube(3, 0.1, 7)
    K = EToV.shape[0]
    eps, mu = _materials(K, 10)
    bc = I.random_face_bc(K, 12)
    m = Me.Mesh(N, VX, EToV, face_bc=bc, eps=eps, mu=mu)
    u0 = I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-2, 3)
    dt = 0.5 * D.dt_cfl(m, 0.5)
    ref = L.integrate(lambda v, t: Mx.rhs(m, v), u0, 0.0, dt, 20)
    p = dg.Problem(N, VX, EToV, "fp64", face_bc=bc, eps=eps, mu=mu)
    p.set_variant(variant)
    assert p.info.dt_cfl1 > 0
    du = p.pack(u0)
    res = p.zeros_state()
    p.rk_step(du, res, 0.0, dt, 20)
    torch.cuda.synchronize()
    got = p.unpack(du)
    p.close()
    err = _rel(got, ref)
    _say(f"  rel err after 20 steps {err:.3e}")
    assert err < 1e-11
    assert D.energy(m, got) <= D.energy(m, u0)


def test_batch_refuses_materials(dg):
    import ctypes as C
    VX, EToV = I.kuhn_cube(1, 0.0, 0)
    descs = (dg.MeshDesc * 1)()
    descs[0], keep = dg.mesh_desc(2, VX, EToV, "fp32", 1.0, None, 2.0, None)
    h = C.c_void_p()
    assert dg.lib.dg_setup_batch(1, descs, C.byref(h)) == dg.DG_EUNSUPPORTED
    del keep


def test_batch_with_boundary_codes_matches_oracle(dg):
    import torch
    specs = [(3, 2, 31), (5, 1, 32), (2, 2, 33)]
    meshes, oms, us = [], [], []
    for N, k, seed in specs:
        VX, EToV = I.kuhn_cube(k, 0.1, seed)
        bc = I.random_face_bc(EToV.shape[0], seed)
        meshes.append((N, VX, EToV, bc))
        m = Me.Mesh(N, VX, EToV, face_bc=bc)
        oms.append(m)
        us.append(I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-2, seed))
    dts = [D.dt_cfl(m, 0.5) for m in oms]
    b = dg.Batch(meshes, "fp64")
    du = [p.pack(u) for p, u in zip(b.problems, us)]
    res = [p.zeros_state() for p in b.problems]
    b.rk_step(du, res, dts, 2, "graph")
    torch.cuda.synchronize()
    for i, (p, m) in enumerate(zip(b.problems, oms)):
        ref = L.integrate(lambda v, t: Mx.rhs(m, v), us[i], 0.0, dts[i], 2)
        err = _rel(p.unpack(du[i]), ref)
        _say(f"  batch problem {i} with codes: {err:.3e}")
        assert err < 1e-12
    b.close()
