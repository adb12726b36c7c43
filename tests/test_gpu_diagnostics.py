"""On-device diagnostics (dg_energy) against the oracle's energy and mass norm.

The device computes 1/2 sum_k J_k (eps E^T M E + mu H^T M H) of u - ref in
binary64; the oracle computes the same quadratic form with NumPy on the
unpacked state (the exact values the device holds), so they agree to the
rounding of two binary64 summation orders.
"""
import sys

import numpy as np
import pytest

import dg_inputs as I
from oracle import diag as D
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


@pytest.mark.parametrize("precision", ["fp64", "fp32", "f16x3"])
@pytest.mark.parametrize("N,k", [(1, 3), (4, 3), (9, 1)])
def test_energy_and_error_norm_match_oracle(dg, N, k, precision):
    _say(f"[gpu] energy N={N} k={k} {precision}")
    VX, EToV = I.kuhn_cube(k, 0.1, 2)
    m = Me.Mesh(N, VX, EToV)
    u = I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-2, 3)
    ex = I.cavity_mode(m.x, m.y, m.z, 0.1)
    p = dg.Problem(N, VX, EToV, precision)
    du, dex = p.pack(u), p.pack(ex)
    uh, exh = p.unpack(du), p.unpack(dex)       # the values the device holds
    e_dev = float(p.energy(du).item())
    e_ref = D.energy(m, uh)
    assert abs(e_dev - e_ref) <= 1e-13 * e_ref
    err_dev = p.error_norm(du, dex)
    err_ref = D.mass_norm(m, uh - exh)
    assert abs(err_dev - err_ref) <= 1e-12 * err_ref
    a, b = p.energy(du), p.energy(du)
    assert a.item() == b.item()                   # fixed summation order
    p.close()


def test_energy_with_materials(dg):
    VX, EToV = I.kuhn_cube(2, 0.1, 4)
    K = EToV.shape[0]
    rng = np.random.default_rng(5)
    eps, mu = rng.uniform(1, 3, K), rng.uniform(0.5, 2, K)
    m = Me.Mesh(3, VX, EToV, eps=eps, mu=mu)
    u = I.field_noise((6, m.K, m.Np), 1.0, 6)
    p = dg.Problem(3, VX, EToV, "fp64", eps=eps, mu=mu)
    du = p.pack(u)
    assert abs(float(p.energy(du).item()) - D.energy(m, u)) <= 1e-13 * D.energy(m, u)
    p.close()


def test_self_checking_run_energy_never_increases(dg):
    """A long run checked on the device only: the energy after every 10 steps,
    read once at the end, never increases (upwind flux, FP64)."""
    import torch
    VX, EToV = I.kuhn_cube(4, 0.1, 0)
    N = 3
    p = dg.Problem(N, VX, EToV, "fp64")
    xyz = p.nodes()
    u0 = I.cavity_mode(xyz[..., 0], xyz[..., 1], xyz[..., 2]) + I.field_noise((6, p.info.K, p.info.Np), 1e-3, 1)
    du = p.pack(u0)
    res = p.zeros_state()
    energies = torch.zeros(11, dtype=torch.float64, device="cuda")
    dt = 0.5 * p.info.dt_cfl1
    p.energy(du, out=energies[0:1])
    for i in range(10):
        p.rk_step(du, res, 0.0, dt, 10)
        p.energy(du, out=energies[i + 1:i + 2])
    e = energies.cpu().numpy()
    _say(f"  energies {e[0]:.12e} -> {e[-1]:.12e}")
    assert np.all(np.diff(e) <= 1e-14 * e[0])
    assert e[-1] < e[0]
    m = Me.Mesh(N, VX, EToV)
    assert abs(e[-1] - D.energy(m, p.unpack(du))) <= 1e-13 * e[0]
    p.close()
