"""GPU parity of run-time compiled systems (hipRTC) against the oracles.

Each system is written in the flux front end (paper_1211_0582_amd/systems.py),
compiled by the library at setup and run through the C ABI like the built-in
kernels.  References: the Maxwell oracle for the generated Maxwell system (so
the generated kernel also matches the hand-written one), the general
linear-hyperbolic oracle for acoustics and advection.  Tolerances: FP64 1e-12
and FP32 5e-5 relative to max |rhs|, as for the built-in kernels.
"""
import sys

import numpy as np
import pytest

import dg_inputs as I
from oracle import diag as D
from oracle import linear as Li
from oracle import lserk as L
from oracle import maxwell as Mx
from oracle import mesh as Me

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 5e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_1211_0582_amd import systems
    return systems


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _run(S, spec, N, VX, EToV, u, precision, alpha=1.0, face_bc=None):
    import torch
    p = S.SystemProblem(spec, N, VX, EToV, precision, alpha, face_bc)
    du = p.pack(u)
    out = p.zeros_state()
    p.rhs(du, out)
    torch.cuda.synchronize()
    r = p.unpack(out)
    p.close()
    return r


def _advection_oracle(beta):
    A = np.zeros((3, 1, 1))
    A[:, 0, 0] = beta
    zero = lambda n: np.zeros(n.shape[:-1] + (1, 1))  # noqa: E731
    return Li.LinearSystem(("u",), A, {0: zero, 1: zero, 2: zero})


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [1, 3, 5])
def test_generated_maxwell_matches_the_maxwell_oracle(S, N, precision):
    _say(f"[gpu] generated maxwell N={N} {precision}")
    VX, EToV = I.kuhn_cube(2, 0.1, 3)
    bc = I.random_face_bc(EToV.shape[0], 4)
    m = Me.Mesh(N, VX, EToV, face_bc=bc)
    u = I.field_noise((6, m.K, m.Np), 1.0, 5)
    ref = Mx.rhs(m, u, 0.8)
    got = _run(S, S.maxwell(), N, VX, EToV, u, precision, 0.8, bc)
    err = _rel(got, ref)
    _say(f"  rel err {err:.3e}")
    assert err < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [2, 4, 6])
def test_acoustics_matches_the_linear_oracle(S, N, precision):
    _say(f"[gpu] acoustics N={N} {precision}")
    VX, EToV = I.kuhn_cube(3, 0.1, 6)
    bc = I.random_face_bc(EToV.shape[0], 7)
    m = Me.Mesh(N, VX, EToV, face_bc=bc)
    u = I.field_noise((4, m.K, m.Np), 1.0, 8)
    ref = Li.rhs(m, Li.acoustics_system(), u, 1.0)
    got = _run(S, S.acoustics(), N, VX, EToV, u, precision, 1.0, bc)
    err = _rel(got, ref)
    _say(f"  rel err {err:.3e}")
    assert err < TOL[precision]


@pytest.mark.parametrize("N", [1, 3])
def test_advection_matches_the_linear_oracle(S, N):
    beta = (1.0, -0.5, 0.25)
    VX, EToV = I.kuhn_cube(3, 0.1, 9)
    m = Me.Mesh(N, VX, EToV)
    u = I.field_noise((1, m.K, m.Np), 1.0, 10)
    for alpha in (0.0, 1.0):
        ref = Li.rhs(m, _advection_oracle(beta), u, alpha)
        got = _run(S, S.advection(beta), N, VX, EToV, u, "fp64", alpha)
        assert _rel(got, ref) < 1e-12


def test_acoustic_cavity_on_the_gpu_converges_and_keeps_energy(S):
    """LSERK on the GPU (compiled right-hand side + update kernel) against the
    closed-form acoustic cavity mode; the device energy never increases."""
    import torch
    N, T = 3, 0.25
    errs = []
    for k in (2, 4):
        VX, EToV = I.kuhn_cube(k, 0.1, k)
        m = Me.Mesh(N, VX, EToV)
        u0 = Li.acoustic_cavity_mode(m.x, m.y, m.z, 0.0)
        ns = int(np.ceil(T / D.dt_cfl(m, 0.5)))
        p = S.SystemProblem(S.acoustics(), N, VX, EToV, "fp64")
        du = p.pack(u0)
        res = p.zeros_state()
        e = torch.zeros(ns + 1, dtype=torch.float64, device="cuda")
        p.energy(du, out=e[0:1])
        for i in range(ns):
            p.rk_step(du, res, 0.0, T / ns, 1)
            p.energy(du, out=e[i + 1:i + 2])
        u = p.unpack(du)
        ev = e.cpu().numpy()
        assert np.all(np.diff(ev) <= 1e-14 * ev[0])
        assert abs(ev[-1] - Li.energy(m, u)) <= 1e-12 * ev[0]
        p.close()
        ex = Li.acoustic_cavity_mode(m.x, m.y, m.z, T)
        errs.append(np.sqrt(2 * Li.energy(m, u - ex)) / np.sqrt(2 * Li.energy(m, u0)))
    rate = float(np.log2(errs[0] / errs[1]))
    _say(f"  acoustic cavity errors {errs} rate {rate:.2f}")
    assert rate > N + 0.5


def test_acoustics_steps_match_the_oracle_integration(S):
    import torch
    N = 4
    VX, EToV = I.kuhn_cube(2, 0.1, 11)
    bc = I.random_face_bc(EToV.shape[0], 12)
    m = Me.Mesh(N, VX, EToV, face_bc=bc)
    s = Li.acoustics_system()
    u0 = I.field_noise((4, m.K, m.Np), 1.0, 13)
    dt = D.dt_cfl(m, 0.5)
    ref = L.integrate(lambda v, t: Li.rhs(m, s, v), u0, 0.0, dt, 7)
    p = S.SystemProblem(S.acoustics(), N, VX, EToV, "fp64", face_bc=bc)
    du = p.pack(u0)
    res = p.empty_state()
    res.fill_(float("nan"))           # the first stage does not read res
    p.rk_step(du, res, 0.0, dt, 7)
    torch.cuda.synchronize()
    assert _rel(p.unpack(du), ref) < 1e-11
    p.close()


def test_system_problem_contract(S):
    from paper_1211_0582_amd import dg
    VX, EToV = I.kuhn_cube(1, 0.0, 0)
    p = S.SystemProblem(S.acoustics(), 2, VX, EToV, "fp32")
    assert p.info.nfields == 4 and p.info.state_elems == 4 * p.info.field_stride
    with pytest.raises(dg.DgError) as e:
        p.set_variant("mfma")
    assert e.value.status == dg.DG_EUNSUPPORTED
    p.close()
    with pytest.raises(dg.DgError) as e:
        dg.dg_setup_system(2, VX, EToV, "struct System {};", 4)
    assert e.value.status == dg.DG_EINVAL


# ---------------------------------------------------------------------------
# A nonlinear system through the same front end: compressible Euler with the
# local Lax-Friedrichs flux, against the nonlinear oracle.
# ---------------------------------------------------------------------------
def _euler_state(m, seed):
    from oracle import euler as Eu
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, 6)
    rho = 1.0 + 0.2 * np.sin(a[0] * m.x + a[1] * m.y) * np.cos(a[2] * m.z)
    vel = [0.2 * np.cos(a[3] * m.y), -0.1 * np.sin(a[4] * m.z), 0.15 * np.cos(a[5] * m.x)]
    p = 1.0 + 0.1 * np.cos(m.x + m.y + m.z)
    u = np.zeros((5,) + m.x.shape)
    u[0] = rho
    for d in range(3):
        u[1 + d] = rho * vel[d]
    u[4] = p / (Eu.GAMMA - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    return u


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 5e-5)])
@pytest.mark.parametrize("N", [2, 4])
def test_euler_matches_the_nonlinear_oracle(S, N, precision, tol):
    from oracle import euler as Eu
    _say(f"[gpu] euler N={N} {precision}")
    VX, EToV = I.kuhn_cube(2, 0.1, 21)
    bc = I.random_face_bc(EToV.shape[0], 22)
    m = Me.Mesh(N, VX, EToV, face_bc=bc)
    u = _euler_state(m, 23)
    ref = Eu.rhs(m, u)
    got = _run(S, S.euler(), N, VX, EToV, u, precision, 1.0, bc)
    err = _rel(got, ref)
    _say(f"  rel err {err:.3e}")
    assert err < tol


def test_euler_steps_match_the_oracle_integration(S):
    import torch
    from oracle import euler as Eu
    N = 3
    VX, EToV = I.kuhn_cube(2, 0.1, 24)
    m = Me.Mesh(N, VX, EToV)                     # slip walls everywhere
    u0 = _euler_state(m, 25)
    dt = 0.25 * D.dt_cfl(m, 0.5)
    ref = L.integrate(lambda v, t: Eu.rhs(m, v), u0, 0.0, dt, 6)
    p = S.SystemProblem(S.euler(), N, VX, EToV, "fp64")
    du = p.pack(u0)
    res = p.zeros_state()
    p.rk_step(du, res, 0.0, dt, 6)
    torch.cuda.synchronize()
    got = p.unpack(du)
    p.close()
    assert _rel(got, ref) < 1e-11
    # inside slip walls mass and energy totals stay constant
    w = m.J[:, None] * np.sum(m.re.M, axis=0)[None, :]
    for q in (0, 4):
        assert abs(np.sum(w * got[q]) - np.sum(w * u0[q])) < 1e-12 * np.sum(w * np.abs(u0[q]))
