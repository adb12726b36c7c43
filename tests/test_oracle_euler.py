"""Pins of the nonlinear Euler oracle (oracle/euler.py), CPU only.

  * exact steady states: a uniform flow with transmissive boundaries and a
    resting density perturbation at uniform pressure inside slip walls give
    rhs = 0 to roundoff;
  * discrete conservation: every conserved quantity changes exactly by the
    boundary fluxes (interior numerical fluxes cancel), computed from traces;
    inside slip walls mass and energy are conserved;
  * linearisation about a resting state equals the (separately pinned) linear
    oracle with the Euler flux Jacobians and the Rusanov penalty at the sound
    speed (central differences in the state: second-order accurate except for
    the |n.m| / rho term of the penalty speed, which is first order in the
    step, so the step is small).
"""
import numpy as np
import pytest

import dg_inputs as I
from oracle import euler as Eu
from oracle import linear as Li
from oracle import mesh as Me


def _state(rho, vel, p, shape):
    u = np.zeros((5,) + shape)
    u[0] = rho
    for d in range(3):
        u[1 + d] = rho * vel[d]
    u[4] = p / (Eu.GAMMA - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    return u


def _smooth_state(m, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, 6)
    rho = 1.0 + 0.2 * np.sin(a[0] * m.x + a[1] * m.y) * np.cos(a[2] * m.z)
    vel = [0.2 * np.cos(a[3] * m.y), -0.1 * np.sin(a[4] * m.z), 0.15 * np.cos(a[5] * m.x)]
    p = 1.0 + 0.1 * np.cos(m.x + m.y + m.z)
    return _state(rho, vel, p, m.x.shape)


def test_uniform_flow_is_steady():
    VX, EToV = I.kuhn_cube(2, 0.1, 1)
    m = Me.Mesh(3, VX, EToV, face_bc=np.ones((EToV.shape[0], 4), dtype=np.int8))
    u = _state(1.2, (0.3, -0.2, 0.1), 0.8, m.x.shape)
    assert np.abs(Eu.rhs(m, u)).max() < 1e-13


def test_resting_density_perturbation_is_steady_inside_walls():
    VX, EToV = I.kuhn_cube(2, 0.1, 2)
    m = Me.Mesh(4, VX, EToV)
    rho = 1.0 + 0.2 * np.cos(np.pi * m.x) * np.cos(np.pi * m.y) * np.cos(np.pi * m.z)
    u = _state(rho, (0.0, 0.0, 0.0), 1.0, m.x.shape)
    assert np.abs(Eu.rhs(m, u)).max() < 1e-13


@pytest.mark.parametrize("codes", [(0, 1, 2), (0,)])
def test_conservation_through_boundary_fluxes_only(codes):
    VX, EToV = I.kuhn_cube(2, 0.1, 3)
    bc = I.random_face_bc(EToV.shape[0], 4, codes=codes)
    m = Me.Mesh(3, VX, EToV, face_bc=bc)
    u = _smooth_state(m, 5)
    r = Eu.rhs(m, u)
    a = Eu.total_rate(m, r)
    b = Eu.boundary_flux_rate(m, u)
    scale = np.abs(Eu.total_rate(m, np.abs(r))).max()
    assert np.abs(a - b).max() < 1e-12 * scale
    if codes == (0,):
        assert abs(a[0]) < 1e-12 * scale and abs(a[4]) < 1e-12 * scale


def test_linearisation_about_rest_is_the_linear_oracle():
    VX, EToV = I.kuhn_cube(2, 0.1, 6)
    bc = I.random_face_bc(EToV.shape[0], 7, codes=(0, 1))
    m = Me.Mesh(3, VX, EToV, face_bc=bc)
    rho0, p0 = 1.0, 1.0 / Eu.GAMMA                       # sound speed 1
    u0 = _state(rho0, (0.0, 0.0, 0.0), p0, m.x.shape)
    d = I.field_noise((5, m.K, m.Np), 1.0, 8)
    eps = 1e-7
    lin = (Eu.rhs(m, u0 + eps * d) - Eu.rhs(m, u0 - eps * d)) / (2 * eps)

    def wall(n):
        B = np.zeros(n.shape[:-1] + (5, 5))
        B[..., 0, 0] = B[..., 4, 4] = 1.0
        B[..., 1:4, 1:4] = np.eye(3) - 2.0 * n[..., :, None] * n[..., None, :]
        return B

    ident = lambda n: np.broadcast_to(np.eye(5), n.shape[:-1] + (5, 5))  # noqa: E731
    sys = Li.LinearSystem(("rho", "mx", "my", "mz", "E"), Eu.jacobians_at_rest(rho0, p0),
                          {0: wall, 1: ident, 2: ident}, speed=1.0)
    ref = Li.rhs(m, sys, d, 1.0)
    assert np.abs(lin - ref).max() < 1e-6 * np.abs(ref).max()
    ref0 = Li.rhs(m, sys, d, 0.0)                        # central flux: no penalty, second order
    lin0 = (Eu.rhs(m, u0 + 1e-5 * d, alpha=0.0) - Eu.rhs(m, u0 - 1e-5 * d, alpha=0.0)) / 2e-5
    assert np.abs(lin0 - ref0).max() < 1e-8 * np.abs(ref0).max()
