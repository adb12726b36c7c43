"""Pins for the oracle's LSERK scheme and end-to-end time integration (CPU only)."""
import numpy as np
import pytest
from scipy.linalg import expm

import dg_inputs as I
from oracle import diag as D
from oracle import lserk as L
from oracle import maxwell as Mx
from oracle import mesh as Me


def test_order_conditions():
    a, b, c = L.butcher()
    assert np.allclose(c, L.C, atol=1e-15)
    conds = [b.sum() - 1, b @ c - 1 / 2, b @ c ** 2 - 1 / 3, b @ (a @ c) - 1 / 6,
             b @ c ** 3 - 1 / 4, b @ (c * (a @ c)) - 1 / 8, b @ (a @ c ** 2) - 1 / 12,
             b @ (a @ (a @ c)) - 1 / 24]
    assert np.abs(conds).max() < 1e-15
    # not fifth order: the z^5 coefficient is 1/200, not 1/120
    assert abs(b @ (a @ (a @ (a @ c))) - 1 / 200) < 1e-15


def test_stability_polynomial():
    zs = np.array([0.3, -0.7, 1.1, -2.0, 0.5 + 1.5j, -1.0 + 2.5j])
    coef = np.array([1, 1, 1 / 2, 1 / 6, 1 / 24, 1 / 200])
    for z in zs:
        u = np.array([1.0 + 0j])
        res = np.zeros(1, complex)
        L.step(lambda v, t: z * v, u, res, 0.0, 1.0)
        assert abs(u[0] - np.polyval(coef[::-1], z)) < 1e-14 * max(1, abs(z) ** 5)


def test_fourth_order_convergence_on_linear_system():
    rng = np.random.default_rng(0)
    Q = rng.normal(size=(6, 6))
    A = Q - Q.T - 0.1 * np.eye(6)
    y0 = rng.normal(size=6)
    T = 1.0
    exact = expm(A * T) @ y0
    errs = []
    for n in (20, 40, 80):
        y = L.integrate(lambda v, t: A @ v, y0, 0.0, T / n, n)
        errs.append(np.linalg.norm(y - exact))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8)


def test_time_dependent_rhs_uses_stage_times():
    # y' = 4 t^3 has y(1) = 1 exactly for a 4th-order scheme with correct C
    y = L.integrate(lambda v, t: np.array([4 * t ** 3]), np.array([0.0]), 0.0, 0.25, 4)
    assert abs(y[0] - 1.0) < 1e-14


@pytest.mark.parametrize("N,ks,expect", [(2, (2, 4), 2.5), (3, (2, 4), 3.5)])
def test_cavity_h_convergence(N, ks, expect):
    T = 0.25
    errs = []
    for k in ks:
        VX, EToV = I.kuhn_cube(k, 0.1, k)
        m = Me.Mesh(N, VX, EToV)
        u0 = I.cavity_mode(m.x, m.y, m.z, 0.0)
        dt0 = D.dt_cfl(m, 0.5)
        ns = int(np.ceil(T / dt0))
        u = L.integrate(lambda v, t: Mx.rhs(m, v), u0, 0.0, T / ns, ns)
        ex = I.cavity_mode(m.x, m.y, m.z, T)
        errs.append(D.mass_norm(m, u - ex) / D.mass_norm(m, u0))
    rate = np.log2(errs[0] / errs[1])
    assert rate > expect


def test_energy_non_increasing_over_steps():
    VX, EToV = I.kuhn_cube(4, 0.1, 0)
    m = Me.Mesh(3, VX, EToV)
    u0 = I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, 1)
    dt = D.dt_cfl(m, 0.5)
    energies = [D.energy(m, u0)]
    L.integrate(lambda v, t: Mx.rhs(m, v), u0, 0.0, dt, 40, callback=lambda n, v: energies.append(D.energy(m, v)))
    assert np.all(np.diff(energies) <= 1e-14 * energies[0])
    assert energies[-1] < energies[0]


def test_cfl_step_inside_stability_region():
    """Spectral radius gate for the dt reading: rho * dt within the imaginary-axis
    limit of the stability polynomial (about 3.34), on a tiny mesh."""
    VX, EToV = I.kuhn_cube(1, 0.1, 0)
    for N in (2, 3, 4):
        m = Me.Mesh(N, VX, EToV)
        A = D.assemble(m, 1.0)
        lam = np.linalg.eigvals(A)
        dt = D.dt_cfl(m, 0.5)
        z = lam * dt
        R = np.polyval(np.array([1, 1, 1 / 2, 1 / 6, 1 / 24, 1 / 200])[::-1], z)
        assert np.abs(R).max() <= 1.0 + 1e-12
