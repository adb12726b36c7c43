"""Five-stage, fourth-order low-storage Runge-Kutta (Carpenter & Kennedy, 2N storage).  Test infrastructure only.

The paper's timings (Section 5) cover whole time steps with a fourth-order
Runge-Kutta update but do not name the scheme; the reading taken here is the
5-stage 2N-storage RK4 of Carpenter and Kennedy (1994):
    res <- A_s res + dt f(u, t + C_s dt);   u <- u + B_s res,   s = 1..5, A_1 = 0.

Parity: pinned by tests/test_oracle_lserk.py -- the stage coefficients,
written out as a Butcher tableau, satisfy all eight order-<=4 conditions; the
stability polynomial read off from y' = lambda y is
1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/200; a linear ODE system is integrated
with fourth-order convergence against its matrix exponential.
"""
from __future__ import annotations

import numpy as np

A = np.array([0.0,
              -567301805773.0 / 1357537059087.0,
              -2404267990393.0 / 2016746695238.0,
              -3550918686646.0 / 2091501179385.0,
              -1275806237668.0 / 842570457699.0])
B = np.array([1432997174477.0 / 9575080441755.0,
              5161836677717.0 / 13612068292357.0,
              1720146321549.0 / 2090206949498.0,
              3134564353537.0 / 4481467310338.0,
              2277821191437.0 / 14882151754819.0])
C = np.array([0.0,
              1432997174477.0 / 9575080441755.0,
              2526269341429.0 / 6820363962896.0,
              2006345519317.0 / 3224310063776.0,
              2802321613138.0 / 2924317926251.0])


def step(f, u, res, t: float, dt: float):
    """One time step in place on (u, res); f(u, t) returns du/dt."""
    for s in range(5):
        k = f(u, t + C[s] * dt)
        res *= A[s]
        res += dt * k
        u += B[s] * res
    return u, res


def integrate(f, u0, t0: float, dt: float, nsteps: int, callback=None):
    """nsteps steps from u0 (copied); callback(step_index, u) after each step."""
    u = np.array(u0, dtype=np.float64, copy=True)
    res = np.zeros_like(u)
    t = t0
    for n in range(nsteps):
        step(f, u, res, t, dt)
        t += dt
        if callback is not None:
            callback(n, u)
    return u


def butcher():
    """Equivalent Butcher tableau (a, b, c) of the 2N-storage scheme.

    With res_s = A_s res_{s-1} + dt k_s and u_s = u_{s-1} + B_s res_s, the
    increment carried by res_s is sum_j G[s, j] k_j with G[s, s] = 1,
    G[s, j] = A_s G[s-1, j]; stage s+1 sees u_0 + sum_{m<=s} B_m res_m."""
    G = np.zeros((5, 5))
    for s in range(5):
        if s > 0:
            G[s, :s] = A[s] * G[s - 1, :s]
        G[s, s] = 1.0
    a = np.zeros((5, 5))
    for s in range(1, 5):
        a[s] = B[:s] @ G[:s]
    b = B @ G
    c = a.sum(axis=1)
    return a, b, c
