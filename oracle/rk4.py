"""Classical fourth-order Runge-Kutta integration of one electron in given
analytic fields: the comparator the paper uses for its single-particle tests
of the pusher (Section 3), for convergence studies.

TEST INFRASTRUCTURE ONLY (see package header).

State (x, u) at the same time t (no staggering): dx/dt = u / gamma and
du/dt = the right-hand side of Eq. (3dLL) for an electron - the Lorentz
force alone (rr = "off"), with the non-derivative RR terms ("reduced", the
force the PIC integrates) or with the derivative term as well ("full").
Pinned (tests/test_oracle_rk4.py) by fourth-order convergence to the exact
plane-wave orbits of ``analytic``.
"""
from __future__ import annotations

import numpy as np

from . import pusher


def rhs(wave, x, t, u, eps, rr):
    """(dx/dt, du/dt) for position x (3,), time t, momentum u (3,)."""
    E, B = wave.fields(x[..., 0], t)
    g = pusher.gamma_of(u)
    if rr == "off":
        du = pusher.ll_nonderivative(E, B, u, 0.0)
    elif rr == "reduced":
        du = pusher.ll_nonderivative(E, B, u, eps)
    elif rr == "full":
        du = pusher.ll_full(E, B, wave.partials(x[..., 0], t), u, eps)
    else:
        raise ValueError(rr)
    return u / g[..., None] if np.ndim(g) else u / g, du


def track(wave, x0, u0, t0, dt, n, eps, rr="reduced"):
    """n RK4 steps of size dt from (x0, u0) at t0; returns (x, u) at t0 + n dt."""
    x = np.array(x0, dtype=np.float64)
    u = np.array(u0, dtype=np.float64)
    for k in range(n):
        t = t0 + k * dt
        k1x, k1u = rhs(wave, x, t, u, eps, rr)
        k2x, k2u = rhs(wave, x + 0.5 * dt * k1x, t + 0.5 * dt, u + 0.5 * dt * k1u, eps, rr)
        k3x, k3u = rhs(wave, x + 0.5 * dt * k2x, t + 0.5 * dt, u + 0.5 * dt * k2u, eps, rr)
        k4x, k4u = rhs(wave, x + dt * k3x, t + dt, u + dt * k3u, eps, rr)
        x = x + dt / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x)
        u = u + dt / 6.0 * (k1u + 2.0 * k2u + 2.0 * k3u + k4u)
    return x, u
