"""Exact single-electron solutions used to pin the pusher.

TEST INFRASTRUCTURE ONLY (see package header).

Plane wave (Section 2 refers to the exact LL solution in a plane wave as the
benchmark; Section 3 validates the pusher against it).  The wave travels
along +x with phase phi = t - x, transverse field E_perp(phi) = (E_y, E_z),
B = (0, -E_z, E_y) and potential A(phi) with E_perp = -dA/dphi.  For an
electron under the Lorentz force plus the non-derivative LL terms
(Eq. (3dLL) without its derivative term, i.e. the force the PIC pusher
integrates) the equations reduce to quadratures:

  h = gamma - u_x obeys dh/dphi = -eps E_perp^2 h^2, so
      1/h(phi) = 1/h0 + eps I(phi),   I(phi) = int_{phi0}^{phi} E_perp^2,
  u_perp / h obeys d(u_perp/h)/dphi = -E_perp / h, so
      u_perp = (h/h0) [u_perp0 + A(phi) - A(phi0) - eps h0 K(phi)],
      K(phi) = int_{phi0}^{phi} E_perp I,
  u_x = (1 + u_perp^2 - h^2) / (2 h),  dt/dphi = gamma / h,  dx/dphi = u_x / h.

With eps = 0 this is the textbook Lorentz orbit (h conserved, u_perp =
u_perp0 + A - A0).

The complete Eq. (3dLL) adds -eps gamma [D E + v x D B], D = d/dt + v.grad
the total derivative along the orbit.  In a plane wave D F = (1 - v_x) F'
(prime: d/dphi), so the term is -eps h [E' + v x B']: it does no work on
h (dh/dphi unchanged) and adds -eps h E_perp' to du_perp/dphi, hence
-eps E_perp' to d(u_perp/h)/dphi.  The complete solution therefore has the
extra term -eps h0 (E_perp(phi) - E_perp(phi0)) inside the bracket of
u_perp, with h as above (``full_ll``).  The derivation uses only f_L x B + (v.E) E =
(1 - v_x) E_perp^2 x_hat and gamma^2 [F^2 - (v.E)^2] = h^2 E_perp^2 for a
plane wave; both identities are checked numerically in the tests.  The
quadratures are integrated by an adaptive 8th-order method at 1e-13
tolerance, far below any pusher error being measured.

Uniform magnetic field, E = 0, u perpendicular to B:
  * Boris rotates u by exactly 2 atan(|qm| |B| dt / (2 gamma)) per step;
  * with RR, d gamma/dt = -eps B^2 (gamma^2 - 1), so
    gamma(t) = coth(eps B^2 t + atanh(1/gamma0)).
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp
from scipy.optimize import brentq


class MonochromaticWave:
    """Plane wave with A_y = a_y sin(phi + psi), A_z = a_z cos(phi + psi)
    (a_z = 0: linear polarisation) so E_perp = -dA/dphi."""

    def __init__(self, a_y: float, a_z: float = 0.0, psi: float = 0.0):
        self.ay, self.az, self.psi = float(a_y), float(a_z), float(psi)

    def A(self, phi):
        ph = phi + self.psi
        return np.array([self.ay * np.sin(ph), self.az * np.cos(ph)])

    def E(self, phi):
        ph = phi + self.psi
        return np.array([-self.ay * np.cos(ph), self.az * np.sin(ph)])

    def dE(self, phi):
        """dE_perp/dphi."""
        ph = phi + self.psi
        return np.array([self.ay * np.sin(ph), self.az * np.cos(ph)])

    def partials(self, x, t):
        """(dE/dt, dE/dx, dB/dt, dB/dx) in the lab frame at (x, t), each of
        shape (..., 3): a function of phi = t - x, so d/dx = -d/dt."""
        phi = np.asarray(t - x, dtype=np.float64)
        dp = self.dE(phi)
        zero = np.zeros_like(phi)
        Et = np.stack([zero, dp[0], dp[1]], axis=-1)
        Bt = np.stack([zero, -dp[1], dp[0]], axis=-1)
        return Et, -Et, Bt, -Bt

    def fields(self, x, t):
        """Lab-frame E and B (shape (..., 3)) at position x and time t."""
        phi = np.asarray(t - x, dtype=np.float64)
        Ep = self.E(phi)
        zero = np.zeros_like(phi)
        E = np.stack([zero, Ep[0], Ep[1]], axis=-1)
        B = np.stack([zero, -Ep[1], Ep[0]], axis=-1)
        return E, B


class PlaneWaveOrbit:
    """Exact electron orbit in a plane wave, Lorentz plus the non-derivative
    LL terms (``full_ll``: plus the derivative term as well).

    Initial condition: position x0 and momentum u0 at time t0."""

    def __init__(self, wave, u0, x0=0.0, t0=0.0, eps=0.0, phi_span=200.0, full_ll=False):
        self.w, self.eps, self.full = wave, float(eps), bool(full_ll)
        u0 = np.asarray(u0, dtype=np.float64)
        self.phi0 = t0 - x0
        g0 = np.sqrt(1.0 + u0 @ u0)
        self.h0 = g0 - u0[0]
        self.up0 = u0[1:].copy()
        self.A0 = wave.A(self.phi0)
        self.E0 = wave.E(self.phi0)
        y0 = np.array([0.0, 0.0, 0.0, t0, x0])
        kw = dict(method="DOP853", rtol=1e-13, atol=1e-13, dense_output=True)
        self.fwd = solve_ivp(self._rhs, (self.phi0, self.phi0 + phi_span), y0, **kw)
        self.bwd = solve_ivp(self._rhs, (self.phi0, self.phi0 - 20.0), y0, **kw)
        if not (self.fwd.success and self.bwd.success):
            raise RuntimeError("quadrature failed")

    def _state(self, phi, I, K):
        h = 1.0 / (1.0 / self.h0 + self.eps * I)
        br = self.up0 + self.w.A(phi) - self.A0 - self.eps * self.h0 * K
        if self.full:
            br = br - self.eps * self.h0 * (self.w.E(phi) - self.E0)
        up = (h / self.h0) * br
        ux = (1.0 + up @ up - h * h) / (2.0 * h)
        return h, ux, up

    def _rhs(self, phi, y):
        I, K = y[0], y[1:3]
        Ep = self.w.E(phi)
        h, ux, up = self._state(phi, I, K)
        g = h + ux
        return np.array([Ep @ Ep, Ep[0] * I, Ep[1] * I, g / h, ux / h])

    def _y(self, phi):
        return (self.fwd if phi >= self.phi0 else self.bwd).sol(phi)

    def at_phase(self, phi):
        """(t, x, u) on the orbit at phase ``phi``."""
        y = self._y(phi)
        h, ux, up = self._state(phi, y[0], y[1:3])
        return y[3], y[4], np.array([ux, up[0], up[1]])

    def at_time(self, t):
        """(x, u, phi) on the orbit at lab time ``t``."""
        f = lambda ph: self._y(ph)[3] - t
        lo = self.bwd.t[-1]
        hi = self.fwd.t[-1]
        if f(hi) < 0 or f(lo) > 0:
            raise ValueError("time outside integrated phase range")
        phi = brentq(f, lo, hi, xtol=1e-13, rtol=1e-15, maxiter=500)
        _, x, u = self.at_phase(phi)
        return x, u, phi


def px_time_lag(orbit, t, px, span=1.0, step=1e-4):
    """Phase error of a computed longitudinal momentum against the exact
    orbit (Section 3 quotes it for its worked example): the time shift tau,
    |tau| <= span, that best maps the samples px(t) onto the exact p_x, in the
    least-squares sense (the exact p_x(t + tau) from the orbit's dense
    solution, sampled on a fine grid of phases and interpolated linearly)."""
    t = np.asarray(t, dtype=np.float64)
    px = np.asarray(px, dtype=np.float64)
    _, _, ph_lo = orbit.at_time(t.min() - span - 0.1)
    _, _, ph_hi = orbit.at_time(t.max() + span + 0.1)
    ph = np.linspace(ph_lo, ph_hi, 200001)
    tt = np.empty_like(ph)
    ux = np.empty_like(ph)
    for i, p in enumerate(ph):
        tt[i], _, u = orbit.at_phase(p)
        ux[i] = u[0]
    taus = np.arange(-span, span + 0.5 * step, step)
    err = np.array([np.sum((np.interp(t + tau, tt, ux) - px) ** 2) for tau in taus])
    k = int(np.argmin(err))
    if 0 < k < taus.size - 1:  # parabola through the three smallest
        y0, y1, y2 = err[k - 1], err[k], err[k + 1]
        den = y0 - 2.0 * y1 + y2
        if den > 0:
            return float(taus[k] + 0.5 * step * (y0 - y2) / den)
    return float(taus[k])


def boris_rotation_angle(qm, B_abs, dt, gamma):
    """Angle of one Boris rotation in a pure magnetic field."""
    return 2.0 * np.arctan(abs(qm) * B_abs * dt / (2.0 * gamma))


def rr_cooling_gamma(t, gamma0, B_abs, eps):
    """gamma(t) of an electron gyrating perpendicular to a uniform B with the
    non-derivative LL force: coth(eps B^2 t + atanh(1/gamma0))."""
    return 1.0 / np.tanh(eps * B_abs * B_abs * t + np.arctanh(1.0 / gamma0))
