"""Particle pusher with the reduced Landau-Lifshitz radiation reaction, FP64.

TEST INFRASTRUCTURE ONLY (see package header).

Units (paper, Section 2): t in 1/omega, x in c/omega, momentum in m c,
fields in m omega c/|e|.  ``u`` is the momentum per unit mass of the
species (u = p / (M c), gamma = sqrt(1 + u^2)); ``qm`` is the charge-to-mass
ratio in electron units (-1 for electrons, +1/1836 for protons).

Pins (tests/test_oracle_pusher.py): exact E-only kick, Boris rotation angle
in a uniform B field, reduction to a Rodrigues rotation, agreement of
Eq. (f_r) with the non-derivative part of Eq. (3dLL), the two forms of
Eq. (damping), the limits of d stated after Eq. (damping), the closed-form
plane-wave orbit with and without RR, radiative cooling in a uniform B field.
"""
from __future__ import annotations

import numpy as np

# classical electron radius in micrometres (CODATA 2018: 2.8179403262e-15 m)
R_E_UM = 2.8179403262e-9


def rr_coefficient(lambda_um: float) -> float:
    """The RR strength (4 pi / 3) r_e / lambda that multiplies every RR term
    of Eq. (3dLL); lambda is the laser wavelength in micrometres."""
    return 4.0 * np.pi / 3.0 * R_E_UM / lambda_um


def _dot(a, b):
    return np.sum(a * b, axis=-1)


def gamma_of(u):
    """Lorentz factor sqrt(1 + u^2) of momentum ``u`` (..., 3)."""
    return np.sqrt(1.0 + _dot(u, u))


def boris(u, E, B, qm, dt):
    """Boris step for the Lorentz force alone: u^{n-1/2} -> u_L^{n+1/2}.

    Half electric kick, rotation about B by the angle 2 atan(|t|) with
    t = (qm dt / 2) B / gamma^-, second half electric kick (the standard
    scheme the paper keeps unchanged, Section 3)."""
    h = 0.5 * qm * dt
    um = u + h * E
    g = gamma_of(um)
    t = (h / g)[..., None] * B if np.ndim(g) else (h / g) * B
    s = 2.0 * t / (1.0 + _dot(t, t))[..., None]
    up = um + np.cross(um, t)
    upl = um + np.cross(up, s)
    return upl + h * E


def rr_force(E, B, p, eps):
    """RR force of Eq. (f_r) on an electron with momentum ``p``:

        f_R = -eps { f_L x B - (v.E) E + gamma^2 [ f_L^2 - (v.E)^2 ] v },
        f_L = -(E + v x B),  v = p / gamma,  gamma = sqrt(1 + p^2).

    The bracket f_L^2 - (v.E)^2 is non-negative in exact arithmetic (it is
    d / (eps gamma^2), Eq. (damping)); it is clamped at zero so rounding can
    never turn the friction into an acceleration."""
    g = gamma_of(p)
    v = p / g[..., None]
    fL = -(E + np.cross(v, B))
    vE = _dot(v, E)
    bracket = np.maximum(_dot(fL, fL) - vE * vE, 0.0)
    return -eps * (np.cross(fL, B) - vE[..., None] * E
                   + (g * g * bracket)[..., None] * v)


def derivative_force(Et, Ex, Bt, Bx, p, eps):
    """The derivative term of Eq. (3dLL) for an electron with momentum p:
    -eps gamma [D E + v x D B], D = d/dt + v_x d/dx (fields of x and t only,
    as on the 1D grid), from the partial derivatives at the particle."""
    g = gamma_of(p)
    v = p / g[..., None]
    vx = v[..., :1]
    DE = Et + vx * Ex
    DB = Bt + vx * Bx
    return -eps * g[..., None] * (DE + np.cross(v, DB))


def push(u_old, E, B, qm, dt, eps, rr, partials=None):
    """One leapfrog momentum step of the paper's scheme (Section 3).

    1. Lorentz part by Boris: u_L^{n+1/2} (Eq. (part1), left).
    2. Mid-step estimate p^(n) = (u_L^{n+1/2} + u^{n-1/2}) / 2, gamma^(n) and
       v^(n) from it (Eqs. (estim1), (estimgamma)).
    3. u^{n+1/2} = u_L^{n+1/2} + f_R^(n) dt with f_R from Eq. (f_r) at the
       fields E^(n), B^(n) (Eq. (pertfull)).

    With ``partials`` = (dE/dt, dE/dx, dB/dt, dB/dx) at the particle the
    derivative term of Eq. (3dLL) is added to f_R, evaluated at the same
    p^(n) (the complete LL force of the paper's single-particle tests).

    Returns (u_new, u_L).  With ``rr`` false (or eps = 0) u_new = u_L."""
    uL = boris(u_old, E, B, qm, dt)
    if not rr:
        return uL, uL
    p_mid = 0.5 * (uL + u_old)
    f = rr_force(E, B, p_mid, eps)
    if partials is not None:
        f = f + derivative_force(*partials, p_mid, eps)
    return uL + dt * f, uL


def ll_full(E, B, partials, u, eps):
    """Right-hand side of the complete Eq. (3dLL) for an electron."""
    return ll_nonderivative(E, B, u, eps) + derivative_force(*partials, u, eps)


def ll_nonderivative(E, B, u, eps):
    """Right-hand side of Eq. (3dLL) for an electron without the term with
    total time derivatives of the fields:

        -(E + v x B) + eps [(E + v x B) x B + (v.E) E]
                     - eps gamma^2 [(E + v x B)^2 - (v.E)^2] v."""
    g = gamma_of(u)
    v = u / g[..., None]
    F = E + np.cross(v, B)
    vE = _dot(v, E)
    return (-F + eps * (np.cross(F, B) + vE[..., None] * E)
            - eps * (g * g * (_dot(F, F) - vE * vE))[..., None] * v)


def damping(E, B, u, eps):
    """Friction coefficient d of Eq. (damping), both printed forms.

    Returns (d_expanded, d_compact):
      expanded: eps g^2 [E^2 - (v.E)^2 + v^2 B^2 - (v.B)^2 - 2 v.(E x B)]
      compact:  eps g^2 [f_L^2 - (v.f_L)^2],  f_L = -(E + v x B)."""
    g = gamma_of(u)
    v = u / g[..., None]
    vE, vB = _dot(v, E), _dot(v, B)
    expanded = (_dot(E, E) - vE * vE + _dot(v, v) * _dot(B, B) - vB * vB
                - 2.0 * _dot(v, np.cross(E, B)))
    fL = -(E + np.cross(v, B))
    vf = _dot(v, fL)
    compact = _dot(fL, fL) - vf * vf
    return eps * g * g * expanded, eps * g * g * compact
