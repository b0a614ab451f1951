"""Pins of the complete Landau-Lifshitz force (Eq. (3dLL) with its derivative
term) and of the RK4 comparator (Section 3's single-particle tests).

The closed-form plane-wave orbits (analytic.PlaneWaveOrbit, reduced and
complete) are checked against a direct adaptive integration of Eq. (3dLL)
itself in lab time, an independent route to the same orbit; the RK4
comparator must converge to them at fourth order; the derivative force is
checked against a finite difference of the fields along the orbit."""
import json
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import analytic, pusher, rk4

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _direct(wave, u0, t_end, eps, full):
    """Eq. (3dLL) for an electron, integrated in t with DOP853 at 1e-12."""
    def f(t, y):
        x, u = y[:3], y[3:]
        E, B = wave.fields(x[0], t)
        if full:
            du = pusher.ll_full(E, B, wave.partials(x[0], t), u, eps)
        else:
            du = pusher.ll_nonderivative(E, B, u, eps)
        return np.concatenate([u / np.sqrt(1 + u @ u), du])
    sol = solve_ivp(f, (0.0, t_end), np.concatenate([np.zeros(3), u0]), method="DOP853",
                    rtol=1e-12, atol=1e-12)
    assert sol.success
    return sol.y[:3, -1], sol.y[3:, -1]


@pytest.mark.parametrize("full", [False, True])
def test_closed_form_orbit_matches_direct_integration_of_eq_3dll(full):
    # amplified RR so that both RR terms matter; CP with a phase offset
    wave = analytic.MonochromaticWave(30.0, 20.0, psi=0.4)
    u0 = np.array([-8.0, 2.0, -1.0])
    eps = 3e-4
    t_end = 25.0
    orb = analytic.PlaneWaveOrbit(wave, u0, eps=eps, phi_span=400.0, full_ll=full)
    x, u = _direct(wave, u0, t_end, eps, full)
    xa, ua, _ = orb.at_time(t_end)
    assert abs(x[0] - xa) <= 1e-8 * max(1.0, abs(xa))
    np.testing.assert_allclose(u, ua, rtol=1e-8, atol=1e-8 * np.abs(ua).max())


def test_derivative_term_changes_the_orbit_only_slightly():
    # the complete and reduced orbits differ, but by far less than RR itself
    wave = analytic.MonochromaticWave(30.0, 20.0, psi=0.4)
    u0 = np.array([-8.0, 2.0, -1.0])
    eps = 3e-4
    red = analytic.PlaneWaveOrbit(wave, u0, eps=eps, phi_span=400.0)
    full = analytic.PlaneWaveOrbit(wave, u0, eps=eps, phi_span=400.0, full_ll=True)
    none = analytic.PlaneWaveOrbit(wave, u0, eps=0.0, phi_span=400.0)
    xr, ur, _ = red.at_time(25.0)
    xf, uf, _ = full.at_time(25.0)
    x0, u0_, _ = none.at_time(25.0)
    d_rr = np.linalg.norm(ur - u0_)
    d_der = np.linalg.norm(uf - ur)
    assert 0 < d_der < 0.05 * d_rr


def test_derivative_force_is_the_total_derivative_of_the_fields():
    # D F = d/dt F(x(t), t) along a straight path x = x0 + v t: finite difference
    wave = analytic.MonochromaticWave(50.0, 10.0, psi=1.1)
    rng = np.random.default_rng(3)
    for _ in range(20):
        u = rng.normal(size=3) * 5
        g = np.sqrt(1 + u @ u)
        v = u / g
        x0, t0, h = rng.normal(), rng.normal(), 1e-5
        E1, B1 = wave.fields(x0 + v[0] * h, t0 + h)
        E0, B0 = wave.fields(x0 - v[0] * h, t0 - h)
        DE, DB = (E1 - E0) / (2 * h), (B1 - B0) / (2 * h)
        want = -1e-3 * g * (DE + np.cross(v, DB))
        got = pusher.derivative_force(*wave.partials(x0, t0), u, 1e-3)
        np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("rr", ["off", "reduced", "full"])
def test_rk4_converges_at_fourth_order(rr):
    # RR amplified so that it changes the final momentum by ~30%, yet not
    # stiff at these steps (with eps = 3e-4 the ratio is still 22 at 0.01)
    wave = analytic.MonochromaticWave(30.0, 20.0, psi=0.4)
    u0 = np.array([-8.0, 2.0, -1.0])
    eps = 3e-5
    t_end = 12.0
    orb = analytic.PlaneWaveOrbit(wave, u0, eps=eps if rr != "off" else 0.0, phi_span=400.0,
                                  full_ll=(rr == "full"))
    xa, ua, _ = orb.at_time(t_end)
    errs = []
    for dt in (0.02, 0.01):
        x, u = rk4.track(wave, np.zeros(3), u0, 0.0, dt, int(round(t_end / dt)), eps, rr)
        errs.append(np.linalg.norm(u - ua) / np.linalg.norm(ua))
    assert errs[1] < 1e-6
    assert errs[0] / errs[1] == pytest.approx(16.0, rel=0.2)


def test_paper_scheme_with_the_derivative_term_converges_to_the_complete_solution():
    wave = analytic.MonochromaticWave(30.0, 20.0, psi=0.4)
    u0 = np.array([-8.0, 2.0, -1.0])
    eps = 3e-6
    t_end = 12.0
    orb = analytic.PlaneWaveOrbit(wave, u0, eps=eps, phi_span=400.0, full_ll=True)
    errs = []
    for dt in (0.02, 0.01):
        _, u, _ = orb.at_time(-0.5 * dt)
        x = np.zeros(3)
        n = int(round(t_end / dt))
        for k in range(n):
            E, B = wave.fields(x[0], k * dt)
            u, _ = pusher.push(u, E, B, -1.0, dt, eps, True, partials=wave.partials(x[0], k * dt))
            x = x + dt * u / np.sqrt(1 + u @ u)
        xa, _, _ = orb.at_time(n * dt)
        errs.append(abs(x[0] - xa))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.2)


def test_worked_example_derivative_term_is_negligible():
    # Section 3: the derivative term of Eq. (3dLL) is negligible in the worked
    # example (p_x0 = -200, a0 = 350, 0.8 um, 500/omega).  Its effect on the
    # longitudinal displacement is far below the scheme's own error there.
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    wave = analytic.MonochromaticWave(g["a0"])
    eps = pusher.rr_coefficient(g["lambda_um"])
    u0 = np.array([g["p_x0"], 0.0, 0.0])
    red = analytic.PlaneWaveOrbit(wave, u0, eps=eps, phi_span=4000.0)
    full = analytic.PlaneWaveOrbit(wave, u0, eps=eps, phi_span=4000.0, full_ll=True)
    xr, _, _ = red.at_time(g["t_end"])
    xf, _, _ = full.at_time(g["t_end"])
    rel = abs(xf - xr) / abs(xr)
    assert rel < 0.1 * g["rel_displacement_error_reported"]
