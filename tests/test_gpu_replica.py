"""The paper's own laser-foil runs (Section 4), reproduced qualitatively.

Intensity 2.33e23 W/cm^2 at 0.8 um (a0 = 328), hydrogen foil at n0 = 100 n_c
and 14 wavelengths, trapezoidal pulse (1-cycle sin^2 rise and fall, 5-cycle
plateau), LP and CP, foil 1 wavelength (CP also 0.3: the transparency
case), with and without RR.  The paper's time t_p starts when the pulse
front reaches the foil (here t = t_p + 14 T).  The paper prints no grid or
particle numbers; the runs use 200 cells per wavelength and 1,000 particles
per cell per species, in a 70-wavelength box so that the ions stay inside
until t_p = 46 T.  Its figures are absent, so what is checked are the
statements of Section 4, with wide margins:
* LP: RR dissipates "about 20%" of the pulse energy; the friction
  coefficient d of Eq. (damping) reaches ~1e2 in the skin layer near
  t_p = 1.7 T, against ~1e-2 for CP; at t_p = 12 T the ion spectrum is
  narrower and has lost its low-energy tail with RR; at 46 T the missing ion
  energy is about the dissipated fraction;
* CP, 1 wavelength: RR effects on the ions are negligible;
* CP, 0.3 wavelength: the pulse breaks through and RR raises the ion
  energies."""
import numpy as np
import pytest

from oracle import spectrum
from workloads import preset

pytestmark = pytest.mark.gpu

DEAD = np.iinfo(np.int32).min


def _ions(run, cfg):
    ions = run.get_particles(1, 0, run.get_info()["capacity"], keys=("cell", "ux", "uy", "uz"))
    alive = ions["cell"] != DEAD
    u = np.stack([ions[k][alive] for k in ("ux", "uy", "uz")], 1)
    E = spectrum.ion_energies_mev(u, cfg["mass_ratio"])
    return dict(mean=float(E.mean()), p10=float(np.percentile(E, 10)), p50=float(np.median(E)),
                p90=float(np.percentile(E, 90)), max=float(E.max()))


def _friction(run):
    """Friction coefficient d of Eq. (damping) of the electrons, from the GPU:
    its maximum and 99th percentile (from the histogram in log10 d)."""
    bins, lo, hi = 600, -9.0, 6.0
    h, st = run.friction(bins, lo, hi)
    edges = np.linspace(lo, hi, bins + 1)
    h = h.copy()
    h[0] += st["below"]  # (electrons with d below 1e-9 count in the lowest bin)
    p99 = spectrum.central_range(h / np.diff(edges), edges, 0.99, 0.99)[0]
    return st["max"], 10.0 ** p99


@pytest.fixture(scope="module")
def campaign():
    import torch

    from paper_1008_1685_amd import Run

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    out = {}
    for pol, ell in (("LP", 1.0), ("CP", 1.0), ("CP", 0.3)):
        for rr in (True, False):
            print(f"\n[gpu] paper run {pol} {ell} lambda rr={rr}", flush=True)
            cfg = preset("paper", pol=pol, thickness=ell, rr=rr, box_lambda=70.0, periods=60.0)
            run = Run(cfg)
            spp = cfg["cells_per_lambda"] / cfg["cfl"]
            done = 0
            rec = {"curve": []}
            # the absorption curve every period (Section 4's fractional energy
            # absorption against time), d at 1.7 periods, spectra at 12 and 46
            for tp in sorted(set(np.arange(0.0, 47.0)) | {1.7}):
                n = int(round((cfg["x_foil"] + tp) * spp)) - done
                run.step(n)
                done += n
                if tp == 1.7:
                    rec["d_max"], rec["d_p99"] = _friction(run)
                    continue
                dg = run.diag()
                assert dg["gauss_int"] == 0 and not dg["nonfinite"]
                e_in = max(dg["E_in"], 1e-300)
                rec["curve"].append(dict(t_p=tp, K_e=dg["K_e"] / e_in, K_i=dg["K_i"] / e_in,
                                         E_rad=dg["E_rad"] / e_in, E_in=dg["E_in"]))
                if tp in (12.0, 46.0):
                    rec[f"ions_{tp:g}"] = _ions(run, cfg)
                    rec[f"E_rad_{tp:g}"] = dg["E_rad"] / dg["E_in"]
                    rec[f"K_i_{tp:g}"] = dg["K_i"] / dg["E_in"]
            run.close()
            out[(pol, ell, rr)] = rec
            print({k: v for k, v in rec.items() if k != "curve"}, flush=True)
            print("absorption curve (t_p, K_e, K_i, E_rad as fractions of E_in):",
                  [(c["t_p"], round(c["K_e"], 4), round(c["K_i"], 4), round(c["E_rad"], 4))
                   for c in rec["curve"][::3]], flush=True)
    return out


def test_lp_dissipates_about_a_fifth_of_the_pulse(campaign):
    f = campaign[("LP", 1.0, True)]["E_rad_46"]
    assert 0.08 < f < 0.35, f


def test_lp_absorption_curve(campaign):
    # Section 4 (fractional energy absorption against time, LP): RR dissipates
    # its share during the laser-foil interaction, which lasts about 22
    # periods with RR (30 without), and the loss then stops growing; during
    # the interaction the ions hold almost the same energy with and without RR
    rr = {c["t_p"]: c for c in campaign[("LP", 1.0, True)]["curve"]}
    no = {c["t_p"]: c for c in campaign[("LP", 1.0, False)]["curve"]}
    final = rr[46.0]["E_rad"]
    assert all(rr[t + 1]["E_rad"] * rr[t + 1]["E_in"] >= rr[t]["E_rad"] * rr[t]["E_in"] - 1e-9
               for t in np.arange(0.0, 46.0))  # the radiated energy only grows
    t95 = min(t for t, c in rr.items() if c["E_rad"] >= 0.95 * final)
    assert 8.0 <= t95 <= 35.0, t95
    assert rr[46.0]["E_rad"] - rr[35.0]["E_rad"] < 0.05 * final
    assert rr[12.0]["K_i"] == pytest.approx(no[12.0]["K_i"], rel=0.15)
    assert all(c["E_rad"] == 0.0 for c in no.values())


def test_friction_coefficient_lp_against_cp(campaign):
    lp, cp = campaign[("LP", 1.0, True)], campaign[("CP", 1.0, True)]
    assert 30.0 < lp["d_max"] < 1000.0
    assert 1e-3 < cp["d_p99"] < 1.0
    assert lp["d_max"] > 100 * cp["d_max"]


def test_lp_spectrum_at_12_periods_is_narrower_without_its_low_energy_tail(campaign):
    rr, no = campaign[("LP", 1.0, True)]["ions_12"], campaign[("LP", 1.0, False)]["ions_12"]
    assert (rr["p90"] - rr["p10"]) < 0.7 * (no["p90"] - no["p10"])
    assert rr["p10"] > 2.0 * no["p10"]
    assert rr["p50"] < no["p50"]  # lower peak energy with RR


def test_lp_missing_ion_energy_is_about_the_dissipated_fraction(campaign):
    rr, no = campaign[("LP", 1.0, True)], campaign[("LP", 1.0, False)]
    ratio = rr["K_i_46"] / no["K_i_46"]
    assert abs(ratio - (1.0 - rr["E_rad_46"])) < 0.07, (ratio, rr["E_rad_46"])


def test_cp_thick_foil_rr_is_negligible(campaign):
    rr, no = campaign[("CP", 1.0, True)], campaign[("CP", 1.0, False)]
    assert rr["E_rad_46"] < 1e-3
    assert rr["ions_46"]["mean"] == pytest.approx(no["ions_46"]["mean"], rel=0.01)
    assert rr["ions_46"]["p50"] == pytest.approx(no["ions_46"]["p50"], rel=0.02)


def test_cp_thin_foil_breaks_through_and_rr_raises_ion_energies(campaign):
    rr, no = campaign[("CP", 0.3, True)], campaign[("CP", 0.3, False)]
    thick = campaign[("CP", 1.0, True)]
    assert rr["E_rad_46"] > 0.02  # RR matters once the pulse breaks through
    assert rr["ions_46"]["mean"] > 1.05 * no["ions_46"]["mean"]
    assert rr["ions_46"]["p50"] > no["ions_46"]["p50"]
    # the spectrum is far from monoenergetic: much broader than the thick foil's
    assert (rr["ions_46"]["p90"] - rr["ions_46"]["p10"]) > 2 * (thick["ions_46"]["p90"] - thick["ions_46"]["p10"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_reduced_lp_replica_matches_the_oracle(precision):
    # the paper's LP run at 100 cells per wavelength and 64 particles per cell
    # (tests/golden/make_replica_reference.py, oracle, seeds 0-2), to
    # t_p = 12: each run's balance within 1e-3 of the injected energy; the
    # absorption curve (electron, ion, radiated and field fractions every
    # period) as seed means, within 1e-3 of the injected energy plus the
    # oracle's own seed spread (the LP heating is chaotic: single runs differ
    # by ~1e-2); the friction coefficient d at t_p = 1.7 run by run within 1%
    import json
    import os

    from paper_1008_1685_amd import Run

    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "replica_reference.json")))
    seeds = sorted(ref["seeds"], key=int)
    curves, fr = [], []
    for s in seeds:
        r = ref["seeds"][s]
        cfg = preset("paper", seed=int(s), precision=precision, **ref["overrides"])
        run = Run(cfg)
        done = 0
        rows = []
        for c in sorted([dict(step=r["friction"]["step"], friction=True)] + r["curve"],
                        key=lambda c: c["step"]):
            run.step(c["step"] - done)
            done = c["step"]
            if c.get("friction"):
                _, st = run.friction(64, -8.0, 8.0)
                fr.append((st["max"], st["mean"]))
                continue
            d = run.diag()
            assert d["gauss_int"] == 0
            assert d["E_in"] == pytest.approx(c["E_in"], rel=1e-6)
            assert abs(d["balance"] / d["E_in"] - c["balance"]) <= 1e-3, (s, c["t_p"])
            rows.append({k: d[k] / d["E_in"] for k in ("K_e", "K_i", "E_rad", "U_field")})
        curves.append(rows)
        run.close()
    for i, c in enumerate(ref["seeds"][seeds[0]]["curve"]):
        for k in ("K_e", "K_i", "E_rad", "U_field"):
            o = np.array([ref["seeds"][s]["curve"][i][k] for s in seeds])
            g = np.array([cv[i][k] for cv in curves])
            if k == "E_rad":
                print(f"[{precision} t_p {c['t_p']:g}] {k}: GPU {g.mean():.4f} oracle {o.mean():.4f} "
                      f"(seed spread {np.ptp(o):.4f})", flush=True)
            assert abs(g.mean() - o.mean()) <= 1e-3 + np.ptp(o), (c["t_p"], k, g, o)
    # at t_p = 1.7 the heating has not yet turned chaotic: d run by run, within 1%
    for s, (gmax, gmean) in zip(seeds, fr):
        o = ref["seeds"][s]["friction"]
        print(f"[{precision} seed {s}] d at t_p = 1.7: max {gmax:.3f} (oracle {o['max']:.3f}), "
              f"mean {gmean:.4f} (oracle {o['mean']:.4f})", flush=True)
        assert abs(gmax - o["max"]) <= 0.01 * o["max"], (s, gmax, o)
        assert abs(gmean - o["mean"]) <= 0.01 * o["mean"], (s, gmean, o)
