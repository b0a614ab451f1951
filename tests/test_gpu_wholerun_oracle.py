"""Whole laser-foil runs against the FP64 oracle (Section 2 energy balance,
Section 4 proton spectra).

References come from tests/golden/make_c1_reference.py and
make_c2_reference.py, which call only the oracle.  Each GPU run uses the
same configuration and seed as its reference.  The comparisons:

* the injected energy to 1e-6 (the laser is analytic) and the integer Gauss
  law exactly, at every stored step;
* the energy balance (what is in the box, plus what was radiated or left,
  minus what entered; a fraction of the injected energy) of every run within
  1e-3 of the oracle's, at every stored step: conservation is not chaotic;
* each budget term: a term of at least 1e-3 of the injected energy within
  1e-3 of it; a smaller term within 1e-3 of its own size plus twice the
  oracle's noise floor of that term at that step (the larger of its
  seed-to-seed spread and its response to a float32-rounded start), plus
  1e-10 of the injected energy, below which a term is rounding noise: RR
  before the pulse arrives, where FP32 partial sums round 1e-83 to zero, or
  the 2e-9 reflected at the entrance before the pulse reaches the foil,
  which FP32 fields of the incident amplitude resolve to ~0.3%.  The small terms (the radiated energy of these circularly polarised
  runs, light leaving at the far end, escaped particles) move by 5-50%
  between runs: the light transmitted through the c1 foil (6e-5 of the
  injected energy) moves by up to 8% when only the start is rounded, more
  than its spread over eight seeds;
* the proton spectrum's peak (maximum of E f(E), 512 bins) and width (the
  energy range of the central 80% of the protons) within 1%, as means over
  eight seeds.
At 512 particles per cell (c1w) every run is held to the budget bounds run
by run.  The spectrum is compared as seed means at both resolutions: single
runs move the peak by 0.05-1.4% and the width by 0.3-1.4% when only their
start is rounded to float32 (the oracle's own response, measured), so a
single run cannot be held to 1% (the bunch carries spikes a few tenths of a
MeV wide; at 4,096 bins the maximum of E f(E) picks one of them).  At 64
particles per cell (c1, the small workload as specified) single runs respond
to that rounding by about 1e-3 of the injected energy in single terms, so
the terms too are compared as means over eight seeds; the balance is still
held run by run.
"""
import glob
import json
import os

import numpy as np
import pytest

from oracle import spectrum
from workloads import preset

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TERMS = ("U_field", "K_e", "K_i", "E_rad", "E_out_left", "E_out_right", "E_esc")


@pytest.fixture(autouse=True)
def _announce(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def _refs(workload):
    out = {}
    for f in sorted(glob.glob(os.path.join(GOLD, "c1_reference", f"{workload}_seed*.json"))):
        r = json.load(open(f))
        out[(r["seed"], r["f32_start"])] = r
    return out


def _spread(refs):
    """Per stored step and term, the oracle's own noise floor (fraction of
    E_in): the larger of its seed-to-seed spread (max - min over the seeds)
    and its largest response to rounding the initial offsets to float32 (the
    seeds that have both runs)."""
    runs = [r for (s, f), r in refs.items() if not f]
    pairs = [(refs[(s, False)], r) for (s, f), r in refs.items() if f and (s, False) in refs]
    n = len(runs[0]["series"])
    out = []
    for i in range(n):
        row = {}
        for k in TERMS:
            ptp = float(np.ptp([r["series"][i][k] for r in runs]))
            pert = max((abs(a["series"][i][k] - b["series"][i][k]) for a, b in pairs), default=0.0)
            row[k] = max(ptp, pert)
        out.append(row)
    return out


def _gpu_run(cfg, every, n_steps, bins, e_max):
    from paper_1008_1685_amd import Run

    run = Run(cfg)
    rows = []
    for _ in range(n_steps // every):
        run.step(every)
        rows.append(run.diag())
    h = {b: run.spectrum(b, e_max) for b in bins}
    run.close()
    return rows, h


def _figures(h, e_max):
    edges = np.linspace(0.0, e_max, h.size + 1)
    peak, _ = spectrum.peak_and_fwhm(h, edges)
    return peak, spectrum.width80(h, edges)


def _term_tol(ref_value, spread):
    if abs(ref_value) >= 1e-3:
        return 1e-3
    return 1e-3 * abs(ref_value) + 2.0 * spread + 1e-10


def _check_run(name, seed, rows, ref, spread, terms_per_run=True):
    """Per stored step: E_in, Gauss, balance (and, with terms_per_run, each
    term).  Returns the GPU's terms (fraction of E_in) per stored step."""
    out = []
    for i, (d, r) in enumerate(zip(rows, ref["series"])):
        e_in = r["E_in"]
        assert d["step"] == r["step"]
        assert d["E_in"] == pytest.approx(e_in, rel=1e-6)
        assert d["gauss_int"] == 0
        db = d["balance"] / e_in - r["balance"]
        assert abs(db) <= 1e-3, (name, seed, r["step"], "balance", db)
        g = {k: d[k] / e_in for k in TERMS}
        out.append(g)
        if terms_per_run:
            for k in TERMS:
                tol = _term_tol(r[k], spread[i][k])
                assert abs(g[k] - r[k]) <= tol, (name, seed, r["step"], k, g[k], r[k], tol)
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1w_whole_runs_match_the_oracle(precision):
    # 512 particles per cell per species, 8 seeds: budget and balance run by
    # run; the proton spectrum's peak and width as seed means
    refs = _refs("c1w")
    spread = _spread(refs)
    seeds = sorted(s for s, f in refs if not f)
    assert len(seeds) >= 8
    figs = {b: ([], [], [], []) for b in ("512", "4096")}
    for seed in seeds:
        ref = refs[(seed, False)]
        cfg = preset("c1w", precision=precision, seed=seed)
        rows, h = _gpu_run(cfg, ref["every"], ref["steps"], (512, 4096), ref["e_max_mev"])
        g = _check_run("c1w", seed, rows, ref, spread)
        worst = {k: max(abs(gi[k] - r[k]) for gi, r in zip(g, ref["series"])) for k in TERMS}
        print(f"[c1w {precision} seed {seed}] largest |GPU - oracle| (fraction of E_in):",
              {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
        for bins in ("512", "4096"):
            peak, width = _figures(h[int(bins)], ref["e_max_mev"])
            rp, rw = ref["spectrum"][bins]["peak_mev"], ref["spectrum"][bins]["width80_mev"]
            print(f"[c1w {precision} seed {seed} {bins} bins] peak {peak:.2f} (oracle {rp:.2f}) MeV, "
                  f"central-80% width {width:.2f} (oracle {rw:.2f}) MeV", flush=True)
            for lst, v in zip(figs[bins], (peak, rp, width, rw)):
                lst.append(v)
    for bins, (gp, op, gw, ow) in figs.items():
        gp, op, gw, ow = map(np.mean, (gp, op, gw, ow))
        print(f"[c1w {precision} {bins} bins] mean peak {gp:.2f} (oracle {op:.2f}) MeV, mean "
              f"central-80% width {gw:.2f} (oracle {ow:.2f}) MeV", flush=True)
        if bins == "512":  # (at 4,096 bins the peak is one spike of the bunch)
            assert abs(gp - op) <= 0.01 * op, (bins, gp, op)
        assert abs(gw - ow) <= 0.01 * ow, (bins, gw, ow)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_whole_runs_match_the_oracle(precision):
    # the small workload as specified (64 particles per cell per species),
    # 8 seeds: budget and balance run by run, the spectrum as seed means
    refs = _refs("c1")
    spread = _spread(refs)
    seeds = sorted(s for s, f in refs if not f)
    assert len(seeds) >= 8
    g_pk, g_w, o_pk, o_w, g_terms = [], [], [], [], []
    for seed in seeds:
        ref = refs[(seed, False)]
        cfg = preset("c1", precision=precision, seed=seed)
        rows, h = _gpu_run(cfg, ref["every"], ref["steps"], (512,), ref["e_max_mev"])
        g_terms.append(_check_run("c1", seed, rows, ref, spread, terms_per_run=False))
        peak, width = _figures(h[512], ref["e_max_mev"])
        g_pk.append(peak)
        g_w.append(width)
        o_pk.append(ref["spectrum"]["512"]["peak_mev"])
        o_w.append(ref["spectrum"]["512"]["width80_mev"])
    # every term, as the mean over the seeds, at every stored step
    worst = {k: 0.0 for k in TERMS}
    for i in range(len(spread)):
        for k in TERMS:
            gm = np.mean([g[i][k] for g in g_terms])
            om = np.mean([refs[(s, False)]["series"][i][k] for s in seeds])
            worst[k] = max(worst[k], abs(gm - om))
            tol = _term_tol(om, spread[i][k])
            assert abs(gm - om) <= tol, (i, k, gm, om)
    print(f"[c1 {precision}] largest |mean GPU - mean oracle| over {len(seeds)} seeds "
          "(fraction of E_in):", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    g_pk, g_w, o_pk, o_w = map(np.array, (g_pk, g_w, o_pk, o_w))
    print(f"[c1 {precision}] peak GPU {g_pk.round(1)} oracle {o_pk.round(1)} MeV; "
          f"central-80% width GPU {g_w.round(1)} oracle {o_w.round(1)} MeV", flush=True)
    assert abs(g_pk.mean() - o_pk.mean()) <= 0.01 * o_pk.mean()
    assert abs(g_w.mean() - o_w.mean()) <= 0.01 * o_w.mean()


def _c2_refs(rr):
    out = {}
    for f in sorted(glob.glob(os.path.join(GOLD, "c2_reference", f"rr{rr}_seed*.json"))):
        r = json.load(open(f))
        out[(r["seed"], bool(r.get("f32_start", False)))] = r
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("rr", [1, 0])
def test_c2_whole_runs_match_the_oracle(precision, rr):
    # the plain method at scale (LP a0 = 300, 12,000 cells, 4e5 particles,
    # 24,000 steps), RR on and off, the FP64 and FP32 paths, 3 seeds.  LP
    # heats the electrons chaotically: the oracle's runs differ by 1-2% of the
    # injected energy in single terms and by 30% in the spectral peak (which
    # jumps between bunch and tail), so only the balance can be held run by
    # run; terms and spectrum are compared as seed means within 1e-3 (1%)
    # plus twice the oracle's noise floor (its seed spread, or its response to
    # a float32-rounded start where measured, the largest from the pulse's
    # arrival at the foil on)
    refs = _c2_refs(rr)
    seeds = sorted(s for s, f in refs if not f)
    assert len(seeds) >= 3
    # the noise floor of a term: the largest of its per-step floors from the
    # pulse's arrival on (the spread of three seeds at one step can be small
    # by chance; the chaotic state's spread is not)
    spread = _spread(refs)
    arrive = next(i for i, r in enumerate(refs[(seeds[0], False)]["series"]) if r["step"] > 3200)
    for k in TERMS:
        late = max(row[k] for row in spread[arrive:])
        for row in spread[arrive:]:
            row[k] = late
    g_rows, g_spec, o_spec = [], [], []
    for seed in seeds:
        ref = refs[(seed, False)]
        cfg = preset("c2", precision=precision, seed=seed, rr=bool(rr))
        rows, h = _gpu_run(cfg, ref["every"], ref["steps"], (ref["bins"],), ref["e_max_mev"])
        g_rows.append(_check_run("c2", seed, rows, ref, spread, terms_per_run=False))
        g_spec.append(_figures(h[ref["bins"]], ref["e_max_mev"]))
        edges = np.linspace(0.0, ref["e_max_mev"], ref["bins"] + 1)
        oh = np.array(ref["hist"])
        o_spec.append((spectrum.peak_and_fwhm(oh, edges)[0], spectrum.width80(oh, edges)))
        print(f"[c2 rr={rr} {precision} seed {seed}] final balance GPU "
              f"{rows[-1]['balance'] / rows[-1]['E_in']:.2e} oracle {ref['series'][-1]['balance']:.2e}; "
              f"peak {g_spec[-1][0]:.1f} (oracle {o_spec[-1][0]:.1f}) MeV, central-80% width "
              f"{g_spec[-1][1]:.1f} (oracle {o_spec[-1][1]:.1f}) MeV", flush=True)
    worst = {k: 0.0 for k in TERMS}
    for i in range(len(spread)):
        for k in TERMS:
            gm = np.mean([g[i][k] for g in g_rows])
            om = np.mean([refs[(s, False)]["series"][i][k] for s in seeds])
            worst[k] = max(worst[k], abs(gm - om))
            tol = (1e-3 if abs(om) >= 1e-3 else 1e-3 * abs(om)) + 2.0 * spread[i][k] + 1e-10
            assert abs(gm - om) <= tol, (i, k, gm, om, tol)
    print(f"[c2 rr={rr} {precision}] largest |mean GPU - mean oracle| (fraction of E_in):",
          {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    g_spec, o_spec = np.array(g_spec), np.array(o_spec)
    floor = np.ptp(o_spec, axis=0) / o_spec.mean(axis=0)  # relative seed spread of peak, width
    for j, name in enumerate(("peak", "central-80% width")):
        rel = abs(g_spec[:, j].mean() / o_spec[:, j].mean() - 1.0)
        print(f"[c2 rr={rr} {precision}] mean {name}: GPU {g_spec[:, j].mean():.1f} oracle "
              f"{o_spec[:, j].mean():.1f} MeV ({100 * rel:.1f}%; seed spread {100 * floor[j]:.0f}%)",
              flush=True)
        assert rel <= max(0.01, 2.0 * floor[j])
