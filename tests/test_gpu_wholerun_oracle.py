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
  1e-3 of it; a smaller term within 1e-3 of its own size plus the oracle's
  measured seed-to-seed spread of that term at that step (plus 1e-12 of the
  injected energy, below which a term is rounding noise: RR before the pulse
  arrives, say, where FP32 partial sums round 1e-83 to zero).  The small
  terms (the radiated energy of these circularly polarised runs, light
  leaving at the far end, escaped particles) vary by 5-50% between seeds;
* the proton spectrum's peak (maximum of E f(E)) and width (the energy range
  of the central 80% of the protons) within 1%.
At 512 particles per cell (c1w) every run is held to these bounds, except
the spectral width, which is held as the mean over eight seeds: single runs
move it by 0.4-1% when only their start is rounded to float32 (the oracle's
own response, measured), the peak by under 0.1%.  At 64 particles per cell
(c1, the small workload as specified) single runs respond to that rounding by
up to 1.4% in peak and width and by about 1e-3 of the injected energy in
single terms, so terms and spectrum are compared as means over eight seeds;
the balance is still held run by run.
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
    """Per stored step and term: the oracle's seed-to-seed spread (max - min
    over the seeds; fraction of E_in)."""
    runs = [r for (s, f), r in refs.items() if not f]
    n = len(runs[0]["series"])
    return [{k: float(np.ptp([r["series"][i][k] for r in runs])) for k in TERMS} for i in range(n)]


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
    return 1e-3 * abs(ref_value) + spread + 1e-12


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
    # 512 particles per cell per species, 8 seeds: budget, balance and the
    # proton spectrum's peak run by run, its width as the seed mean
    refs = _refs("c1w")
    spread = _spread(refs)
    seeds = sorted(s for s, f in refs if not f)
    assert len(seeds) >= 8
    widths = {b: ([], []) for b in ("512", "4096")}
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
            assert abs(peak - rp) <= 0.01 * rp, (seed, bins, peak, rp)
            widths[bins][0].append(width)
            widths[bins][1].append(rw)
    for bins, (gw, ow) in widths.items():
        gw, ow = np.mean(gw), np.mean(ow)
        print(f"[c1w {precision} {bins} bins] mean central-80% width {gw:.2f} (oracle {ow:.2f}) MeV",
              flush=True)
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
            # (a mean over n seeds: the spread of single runs over sqrt(n))
            tol = _term_tol(om, spread[i][k] / np.sqrt(len(seeds)))
            assert abs(gm - om) <= tol, (i, k, gm, om)
    print(f"[c1 {precision}] largest |mean GPU - mean oracle| over {len(seeds)} seeds "
          "(fraction of E_in):", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    g_pk, g_w, o_pk, o_w = map(np.array, (g_pk, g_w, o_pk, o_w))
    print(f"[c1 {precision}] peak GPU {g_pk.round(1)} oracle {o_pk.round(1)} MeV; "
          f"central-80% width GPU {g_w.round(1)} oracle {o_w.round(1)} MeV", flush=True)
    assert abs(g_pk.mean() - o_pk.mean()) <= 0.01 * o_pk.mean()
    assert abs(g_w.mean() - o_w.mean()) <= 0.01 * o_w.mean()
