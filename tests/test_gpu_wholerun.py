"""Whole runs at the plain-method scale (12,000 cells, 4e5 particles, 60
periods) and at the precision-form scale (20,000 cells, 1e7 particles, 80
periods): the FP32 path (compensated RR) against the plain FP64 path.

The oracle cannot finish runs this long (1e10 to 3e11 FP64 pushes); the
FP64 GPU path stands in for it, itself checked against the oracle on whole
small runs and on short laser-foil runs.  Linear polarisation heats the
electrons chaotically: single runs that differ only in the quiet-start
jitter seed differ by about 1% of the injected energy in the radiated and
field energies, and their ion-spectrum peaks jump between the bunch and the
tail.  A single FP32 run therefore cannot be held to 1e-3 of a single FP64
run; the comparison is between ensembles of runs (8 at the smaller scale, 4 at
the larger):
* every energy term (fraction of the injected energy): |mean32 - mean64|
  <= 1e-3 + 3 standard errors of the difference;
* the energy balance of every run within 1e-3 of the injected energy, and
  FP32 against FP64 within 1e-3 (conservation is not chaotic);
* the ion spectrum's peak and width: |mean32 - mean64| <= 1% or 3 standard
  errors (at least one bin for the width)."""
import numpy as np
import pytest

from oracle import spectrum
from workloads import periods_to_steps, preset

pytestmark = pytest.mark.gpu

DEAD = np.iinfo(np.int32).min
KEYS = ("U_field", "K_e", "K_i", "E_rad", "E_out_left", "E_out_right", "E_esc")
BINS = 512
SEEDS = {"c2": 8, "c3": 4}  # runs per ensemble: the small runs are cheap and noisier


@pytest.fixture(autouse=True)
def _announce(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def _ensemble(base, precision, e_max=None):
    from paper_1008_1685_amd import Run

    rows, shape = [], []
    for seed in range(SEEDS[base["name"]]):
        cfg = dict(base, precision=precision, rr_compensated=True, seed=seed)
        run = Run(cfg)
        run.step(periods_to_steps(cfg))
        d = run.diag()
        assert d["gauss_int"] == 0 and not d["nonfinite"]
        assert abs(d["balance"]) <= 1e-3 * d["E_in"]
        if e_max is None:
            ions = run.get_particles(1, 0, run.get_info()["capacity"], keys=("cell", "ux", "uy", "uz"))
            alive = ions["cell"] != DEAD
            u = np.stack([ions[k][alive] for k in ("ux", "uy", "uz")], 1)
            e_max = 1.05 * float(spectrum.ion_energies_mev(u, cfg["mass_ratio"]).max())
        h = run.spectrum(BINS, e_max)
        run.close()
        rows.append([d[k] / d["E_in"] for k in KEYS] + [d["balance"] / d["E_in"], d["E_in"]])
        shape.append(spectrum.peak_and_fwhm(h, np.linspace(0.0, e_max, BINS + 1)))
    return np.array(rows), np.array(shape), e_max


def _se(a, b):
    return np.sqrt(a.var(0, ddof=1) / len(a) + b.var(0, ddof=1) / len(b))


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_fp32_whole_runs_match_the_fp64_path(name):
    base = preset(name)
    r64, s64, e_max = _ensemble(base, "fp64")
    r32, s32, _ = _ensemble(base, "fp32", e_max)
    np.testing.assert_allclose(r32[:, -1], r64[:, -1], rtol=1e-6)  # injected energy
    n = len(KEYS)
    diff = r32[:, :n].mean(0) - r64[:, :n].mean(0)
    se = _se(r32[:, :n], r64[:, :n])
    print(f"[{name}] fp32 - fp64 (fraction of E_in):", dict(zip(KEYS, np.round(diff, 5))),
          "3 SE:", dict(zip(KEYS, np.round(3 * se, 5))), flush=True)
    for k, dk, sk in zip(KEYS, diff, se):
        assert abs(dk) <= 1e-3 + 3 * sk, (k, dk, sk)
    assert abs(r32[:, n].mean() - r64[:, n].mean()) <= 1e-3
    dpk, dfw = s32.mean(0) - s64.mean(0)
    spk, sfw = _se(s32, s64)
    print(f"[{name}] ion peak fp32 {s32[:, 0].round(1)} fp64 {s64[:, 0].round(1)} MeV; "
          f"fwhm fp32 {s32[:, 1].round(2)} fp64 {s64[:, 1].round(2)} MeV", flush=True)
    assert abs(dpk) <= max(0.01 * s64[:, 0].mean(), 3 * spk)
    assert abs(dfw) <= max(0.01 * s64[:, 1].mean(), 3 * sfw, e_max / BINS)
