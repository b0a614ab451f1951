"""Write tests/golden/c1_reference/{workload}_seed{k}[_f32start].json:
whole-run values of the oracle for the small laser-foil workload (CP
a0 = 200, n0 = 90, 1 wavelength foil at 8 wavelengths, 100 cells per
wavelength, sin^2 pulse of 10 periods, RR on, 30 periods = 6,000 steps) at
64 particles per cell per species ("c1", 12,800 particles) and at 512 ("c1w",
102,400 particles), seeds 0-7 each.

Stored per run:
* the energy budget (Section 2 energy balance) every 500 steps as fractions
  of the injected energy, with the injected energy and the alive counts;
* the final proton spectrum (Section 4 spectra) on [0, e_max), e_max = 1.05 x
  the run's own largest proton energy: in 512 bins its histogram, and in 512
  and 4,096 bins its peak (maximum of E f(E)), full width at half maximum,
  10th and 90th percentiles and the width of the central 80%.

With --f32-start the run starts from the same quiet start with every offset
rounded to float32, as an FP32 run stores it: the oracle's own response to a
perturbation of the size FP32 storage brings in.  The spread of these pairs
and of the seeds is the noise floor of whole-run comparisons.

    python tests/golden/make_c1_reference.py --workload c1 --seed 0 [--f32-start]
    python tests/golden/make_c1_reference.py            # every case in turn

Calls only the oracle and the input presets.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pic, spectrum  # noqa: E402
from workloads import periods_to_steps, preset  # noqa: E402

KEYS = ("U_Ex", "U_Et", "U_B", "U_field", "K_e", "K_i", "E_rad", "E_out_left",
        "E_out_right", "E_esc", "balance")
EVERY = 500
CASES = ([("c1", s, False) for s in range(8)] + [("c1", s, True) for s in range(3)]
         + [("c1w", s, False) for s in range(8)] + [("c1w", 0, True)])


def out_path(workload: str, seed: int, f32_start: bool) -> str:
    tail = "_f32start" if f32_start else ""
    return os.path.join(HERE, "c1_reference", f"{workload}_seed{seed}{tail}.json")


def figures(E, w, bins, e_max):
    h, edges = spectrum.histogram(E, w, bins, e_max)
    peak, fwhm = spectrum.peak_and_fwhm(h, edges)
    q10, q90 = spectrum.central_range(h, edges)
    return h, dict(peak_mev=peak, fwhm_mev=fwhm, q10_mev=q10, q90_mev=q90, width80_mev=q90 - q10)


def run(workload: str, seed: int, f32_start: bool) -> None:
    cfg = preset(workload, seed=seed)
    sim = pic.Pic1D(cfg)
    if f32_start:
        for s in range(2):
            xi = sim.sp[s]["xi"]
            c = np.floor(xi)
            sim.sp[s]["xi"] = c + (xi - c).astype(np.float32).astype(np.float64)
    n = periods_to_steps(cfg)
    series = []
    t0 = time.perf_counter()
    for k in range(n):
        sim.step()
        if (k + 1) % EVERY == 0:
            d = sim.diag()
            series.append(dict(step=k + 1, E_in=d["E_in"], n_alive=list(d["n_alive"]),
                               **{key: d[key] / d["E_in"] for key in KEYS}))
    wall = time.perf_counter() - t0
    E = spectrum.ion_energies_mev(sim.sp[1]["u"], cfg["mass_ratio"])
    w = sim.sp[1]["w"]
    e_max = 1.05 * float(E.max())
    h512, f512 = figures(E, w, 512, e_max)
    _, f4096 = figures(E, w, 4096, e_max)
    out = dict(cite="whole-run reference of the oracle (test infrastructure); Section 2 energy "
                    "balance and Section 4 proton spectra",
               workload=workload, seed=seed, f32_start=f32_start, steps=n, every=EVERY,
               series=series, e_max_mev=e_max, hist512=[float(x) for x in h512],
               spectrum={"512": f512, "4096": f4096}, oracle_wall_s=wall)
    os.makedirs(os.path.dirname(out_path(workload, seed, f32_start)), exist_ok=True)
    with open(out_path(workload, seed, f32_start), "w") as f:
        json.dump(out, f, indent=0)
    print(workload, seed, f32_start, f512, f4096, f"{wall:.0f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("c1", "c1w"))
    ap.add_argument("--seed", type=int)
    ap.add_argument("--f32-start", action="store_true")
    a = ap.parse_args()
    if a.workload is None:
        for case in CASES:
            run(*case)
    else:
        run(a.workload, a.seed if a.seed is not None else 0, a.f32_start)


if __name__ == "__main__":
    main()
