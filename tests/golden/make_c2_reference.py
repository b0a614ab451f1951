"""Write tests/golden/c2_reference/rr{0,1}_seed{k}.json: whole-run values of
the oracle for the plain-method workload at scale (LP a0 = 300, 200 cells per
wavelength, 60 wavelength box (12,000 cells), foil n0 = 100, 1 wavelength at
8 wavelengths, 1,000 particles per cell per species (4e5 particles), sin^2
pulse of 10 periods, 60 periods = 24,000 steps), with radiation reaction on
and off, for seeds 0, 1, 2.

Stored per run:
* the energy budget (Section 2 energy balance: field, kinetic, radiated,
  boundary fluxes, escaped) every 1,000 steps as fractions of the injected
  energy, with the injected energy itself and the alive counts;
* the final proton spectrum (Section 4 spectra, protons per MeV) in 512 bins
  on [0, e_max), e_max = 1.05 x the run's own largest proton energy, with its
  peak and full width at half maximum;
* the oracle's own wall time.

With --f32-start the run starts from the same quiet start with every
offset rounded to float32 (as an FP32 run stores it): the oracle's own
response to a perturbation of the size the FP32 storage brings in, which
bounds how closely any whole run can follow the reference
(rr{rr}_seed{k}_f32start.json).

A run takes about two hours of one core (numpy), so each case is a process of
its own:
    python tests/golden/make_c2_reference.py --rr 1 --seed 0
(no arguments: every case, one after the other).  Calls only the oracle and
the input presets.
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
BINS = 512
EVERY = 1000
SEEDS = (0, 1, 2)


def out_path(rr: int, seed: int, f32_start: bool = False) -> str:
    tail = "_f32start" if f32_start else ""
    return os.path.join(HERE, "c2_reference", f"rr{rr}_seed{seed}{tail}.json")


def run(rr: int, seed: int, f32_start: bool = False) -> None:
    cfg = preset("c2", rr=bool(rr), seed=seed)
    sim = pic.Pic1D(cfg)
    if f32_start:
        for s in range(2):
            xi = sim.sp[s]["xi"]
            c = np.floor(xi)
            sim.sp[s]["xi"] = c + (xi - c).astype(np.float32).astype(np.float64)
    n = periods_to_steps(cfg)
    series = []
    t0 = time.perf_counter()
    pushes = 0
    for k in range(n):
        pushes += sim.sp[0]["xi"].size + sim.sp[1]["xi"].size
        sim.step()
        if (k + 1) % EVERY == 0:
            d = sim.diag()
            series.append(dict(step=k + 1, E_in=d["E_in"], n_alive=list(d["n_alive"]),
                               gauss=d["gauss"], **{key: d[key] / d["E_in"] for key in KEYS}))
            print(f"rr={rr} seed={seed} step {k + 1}/{n} balance {series[-1]['balance']:.2e} "
                  f"E_rad {series[-1]['E_rad']:.4f} {time.perf_counter() - t0:.0f} s", flush=True)
    wall = time.perf_counter() - t0
    E = spectrum.ion_energies_mev(sim.sp[1]["u"], cfg["mass_ratio"])
    w = sim.sp[1]["w"]
    e_max = 1.05 * float(E.max())
    h, edges = spectrum.histogram(E, w, BINS, e_max)
    peak, width = spectrum.peak_and_fwhm(h, edges)
    out = dict(cite="whole-run reference of the oracle (test infrastructure); workload c2, "
                    "Section 2 energy balance and Section 4 proton spectra",
               workload="c2", rr=rr, seed=seed, f32_start=f32_start, steps=n, every=EVERY, series=series,
               bins=BINS, e_max_mev=e_max, hist=[float(x) for x in h], peak_mev=peak,
               fwhm_mev=width, oracle_wall_s=wall, oracle_pushes=pushes)
    os.makedirs(os.path.dirname(out_path(rr, seed, f32_start)), exist_ok=True)
    with open(out_path(rr, seed, f32_start), "w") as f:
        json.dump(out, f, indent=0)
    print(f"rr={rr} seed={seed} done: peak {peak:.2f} MeV fwhm {width:.2f} MeV, {wall:.0f} s",
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rr", type=int, choices=(0, 1))
    ap.add_argument("--seed", type=int)
    ap.add_argument("--f32-start", action="store_true")
    a = ap.parse_args()
    cases = [(rr, s) for rr in (1, 0) for s in SEEDS]
    if a.rr is not None or a.seed is not None:
        cases = [(rr, s) for rr, s in cases
                 if (a.rr is None or rr == a.rr) and (a.seed is None or s == a.seed)]
    for rr, s in cases:
        run(rr, s, a.f32_start)


if __name__ == "__main__":
    main()
