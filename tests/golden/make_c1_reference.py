"""Write tests/golden/c1_reference.json: whole-run values of the oracle for the
small laser-foil workload (CP a0 = 200, n0 = 90, 1 wavelength foil at 8
wavelengths, 100 cells per wavelength, 64 particles per cell per species,
sin^2 pulse of 10 periods, RR on, 30 periods = 6000 steps) for seeds 0, 1, 2.

Stored per seed: the energy budget terms as fractions of the injected energy
at every 1000 steps, and the final proton spectrum's peak energy and full
width at half maximum (512 bins on [0, 1.05 x the largest proton energy of
seed 0]).  The seed-to-seed spread is the noise floor of whole-run checks.

Calls only the oracle and the input presets:
    python tests/golden/make_c1_reference.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pic, spectrum  # noqa: E402
from workloads import preset, periods_to_steps  # noqa: E402

KEYS = ("U_field", "K_e", "K_i", "E_rad", "E_out_left", "E_out_right", "E_esc", "balance")


def run(seed: int):
    cfg = preset("c1", seed=seed)
    sim = pic.Pic1D(cfg)
    n = periods_to_steps(cfg)
    series = []
    for k in range(n):
        sim.step()
        if (k + 1) % 1000 == 0:
            d = sim.diag()
            series.append(dict(step=k + 1, E_in=d["E_in"],
                               **{key: d[key] / d["E_in"] for key in KEYS}))
    E = spectrum.ion_energies_mev(sim.sp[1]["u"], cfg["mass_ratio"])
    return cfg, series, E, sim.sp[1]["w"]


def main():
    out = dict(cite="whole-run reference of the oracle (test infrastructure); workload c1",
               bins=512, seeds={})
    e_max = None
    for seed in (0, 1, 2):
        cfg, series, E, w = run(seed)
        if e_max is None:
            e_max = 1.05 * float(E.max())
        h, edges = spectrum.histogram(E, w, 512, e_max)
        peak, width = spectrum.peak_and_fwhm(h, edges)
        out["seeds"][str(seed)] = dict(series=series, peak_mev=peak, fwhm_mev=width,
                                      n_alive=[int(len(w))])
        print(seed, series[-1], peak, width, flush=True)
    out["e_max_mev"] = e_max
    out["steps"] = periods_to_steps(preset("c1"))
    json.dump(out, open(os.path.join(HERE, "c1_reference.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
