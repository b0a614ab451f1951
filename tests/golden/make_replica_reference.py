"""Write tests/golden/replica_reference.json: the oracle on a reduced copy of
the paper's own LP run (Section 4: a0 = 328, n0 = 100 n_c, 1 wavelength foil
at 14 wavelengths, 1-cycle sin^2 rise and fall around a 5-cycle plateau, RR
on), at 100 cells per wavelength and 64 particles per cell per species in a
40-wavelength box, up to t_p = 12 periods after the pulse front reaches the
foil; seeds 0, 1, 2.

Stored per seed:
* the absorption curve (Section 4's fractional energy absorption against
  time): electron and ion kinetic energy, radiated energy and the balance as
  fractions of the injected energy at every period t_p = 0 .. 12;
* the friction coefficient d of Eq. (damping) of the electrons at
  t_p = 1.7 periods: its maximum and weighted mean;
* the proton spectrum at t_p = 12: peak (maximum of E f(E)) and the width of
  the central 80%, in 512 bins on [0, 1.05 x the run's largest energy).

Calls only the oracle and the input presets:
    python tests/golden/make_replica_reference.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pic, pusher, spectrum  # noqa: E402
from workloads import preset  # noqa: E402

OVERRIDES = dict(cells_per_lambda=100, ppc=64, box_lambda=40.0, periods=26.0)


def config(seed: int) -> dict:
    return preset("paper", seed=seed, **OVERRIDES)


def run(seed: int) -> dict:
    cfg = config(seed)
    sim = pic.Pic1D(cfg)
    spp = cfg["cells_per_lambda"] / cfg["cfl"]
    curve, fr = [], None
    done = 0
    for tp in sorted(set(np.arange(0.0, 13.0)) | {1.7}):
        n = int(round((cfg["x_foil"] + tp) * spp)) - done
        sim.run(n)
        done += n
        if tp == 1.7:
            e = sim.sp[0]
            E, B = sim.gather(e["xi"])
            d = pusher.damping(E, B, e["u"], sim.eps)[1]
            fr = dict(step=done, max=float(d.max()), mean=float(np.sum(e["w"] * d) / np.sum(e["w"])))
            continue
        dg = sim.diag()
        curve.append(dict(t_p=float(tp), step=done, E_in=dg["E_in"],
                          **{k: dg[k] / dg["E_in"] for k in ("K_e", "K_i", "E_rad", "U_field",
                                                             "balance")}))
    E = spectrum.ion_energies_mev(sim.sp[1]["u"], cfg["mass_ratio"])
    e_max = 1.05 * float(E.max())
    h, edges = spectrum.histogram(E, sim.sp[1]["w"], 512, e_max)
    peak, _ = spectrum.peak_and_fwhm(h, edges)
    print(seed, curve[-1], fr, peak, flush=True)
    return dict(curve=curve, friction=fr, e_max_mev=e_max, peak_mev=peak,
                width80_mev=spectrum.width80(h, edges))


def main():
    out = dict(cite="oracle reference (test infrastructure) for a reduced copy of the paper's LP "
                    "laser-foil run, Section 4", overrides=OVERRIDES,
               seeds={str(s): run(s) for s in (0, 1, 2)})
    with open(os.path.join(HERE, "replica_reference.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
