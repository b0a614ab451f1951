"""Write tests/golden/d1_reference.json: the 2D3V oracle on the small 2D
laser-foil workload (320 x 64 cells, LP a0 = 100 with a 0.6-wavelength
waist, 2 x 2 particles per cell per species, foil at 4 wavelengths) after
384 steps (6 periods: the pulse reaches the foil at 4), seeds 0-3: the
energy budget terms (Section 2 energy balance) as fractions of the injected
energy, the injected energy and the alive counts.  The spread over the
seeds is the noise floor of the budget comparison of single runs.

Calls only the oracle and the input presets:
    python tests/golden/make_d1_reference.py
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pic2d  # noqa: E402
from workloads import preset2d  # noqa: E402

KEYS = ("U_Ex", "U_Et", "U_B", "U_field", "K_e", "K_i", "E_rad", "E_out_left", "E_out_right",
        "E_esc", "balance")
STEPS = 384


def main():
    out = dict(cite="oracle reference (test infrastructure): 2D3V workload d1, Section 2 energy "
                    "balance", steps=STEPS, seeds={})
    for seed in range(4):
        sim = pic2d.Pic2D(preset2d("d1", seed=seed)).run(STEPS)
        d = sim.diag()
        out["seeds"][str(seed)] = dict(E_in=d["E_in"], n_alive=[int(x) for x in d["n_alive"]],
                                       **{k: d[k] / d["E_in"] for k in KEYS})
        print(seed, out["seeds"][str(seed)], flush=True)
    with open(os.path.join(HERE, "d1_reference.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
