"""Workload presets: raw physical and numerical parameters only.

Normalisation follows the paper's Section 2 conventions: time in 1/omega,
length in c/omega, momentum in m c, fields in m omega c/|e|, densities in
the critical density n_c.  Presets are written in laser wavelengths and
periods; each consumer converts them (one wavelength = one period = 2 pi).

Laser envelope: a sin^2 rise of ``t_rise`` periods, a flat top of
``t_flat`` periods and a sin^2 fall of ``t_fall`` periods.  A rise and fall
of 5 periods with no plateau is exactly sin^2(pi t / 10 T), the "sin^2
envelope lasting 10 periods"; the paper's own pulse (Section 4) is
rise 1, plateau 5, fall 1.

Circular polarisation at amplitude ``a0`` carries the same intensity as
linear polarisation at ``a0`` (each transverse component has a0/sqrt 2),
because the paper quotes one a0 for one intensity for both polarisations.
"""
from __future__ import annotations

import copy

_BASE = dict(
    precision="fp32",        # particle / field storage: "fp32" or "fp64"
    lambda_um=0.8,           # laser wavelength in micrometres (sets the RR coefficient)
    cells_per_lambda=100,
    box_lambda=20.0,
    cfl=0.5,                 # dt = cfl * dx
    pol="CP",                # "LP" or "CP"
    a0=200.0,
    t_rise=5.0, t_flat=0.0, t_fall=5.0,   # periods
    n0=90.0,                 # foil density in n_c
    x_foil=8.0,              # foil front in wavelengths
    thickness=1.0,           # foil thickness in wavelengths
    ppc=64,                  # particles per cell per species
    mass_ratio=1836.0,       # proton / electron mass
    rr=True,                 # radiation reaction on electrons
    rr_compensated=True,     # compensated accumulation of the RR increment (fp32 only)
    seed=0,
    jitter=0.5,              # quiet-start jitter as a fraction of the particle spacing
    periods=30.0,            # run length in laser periods
    sort_interval=16,        # steps between cell sorts
)

PRESETS = {
    # small plain run that the FP64 oracle finishes
    "c1": dict(_BASE),
    # the small run at 512 particles per cell per species (102,400 particles):
    # enough protons to resolve the spectrum's peak and width in whole-run
    # comparisons (the oracle finishes it in minutes)
    "c1w": dict(_BASE, ppc=512),
    # plain method at scale: LP a0=300, 12,000 cells, 4e5 particles
    "c2": dict(_BASE, cells_per_lambda=200, box_lambda=60.0, pol="LP", a0=300.0,
               n0=100.0, ppc=1000, periods=60.0, precision="fp64"),
    # precision form: 20,000 cells, 1e7 particles (LP or CP, a0 200 or 500)
    # (the cell sort every 32 steps: the push is as fast as with 16, the sort
    # costs half as much per step)
    "c3": dict(_BASE, cells_per_lambda=200, box_lambda=100.0, pol="LP", a0=500.0,
               n0=100.0, ppc=25000, periods=80.0, sort_interval=64),
    # stress case: 80,000 cells, 2e8 particles, RR-dominated
    "c5": dict(_BASE, cells_per_lambda=400, box_lambda=200.0, pol="LP", a0=800.0,
               n0=100.0, thickness=2.0, ppc=125000, periods=150.0, sort_interval=32),
    # the paper's own pulse and foil (Section 4): a0=328, n0=100, 1 wavelength
    "paper": dict(_BASE, cells_per_lambda=200, box_lambda=40.0, pol="LP", a0=328.0,
                  n0=100.0, x_foil=14.0, t_rise=1.0, t_flat=5.0, t_fall=1.0,
                  ppc=1000, periods=46.0),
}


def preset(name: str, **overrides) -> dict:
    """Return a copy of preset ``name`` with ``overrides`` applied."""
    if name not in PRESETS:
        raise KeyError(f"unknown preset {name!r}; known: {sorted(PRESETS)}")
    cfg = copy.deepcopy(PRESETS[name])
    for k, v in overrides.items():
        if k not in cfg:
            raise KeyError(f"unknown parameter {k!r}")
        cfg[k] = v
    cfg["name"] = name
    return cfg


def periods_to_steps(cfg: dict) -> int:
    """Steps in ``cfg['periods']`` laser periods: dt = cfl*dx, dx = lambda/cpl."""
    return int(round(cfg["periods"] * cfg["cells_per_lambda"] / cfg["cfl"]))


# ---------------------------------------------------------------- 2D3V
# The same laser-foil problem on a 2D grid, periodic in y: box_x by box_y
# wavelengths, ppc_x * ppc_y particles per cell per species on a lattice,
# laser with a Gaussian transverse profile of 1/e half-width ``waist``
# wavelengths (0: plane wave).
_BASE_2D = dict(
    precision="fp32",
    lambda_um=0.8,
    cells_per_lambda=32,
    box_x=10.0, box_y=2.0,
    cfl=0.5,
    pol="LP",
    a0=100.0,
    waist=0.6,
    t_rise=3.0, t_flat=0.0, t_fall=3.0,
    n0=90.0,
    x_foil=4.0,
    thickness=1.0,
    ppc_x=2, ppc_y=2,
    mass_ratio=1836.0,
    rr=True,
    rr_compensated=True,
    seed=0,
    jitter=0.5,
    periods=8.0,
    sort_interval=16,
    field_kernel="auto",  # HIP field advance: "auto", "tiles" or "strips" (the oracle has one)
)

PRESETS_2D = {
    # small run that the FP64 oracle finishes: 320 x 64 cells, 16,384 particles
    "d1": dict(_BASE_2D),
    # the 2D counterpart of the precision-form workload: 2,560 x 1,024 cells,
    # 8.4e6 particles (64 per cell per species), LP a0=500, 4-wavelength waist
    "d2": dict(_BASE_2D, cells_per_lambda=64, box_x=40.0, box_y=16.0, a0=500.0, waist=4.0,
               t_rise=5.0, t_fall=5.0, n0=100.0, x_foil=10.0, ppc_x=8, ppc_y=8,
               periods=20.0, sort_interval=24),
}


def preset2d(name: str, **overrides) -> dict:
    """Return a copy of 2D preset ``name`` with ``overrides`` applied."""
    if name not in PRESETS_2D:
        raise KeyError(f"unknown 2D preset {name!r}; known: {sorted(PRESETS_2D)}")
    cfg = copy.deepcopy(PRESETS_2D[name])
    for k, v in overrides.items():
        if k not in cfg:
            raise KeyError(f"unknown parameter {k!r}")
        cfg[k] = v
    cfg["name"] = name
    return cfg
