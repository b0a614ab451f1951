"""Double-precision CPU oracle for the radiation-reaction PIC hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU path: the two meet
only through the seeded inputs of the ``workloads`` package.

Contents and what they follow (Tamburini et al., "Radiation Reaction Effects
on Radiation Pressure Acceleration"):

* ``pusher``   - Boris push for the Lorentz force and the RR force of
                 Eq. (f_r), combined by the leapfrog splitting of
                 Eqs. (tot)-(estimgamma), Section 3; friction coefficient d of
                 Eq. (damping) and the lab-frame LL force of Eq. (3dLL).
* ``analytic`` - exact plane-wave orbits without RR, with the
                 non-derivative LL force and with the complete Eq. (3dLL)
                 (Section 2 and the single-electron test of Section 3),
                 uniform-field gyration and radiative cooling closed forms.
* ``rk4``      - classical Runge-Kutta single-electron integrator, the
                 comparator of the single-particle tests of Section 3.
* ``contract`` - the integer (fixed-point) current-deposition contract,
                 evaluated in float32 exactly as the GPU stores its state.
* ``pic``      - a plain 1D3V PIC loop (laser-foil problem of Section 4)
                 with Yee fields, linear weighting and charge-conserving
                 current deposition.
* ``pic2d``    - the same loop on a 2D grid (2D3V, Section 4's remark that
                 the pusher serves a multi-dimensional code unchanged):
                 2D Yee fields, bilinear weighting, Esirkepov's 2D
                 charge-conserving current.
* ``contract2d`` - the fixed-point deposition contract of the 2D path.
* ``rng``      - SplitMix64 counter-based generator for the quiet start.
* ``spectrum`` - ion energy spectrum, its peak and its full width at half
                 maximum.

Parity status per function is stated in each module header.
"""
from . import pusher, analytic, contract, contract2d, pic, pic2d, rng, spectrum  # noqa: F401
