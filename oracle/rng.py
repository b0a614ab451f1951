"""SplitMix64 as a counter-based generator (Steele, Lea and Flood, OOPSLA 2014).

TEST INFRASTRUCTURE ONLY (see package header).

The i-th output (i = 0, 1, ...) of a SplitMix64 stream whose state starts at
``seed`` is mix(seed + (i + 1) * 0x9E3779B97F4A7C15 mod 2^64), where mix is
the published finalizer (xor-shift 30, multiply 0xBF58476D1CE4E5B9,
xor-shift 27, multiply 0x94D049BB133111EB, xor-shift 31).  A uniform number
in [0, 1) with 24 random bits is (output >> 40) * 2^-24, exact in float32.

Pin: seed 0 gives 0xE220A8397B1DCDAF as its first output (the published
known answer); tests also check uniformity of the 24-bit draws.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, index):
    """Outputs number ``index`` (array of non-negative ints) of the stream
    seeded with ``seed``; returns uint64 array."""
    i = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (i + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform24(seed: int, index):
    """Uniform draws in [0, 1) with 24 bits, as float64 holding float32 values."""
    return (splitmix64(seed, index) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
