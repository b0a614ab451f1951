"""Ion energy spectrum and its peak and width (Section 4 spectra, f(E) =
protons per unit energy; the paper compares spectra by their peak energy and
their energy spread, the width of the spectrum).

TEST INFRASTRUCTURE ONLY (see package header).

Reading: kinetic energy per proton E = (gamma - 1) M m_e c^2 with
m_e c^2 = 0.51099895 MeV; weighted histogram f(E) on [0, e_max].  The
spectra of Section 4 carry a low-energy tail next to the quasi-monoenergetic
bunch, and the plain mode can jump between them; the "peak" is therefore the
bunch that carries the most energy: the maximum of E f(E), refined by a
parabola through the three bins around it.
Width: the energy range that holds the central 80% of the protons (the 10th
to the 90th percentile of f, read off the cumulative histogram with linear
interpolation inside a bin).  The full width at half maximum of f(E) around
the peak is kept as a second figure; it is not a robust width here: the 1D
bunch is only a few bins wide and spiky, and its FWHM changes by tens of
percent when the initial offsets are rounded to float32.
Pins: sampled Gaussians, whose E f(E) peaks at
(mu + sqrt(mu^2 + 4 sigma^2)) / 2, whose FWHM is 2 sqrt(2 ln 2) sigma and
whose central 80% spans 2 z_0.9 sigma; a histogram of uniform bins, whose
percentiles are exact.
"""
from __future__ import annotations

import numpy as np

MEC2_MEV = 0.51099895


def ion_energies_mev(u, mass_ratio):
    u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    return (np.sqrt(1.0 + np.sum(u * u, axis=1)) - 1.0) * mass_ratio * MEC2_MEV


def histogram(E, w, bins, e_max):
    h, edges = np.histogram(E, bins=bins, range=(0.0, e_max), weights=w)
    return h / (edges[1] - edges[0]), edges


def peak_and_fwhm(h, edges):
    """(peak energy, FWHM) of histogram density h with bin edges ``edges``."""
    h = np.asarray(h, dtype=np.float64)
    centers = 0.5 * (edges[:-1] + edges[1:])
    de = edges[1] - edges[0]
    he = h * centers
    k = int(np.argmax(he))
    peak = centers[k]
    if 0 < k < h.size - 1:
        y0, y1, y2 = he[k - 1], he[k], he[k + 1]
        den = y0 - 2.0 * y1 + y2
        if den != 0.0:
            peak += 0.5 * de * (y0 - y2) / den
    half = 0.5 * h[k]
    i = k
    while i > 0 and h[i - 1] >= half:
        i -= 1
    if i > 0:
        left = centers[i - 1] + de * (half - h[i - 1]) / (h[i] - h[i - 1])
    else:
        left = centers[0]
    j = k
    while j < h.size - 1 and h[j + 1] >= half:
        j += 1
    if j < h.size - 1:
        right = centers[j] + de * (h[j] - half) / (h[j] - h[j + 1])
    else:
        right = centers[-1]
    return float(peak), float(right - left)


def central_range(h, edges, lo=0.1, hi=0.9):
    """(E_lo, E_hi): the energies below which fractions lo and hi of the
    histogram's content lie, interpolated linearly inside a bin (the
    content of a bin taken as spread evenly over it)."""
    h = np.asarray(h, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.float64)
    cum = np.concatenate([[0.0], np.cumsum(h * np.diff(edges))])
    total = cum[-1]

    def at(q):
        target = q * total
        k = int(np.searchsorted(cum, target, side="left"))
        k = min(max(k, 1), h.size)
        inside = cum[k] - cum[k - 1]
        frac = (target - cum[k - 1]) / inside if inside > 0 else 0.0
        return float(edges[k - 1] + frac * (edges[k] - edges[k - 1]))

    return at(lo), at(hi)


def width80(h, edges):
    """Energy range of the central 80% of the protons."""
    a, b = central_range(h, edges, 0.1, 0.9)
    return b - a
