"""Pins of the oracle's SplitMix64 generator and spectrum peak/width helpers."""
import numpy as np
import pytest

from oracle import rng, spectrum


def test_splitmix64_published_known_answer():
    # first output of SplitMix64 seeded with 0
    assert int(rng.splitmix64(0, 0)) == 0xE220A8397B1DCDAF


def test_splitmix64_stream_is_counter_based():
    # output i of seed s equals output 0 of seed s + i * golden (mod 2^64)
    for i in (1, 7, 12345):
        s = (5 + i * 0x9E3779B97F4A7C15) % (1 << 64)
        assert int(rng.splitmix64(5, i)) == int(rng.splitmix64(s, 0))


def test_uniform24_is_uniform():
    u = rng.uniform24(42, np.arange(200000))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))
    h, _ = np.histogram(u, bins=50, range=(0, 1))
    chi2 = np.sum((h - 4000.0) ** 2 / 4000.0)
    assert chi2 < 90.0  # 49 degrees of freedom, p ~ 5e-4


def test_peak_and_fwhm_of_a_gaussian():
    r = np.random.default_rng(0)
    mu, sig = 40.0, 7.0
    E = r.normal(mu, sig, size=2_000_000)
    h, edges = spectrum.histogram(E, np.ones_like(E), 400, 250.0)
    peak, width = spectrum.peak_and_fwhm(h, edges)
    # maximum of E exp(-(E - mu)^2 / (2 sigma^2))
    assert peak == pytest.approx(0.5 * (mu + np.sqrt(mu * mu + 4 * sig * sig)), abs=0.3)
    assert abs(peak - mu) > 0.3  # the energy weighting is resolved
    assert width == pytest.approx(2 * np.sqrt(2 * np.log(2)) * sig, rel=0.02)


def test_ion_energy_units():
    # a proton with gamma = 2 carries m_p c^2 = 1836 * 0.511 MeV of kinetic energy
    u = np.array([[np.sqrt(3.0), 0, 0]])
    assert spectrum.ion_energies_mev(u, 1836.0)[0] == pytest.approx(1836 * 0.51099895)


def test_central_range_of_uniform_bins_is_exact():
    # 10 bins of 2 MeV; content only in bins 2..6 (E in [4, 14)), evenly:
    # 10% of it lies below 5 MeV, 90% below 13 MeV
    edges = np.linspace(0.0, 20.0, 11)
    h = np.zeros(10)
    h[2:7] = 3.0
    lo, hi = spectrum.central_range(h, edges)
    assert lo == pytest.approx(5.0, abs=1e-12) and hi == pytest.approx(13.0, abs=1e-12)
    assert spectrum.width80(h, edges) == pytest.approx(8.0, abs=1e-12)
    # an asymmetric case: content 1, 3 in bins [0, 2), [2, 4): the 10th
    # percentile is 0.4 of the way through bin 0, the 90th 0.8666.. through bin 1
    lo, hi = spectrum.central_range(np.array([1.0, 3.0]), np.array([0.0, 2.0, 4.0]))
    assert lo == pytest.approx(0.8) and hi == pytest.approx(2.0 + 2.0 * (3.6 - 1.0) / 3.0)


def test_central_range_of_a_gaussian():
    r = np.random.default_rng(1)
    mu, sig = 300.0, 12.0
    E = r.normal(mu, sig, size=2_000_000)
    h, edges = spectrum.histogram(E, np.ones_like(E), 2048, 600.0)
    lo, hi = spectrum.central_range(h, edges)
    z90 = 1.2815515655446004  # standard normal 90th percentile
    assert lo == pytest.approx(mu - z90 * sig, abs=0.05)
    assert hi == pytest.approx(mu + z90 * sig, abs=0.05)
    # weights count, not particles: doubling half the sample's weights moves the range
    w = np.where(E > mu, 2.0, 1.0)
    h2, _ = spectrum.histogram(E, w, 2048, 600.0)
    assert spectrum.central_range(h2, edges)[0] > lo + 1.0
