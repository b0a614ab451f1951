"""Pins of the integer deposition contract: exact discrete continuity and
Gauss's law, and agreement with the double-precision deposit."""
import numpy as np
import pytest

from oracle import contract, pic
from workloads import preset, random_particles

F32 = np.float32


def _div(J):
    # (J[h = i + 1] - J[h = i]) on nodes i = -1 .. n + 1 (index i + 1)
    n2 = J.size
    d = np.zeros(n2 + 1, dtype=J.dtype)
    d[:n2] += J
    d[1:] -= J
    return d


def test_continuity_is_exact_brute_force():
    # every (cell, offset) start on a 4-cell grid, displacements of both signs
    offs = np.array([0.0, 1e-7, 0.25, 0.4999999, 0.5, 0.75, 0.9999999], dtype=F32)
    disp = np.array([-0.4999, -0.3, -1e-6, 0.0, 1e-6, 0.3, 0.4999], dtype=F32)
    cells, o0, vx = np.meshgrid(np.arange(4), offs, disp, indexing="ij")
    cells, o0, vx = cells.ravel(), o0.ravel(), vx.ravel()
    n = 6
    # choose ux so that vx * cfl gives the wanted displacement (cfl = 0.5)
    ux = (2.0 * vx / np.sqrt(np.maximum(1 - 4 * vx * vx, 1e-12))).astype(F32)
    c1, o1, _, vy, vz, _ = contract.move(cells + 1, o0, ux, np.full_like(ux, 3.0), np.full_like(ux, -2.0), 0.5)
    for qw in (256, -256, 37):
        Jx, Jy, Jz = contract.deposit(cells + 1, o0, c1, o1, vy, vz, qw, n)
        r0 = contract.charge(cells + 1, o0, qw, n)
        r1 = contract.charge(c1, o1, qw, n)
        assert np.array_equal(r1 - r0 + _div(Jx)[: r0.size], np.zeros_like(r0))


def test_move_matches_double_precision_and_wraps():
    p = random_particles(3, 20000, 10, 20, 1.0, u_lo=1e-3, u_hi=1e3)
    c1, o1, vx, vy, vz, g = contract.move(p["cell"], p["off"], p["ux"], p["uy"], p["uz"], 0.5)
    u = np.stack([p["ux"], p["uy"], p["uz"]], 1)
    xi = p["cell"] + p["off"] + 0.5 * u[:, 0] / np.sqrt(1 + np.sum(u * u, 1))
    assert np.all((o1 >= 0) & (o1 < 1))
    assert np.max(np.abs((c1 + o1.astype(np.float64)) - xi)) < 3e-6  # cell ~ 2^4, f32 offsets
    # s rounds to exactly 1.0 when just left of a node: offset 0 of the right cell
    c, o, *_ = contract.move(np.array([5]), np.array([F32(0.0)]), np.array([F32(-1e-9)]),
                             np.zeros(1, F32), np.zeros(1, F32), 0.5)
    assert c[0] == 5 and o[0] == 0.0


def test_gauss_law_exact_after_random_moves():
    n = 80  # 40 steps move a particle by at most 20 cells
    rng = np.random.default_rng(9)
    cell = rng.integers(25, 55, size=3000)
    off = rng.uniform(0, 1, size=3000).astype(F32)
    ce, oe = cell.copy(), off.copy()  # electrons, co-located with protons at start
    Ex = np.zeros(n + 2, dtype=np.int64)
    for step in range(40):
        u = (rng.normal(size=(3000, 3)) * 3.0).astype(F32)
        c1, o1, _, vy, vz, _ = contract.move(ce, oe, u[:, 0], u[:, 1], u[:, 2], 0.5)
        Jx, _, _ = contract.deposit(ce, oe, c1, o1, vy, vz, -256, n)
        Ex -= Jx
        ce, oe = c1, o1
    rho = contract.charge(ce, oe, -256, n) + contract.charge(cell, off, 256, n)
    # node i sits between half-nodes i (index i) and i + 1
    gauss = Ex[1:n + 2] - Ex[0:n + 1] - rho[1:n + 2]
    assert np.array_equal(gauss, np.zeros_like(gauss))
    assert np.any(Ex != 0)


def test_integer_deposit_matches_double_precision_deposit():
    cfg = preset("c1")
    sim = pic.Pic1D(cfg, init_particles=False)
    n = sim.nx
    p = random_particles(4, 5000, 100, 200, sim.w_ref, u_lo=1e-2, u_hi=1e2)
    c1, o1, vx, vy, vz, g = contract.move(p["cell"], p["off"], p["ux"], p["uy"], p["uz"], cfg["cfl"])
    qw = contract.charge_weight(p["w"], sim.w_ref, -1)
    assert np.all(qw == -256)
    Jx, Jy, Jz = contract.deposit(p["cell"], p["off"], c1, o1, vy, vz, qw, n)
    J = (np.zeros(n + 2), np.zeros(n + 3), np.zeros(n + 3))
    xi0 = p["cell"] + p["off"]
    xi1 = c1 + o1.astype(np.float64)
    sim.deposit(xi0, xi1, vy.astype(np.float64), vz.astype(np.float64), -1.0 * p["w"], J)
    s = sim.w_ref * 2.0 ** -32
    scale_x = sim.w_ref / sim.dt
    scale_y = sim.w_ref / sim.dx
    # quantisation: 2^-24 of a particle's shape per node, plus rint of v at 2^-24
    assert np.max(np.abs(Jx * s / sim.dt - J[0])) < 30 * 2.0 ** -24 * scale_x * 2
    assert np.max(np.abs(Jy * s / sim.dx - J[1])) < 30 * 2.0 ** -22 * scale_y
    assert np.max(np.abs(Jz * s / sim.dx - J[2])) < 30 * 2.0 ** -22 * scale_y
    assert np.max(np.abs(J[1])) > 1e3 * 2.0 ** -22 * scale_y


def test_charge_weight_of_non_reference_weights():
    # the contract's charge weight is the particle weight in units of
    # w_ref / 256, rounded to the nearest integer: qw / 256 lies within half
    # a unit (2^-9) of w / w_ref, carries the species' sign, and is exact
    # (+-256) at the reference weight; rounding goes to the nearest integer
    # on both sides of a half-unit boundary
    rng = np.random.default_rng(3)
    for w_ref in (0.0123, 1.7, 56.25):
        w = (w_ref * rng.uniform(0.01, 40.0, 20000)).astype(np.float32)
        for Z in (-1, 1):
            qw = contract.charge_weight(w, w_ref, Z)
            assert qw.dtype == np.int64
            ratio = w.astype(np.float64) / w_ref
            # float32 arithmetic of w * (256 / w_ref): within half a unit plus
            # the float32 rounding of the product
            assert np.all(np.abs(Z * qw / 256.0 - ratio) <= 0.5 / 256.0 + 2.0 ** -22 * ratio)
            assert np.all(np.sign(qw) == Z)
        assert contract.charge_weight(np.float32(w_ref), w_ref, -1) == -256
    # half-unit boundaries round to even like rint: 2.5 units -> 2, 3.5 units -> 4
    w_ref = 256.0
    assert contract.charge_weight(np.float32(2.5), w_ref, 1) == 2
    assert contract.charge_weight(np.float32(3.5), w_ref, 1) == 4
    assert contract.charge_weight(np.float32(3.25), w_ref, 1) == 3
