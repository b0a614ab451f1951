"""Seeded random inputs for unit and parity tests, and the serving request stream.

Everything returned here is plain data.  Floating-point arrays meant to be
fed to both the single-precision GPU path and the double-precision oracle
are rounded to float32 first, so both sides start from identical values.
"""
from __future__ import annotations

import numpy as np


def _isotropic(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def random_push_inputs(seed: int, n: int, u_lo=1e-3, u_hi=1e4, f_max=1600.0,
                       as_float32=True) -> dict:
    """Momenta with |u| log-uniform on [u_lo, u_hi] and isotropic direction;
    E and B with magnitudes uniform on [0, f_max] and isotropic direction."""
    rng = np.random.default_rng(seed)
    mag = np.exp(rng.uniform(np.log(u_lo), np.log(u_hi), size=n))
    u = _isotropic(rng, n) * mag[:, None]
    E = _isotropic(rng, n) * rng.uniform(0.0, f_max, size=n)[:, None]
    B = _isotropic(rng, n) * rng.uniform(0.0, f_max, size=n)[:, None]
    out = dict(u=u, E=E, B=B)
    if as_float32:
        out = {k: v.astype(np.float32).astype(np.float64) for k, v in out.items()}
    return out


def random_particles(seed: int, n: int, cell_lo: int, cell_hi: int, w: float,
                     u_lo=1e-3, u_hi=1e3, sort=True) -> dict:
    """``n`` particles in cells [cell_lo, cell_hi) with uniform in-cell offsets,
    log-uniform isotropic momenta and weight ``w``; values are float32-exact.
    Returned arrays: cell (int32), off, ux, uy, uz, w (float64 holding float32
    values)."""
    rng = np.random.default_rng(seed)
    cell = rng.integers(cell_lo, cell_hi, size=n).astype(np.int32)
    off = rng.uniform(0.0, 1.0, size=n).astype(np.float32)
    off = np.where(off >= np.float32(1.0), np.float32(0.0), off)
    mag = np.exp(rng.uniform(np.log(u_lo), np.log(u_hi), size=n))
    u = (_isotropic(rng, n) * mag[:, None]).astype(np.float32)
    if sort:
        order = np.argsort(cell, kind="stable")
        cell, off, u = cell[order], off[order], u[order]
    wf = np.full(n, np.float32(w), dtype=np.float32)
    f64 = lambda a: a.astype(np.float64)
    return dict(cell=cell, off=f64(off), ux=f64(u[:, 0]), uy=f64(u[:, 1]),
                uz=f64(u[:, 2]), w=f64(wf))


def random_fields(seed: int, n_cells: int, amp: float) -> dict:
    """Random grid fields on a 1D Yee grid with ``n_cells`` cells.

    Node arrays (Ey, Ez) have n_cells+1 entries (nodes 0..n_cells); half-node
    arrays (Ex, By, Bz) have n_cells+2 entries (positions -1/2 .. n_cells+1/2).
    Values are uniform in [-amp, amp] and float32-exact."""
    rng = np.random.default_rng(seed)
    f = lambda m: rng.uniform(-amp, amp, size=m).astype(np.float32).astype(np.float64)
    return dict(Ey=f(n_cells + 1), Ez=f(n_cells + 1),
                Ex=f(n_cells + 2), By=f(n_cells + 2), Bz=f(n_cells + 2))


def poisson_stream(seed: int = 0, n_runs: int = 256, rate: float = 20.0,
                   n_lo=1e4, n_hi=1e6) -> list:
    """Serving request stream: Poisson arrivals (mean ``rate`` per second) of
    independent foil runs with randomised laser, foil and size.

    Per run: a0 ~ U[50, 500]; LP or CP with p = 0.5; n0 ~ U[50, 150];
    thickness ~ U[0.5, 2] wavelengths; particle count log-uniform on
    [n_lo, n_hi]; run length a whole number of periods in [30, 80].
    The grid is 100 cells per wavelength and the box holds the foil, 8
    wavelengths of vacuum in front and one wavelength per period behind."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_runs))
    runs = []
    for i in range(n_runs):
        thick = float(rng.uniform(0.5, 2.0))
        n_part = float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        periods = int(rng.integers(30, 81))
        cpl = 100
        foil_cells = max(1, int(round(thick * cpl)))
        ppc = max(1, int(round(n_part / (2 * foil_cells))))
        runs.append(dict(
            arrival=float(t[i]),
            cfg=dict(precision="fp32", lambda_um=0.8, cells_per_lambda=cpl,
                     box_lambda=float(np.ceil(8.0 + thick + periods)), cfl=0.5,
                     pol="LP" if rng.uniform() < 0.5 else "CP",
                     a0=float(rng.uniform(50.0, 500.0)),
                     t_rise=5.0, t_flat=0.0, t_fall=5.0,
                     n0=float(rng.uniform(50.0, 150.0)), x_foil=8.0,
                     thickness=foil_cells / cpl, ppc=ppc, mass_ratio=1836.0,
                     rr=True, rr_compensated=True, seed=i, jitter=0.5,
                     periods=float(periods), sort_interval=32, name=f"req{i}")))
    return runs


def random_particles2d(seed: int, n: int, ix_lo: int, ix_hi: int, ny: int, w: float,
                       u_lo=1e-3, u_hi=1e3, sort=True) -> dict:
    """``n`` particles of a 2D grid: columns [ix_lo, ix_hi), rows [0, ny),
    uniform in-cell offsets, log-uniform isotropic momenta, weight ``w``;
    values float32-exact.  sort: ordered by (column, row).  Returned arrays:
    ix, iy (int64), ox, oy, ux, uy, uz, w (float64 holding float32 values)."""
    rng = np.random.default_rng(seed)
    ix = rng.integers(ix_lo, ix_hi, size=n)
    iy = rng.integers(0, ny, size=n)
    o = rng.uniform(0.0, 1.0, size=(n, 2)).astype(np.float32)
    o = np.where(o >= np.float32(1.0), np.float32(0.0), o)
    mag = np.exp(rng.uniform(np.log(u_lo), np.log(u_hi), size=n))
    u = (_isotropic(rng, n) * mag[:, None]).astype(np.float32)
    if sort:
        order = np.lexsort((iy, ix))
        ix, iy, o, u = ix[order], iy[order], o[order], u[order]
    f64 = lambda a: a.astype(np.float64)
    return dict(ix=ix, iy=iy, ox=f64(o[:, 0]), oy=f64(o[:, 1]), ux=f64(u[:, 0]), uy=f64(u[:, 1]),
                uz=f64(u[:, 2]), w=f64(np.full(n, np.float32(w), dtype=np.float32)))


def random_fields2d(seed: int, nx: int, ny: int, amp: float) -> dict:
    """Random fields on a 2D Yee grid of nx by ny cells, uniform in [-amp, amp]
    and float32-exact: node components (Ey, Ez, Bx) have nx + 1 columns,
    half-node components (Ex, By, Bz) nx + 2; every array has ny rows."""
    rng = np.random.default_rng(seed)
    f = lambda m: rng.uniform(-amp, amp, size=(m, ny)).astype(np.float32).astype(np.float64)
    return dict(Ey=f(nx + 1), Ez=f(nx + 1), Bx=f(nx + 1), Ex=f(nx + 2), By=f(nx + 2),
                Bz=f(nx + 2))
