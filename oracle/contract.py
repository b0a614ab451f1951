"""Integer current-deposition contract, evaluated from float32 particle state.

TEST INFRASTRUCTURE ONLY (see package header).

The paper does not specify the deposition (it uses "a standard PIC code",
Section 3); this is the reading the GPU path implements so that current,
charge and cell indices are exact integers independent of summation order.

Position.  A particle is stored as an int32 cell index c and a float32
offset o in [0, 1).  After the momentum step, with u the stored float32
momentum and every operation a single IEEE float32 rounding (no fused
multiply-add):
    g  = sqrt(((1 + ux*ux) + uy*uy) + uz*uz),   ig = 1 / g,
    v  = (ux*ig, uy*ig, uz*ig),
    s  = o + vx * cfl          (cfl = dt/dx as float32),
    c' = c + floor(s),  o' = s - floor(s);  if o' == 1 then o' = 0, c' += 1.

Shape weights.  q = floor(o * 2^24) (exact: a power-of-two scale and a
floor); node c carries 2^24 - q and node c+1 carries q.

Charge weight.  qw = Z * rint(w * float32(256 / w_ref)), with w_ref the
run's nominal macro-particle weight; uniform weights give qw = 256 Z.

Current (Esirkepov's charge-conserving rule in 1D for Jx, the average of
old and new shapes for Jy, Jz).  With base = min(c, c') and old / new node
weights Wo[k], Wn[k] on nodes base + k, k = 0, 1, 2:
    Jx[base + 1/2] += qw * (Wo[0] - Wn[0])
    Jx[base + 3/2] += qw * (Wo[0] + Wo[1] - Wn[0] - Wn[1])
    Jy[base + k]   += qw * ((rint(vy * 2^24) * (Wo[k] + Wn[k])) >> 25)
and the same for Jz with vz (">>" is an arithmetic shift, i.e. floor).
Ex is the running integral of the charge flux: each step Ex_int -= Jx_int,
so (Ex_int[i+1/2] - Ex_int[i-1/2]) equals the integer charge on node i
exactly (Gauss's law) for a start with zero charge on every node.

Conversion to floats: Ex = Ex_int * w_ref 2^-32, Jx = Jx_int * w_ref 2^-32 / dt,
Jy, Jz = J_int * w_ref 2^-32 / dx.

Storage indices used here and by the library: node i (-1 .. n_cells + 1) at
index i + 1; half-node (i - 1/2) at index i (0 .. n_cells + 1).

Pins (tests/test_oracle_contract.py): discrete continuity
rho' - rho + div J = 0 exactly on brute-forced tiny grids; agreement with
the double-precision physics deposit of ``pic`` to the quantisation step;
Gauss's law after many random moves.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
TWO24 = 1 << 24


def charge_weight(w, w_ref, Z):
    """qw = Z * rint(w * float32(256 / w_ref)) as int64."""
    sw = F32(256.0 / w_ref)
    return (Z * np.rint(np.asarray(w, dtype=F32) * sw)).astype(np.int64)


def move(cell, off, ux, uy, uz, cfl):
    """New (cell, off) and velocities (vx, vy, vz) in float32, contract order.

    Returns (cell1 int64, off1 float32, vx, vy, vz float32, gamma float32)."""
    off = np.asarray(off, dtype=F32)
    ux, uy, uz = (np.asarray(a, dtype=F32) for a in (ux, uy, uz))
    g = np.sqrt(((F32(1.0) + ux * ux) + uy * uy) + uz * uz)
    ig = F32(1.0) / g
    vx, vy, vz = ux * ig, uy * ig, uz * ig
    s = off + vx * F32(cfl)
    fl = np.floor(s)
    off1 = s - fl
    wrap = off1 >= F32(1.0)
    off1 = np.where(wrap, F32(0.0), off1).astype(F32)
    fl = fl + wrap.astype(F32)
    cell1 = np.asarray(cell, dtype=np.int64) + fl.astype(np.int64)
    return cell1, off1, vx, vy, vz, g


def quantise(off):
    """q = floor(off * 2^24) as int64 (off float32 in [0, 1))."""
    return np.floor(np.asarray(off, dtype=F32) * F32(TWO24)).astype(np.int64)


def deposit(cell0, off0, cell1, off1, vy, vz, qw, n_cells):
    """Integer currents of a set of particle moves.

    Returns (Jx_int, Jy_int, Jz_int): int64 arrays of length n_cells + 2
    (half-nodes) and n_cells + 3 (nodes -1 .. n_cells + 1)."""
    c0 = np.asarray(cell0, dtype=np.int64)
    c1 = np.asarray(cell1, dtype=np.int64)
    qw = np.broadcast_to(np.asarray(qw, dtype=np.int64), c0.shape)
    q0, q1 = quantise(off0), quantise(off1)
    base = np.minimum(c0, c1)
    d0, d1 = c0 - base, c1 - base
    n = c0.size
    Wo = np.zeros((n, 3), dtype=np.int64)
    Wn = np.zeros((n, 3), dtype=np.int64)
    r = np.arange(n)
    Wo[r, d0] = TWO24 - q0
    Wo[r, d0 + 1] = q0
    Wn[r, d1] = TWO24 - q1
    Wn[r, d1 + 1] = q1
    F0 = Wo[:, 0] - Wn[:, 0]
    F1 = F0 + Wo[:, 1] - Wn[:, 1]
    Jx = np.zeros(n_cells + 2, dtype=np.int64)
    np.add.at(Jx, base + 1, qw * F0)
    np.add.at(Jx, base + 2, qw * F1)
    Jy = np.zeros(n_cells + 3, dtype=np.int64)
    Jz = np.zeros(n_cells + 3, dtype=np.int64)
    vy24 = np.rint(np.asarray(vy, dtype=F32) * F32(TWO24)).astype(np.int64)
    vz24 = np.rint(np.asarray(vz, dtype=F32) * F32(TWO24)).astype(np.int64)
    for k in range(3):
        s = Wo[:, k] + Wn[:, k]
        np.add.at(Jy, base + k + 1, qw * ((vy24 * s) >> 25))
        np.add.at(Jz, base + k + 1, qw * ((vz24 * s) >> 25))
    return Jx, Jy, Jz


def charge(cell, off, qw, n_cells):
    """Integer charge on nodes -1 .. n_cells + 1 (index node + 1)."""
    c = np.asarray(cell, dtype=np.int64)
    q = quantise(off)
    qw = np.broadcast_to(np.asarray(qw, dtype=np.int64), c.shape)
    rho = np.zeros(n_cells + 3, dtype=np.int64)
    np.add.at(rho, c + 1, qw * (TWO24 - q))
    np.add.at(rho, c + 2, qw * q)
    return rho
