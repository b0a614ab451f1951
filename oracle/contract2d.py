"""Integer current-deposition contract of the 2D3V path, from float32 state.

TEST INFRASTRUCTURE ONLY (see package header).

The 2D extension of the 1D contract in ``contract``: exact integers for the
current and the cell indices, independent of summation order, with
Esirkepov's 2D decomposition (see ``pic2d``) in fixed point.

Position.  A particle is stored as one int32 cell index L = ix * ny + iy
(column ix in x, row iy in the periodic y direction) and two float32
offsets ox, oy in [0, 1).  After the momentum step, with u the stored
float32 momentum and one IEEE float32 rounding per operation (no fused
multiply-add):
    g = sqrt(((1 + ux*ux) + uy*uy) + uz*uz),  ig = 1 / g,  v = u * ig,
    sx = ox + vx * cfl,  sy = oy + vy * cfl   (cfl = dt/dx = dt/dy, float32),
each offset renormalised as in 1D (floor, and a result of exactly 1 moves
to the next cell), ix' = ix + floor(sx), iy' = (iy + floor(sy)) mod ny.

Shape weights (12 bits per direction).  q = floor(o * 2^12); on the four
nodes (old cell - 1) .. (old cell + 2) of a direction the old weights are
(0, 2^12 - q, q, 0); the new ones are the same pattern moved by the cell
shift s in {-1, 0, 1}.  With dS = S_new - S_old, Sig = S_old + S_new and
C[a] = -(dS[0] + .. + dS[a]) (a = 0, 1, 2):
    Jx[face a + 1/2, row b]    += qw * C_x[a] * Sig_y[b]   (a 0..2, b 0..3)
    Jy[node a, half-row b + 1/2] += qw * Sig_x[a] * C_y[b]   (a 0..3, b 0..2)
    Jz[node a, row b] += qw * rint(vz * 2^12)
                          * ((S_old_x[a] S_old_y[b] + S_new_x[a] S_new_y[b]) >> 12)
(">>" an arithmetic shift); the charge of a particle on node (a, b) is
2 qw S_x[a] S_y[b], so rho' - rho + div J = 0 exactly, node by node.  Every
term is below 2^25 in magnitude (moves of at most half a cell).

Conversion to floats: dt Jx and dt Jy = J_int w_ref 2^-33 / dx,
dt Jz = J_int w_ref 2^-33 dt / dx^2, rho = rho_int w_ref 2^-33 / dx^2.

Storage: Jx[h, iy] on half-nodes h = 0..N+1 (x = (h - 1/2) dx); Jy[i + 1, g]
and Jz[i + 1, iy] on nodes i = -1..N+1; half-row g at y = (g + 1/2) dy.

Pins (tests/test_oracle_pic2d.py): exact continuity on brute-forced moves
including the periodic seam; agreement with the double-precision deposit of
``pic2d`` to the quantisation step.
"""
from __future__ import annotations

import numpy as np

from .contract import charge_weight  # noqa: F401  (same charge-weight rule)

F32 = np.float32
Q = 12
ONE = 1 << Q


def _renorm(s):
    fl = np.floor(s)
    o1 = s - fl
    wrap = o1 >= F32(1.0)
    o1 = np.where(wrap, F32(0.0), o1).astype(F32)
    return o1, (fl + wrap.astype(F32)).astype(np.int64)


def move(ix, iy, ox, oy, ux, uy, uz, cfl, ny):
    """New (ix, iy, ox, oy), cell shifts (sx, sy) and float32 (vx, vy, vz, g)."""
    ox, oy = (np.asarray(a, dtype=F32) for a in (ox, oy))
    ux, uy, uz = (np.asarray(a, dtype=F32) for a in (ux, uy, uz))
    g = np.sqrt(((F32(1.0) + ux * ux) + uy * uy) + uz * uz)
    ig = F32(1.0) / g
    vx, vy, vz = ux * ig, uy * ig, uz * ig
    ox1, sx = _renorm(ox + vx * F32(cfl))
    oy1, sy = _renorm(oy + vy * F32(cfl))
    ix1 = np.asarray(ix, dtype=np.int64) + sx
    iy1 = np.mod(np.asarray(iy, dtype=np.int64) + sy, ny)
    return ix1, iy1, ox1, oy1, sx, sy, vx, vy, vz, g


def quantise(o):
    return np.floor(np.asarray(o, dtype=F32) * F32(ONE)).astype(np.int64)


def _weights(q, shift):
    n = q.size
    S = np.zeros((n, 4), dtype=np.int64)
    r = np.arange(n)
    S[r, 1 + shift] = ONE - q
    S[r, 2 + shift] = q
    return S


def deposit(ix, iy, ox, oy, sx, sy, ox1, oy1, vz, qw, nx, ny):
    """Integer currents of a set of moves; (ix, iy) the old cell, (sx, sy) the
    cell shifts, (ox1, oy1) the new offsets.  Returns int64 arrays
    Jx (nx + 2, ny), Jy (nx + 3, ny), Jz (nx + 3, ny)."""
    ix = np.asarray(ix, dtype=np.int64)
    iy = np.asarray(iy, dtype=np.int64)
    sx = np.asarray(sx, dtype=np.int64)
    sy = np.asarray(sy, dtype=np.int64)
    qw = np.broadcast_to(np.asarray(qw, dtype=np.int64), ix.shape)
    Sx0 = _weights(quantise(ox), np.zeros_like(sx))
    Sy0 = _weights(quantise(oy), np.zeros_like(sy))
    Sx1 = _weights(quantise(ox1), sx)
    Sy1 = _weights(quantise(oy1), sy)
    Cx = -np.cumsum(Sx1 - Sx0, axis=1)
    Cy = -np.cumsum(Sy1 - Sy0, axis=1)
    Sgx, Sgy = Sx0 + Sx1, Sy0 + Sy1
    vz12 = np.rint(np.asarray(vz, dtype=F32) * F32(ONE)).astype(np.int64)
    Jx = np.zeros((nx + 2, ny), dtype=np.int64)
    Jy = np.zeros((nx + 3, ny), dtype=np.int64)
    Jz = np.zeros((nx + 3, ny), dtype=np.int64)
    for a in range(4):
        for b in range(4):
            row = np.mod(iy - 1 + b, ny)
            if a < 3:
                np.add.at(Jx, (ix + a, row), qw * Cx[:, a] * Sgy[:, b])
            if b < 3:
                np.add.at(Jy, (ix + a, row), qw * Sgx[:, a] * Cy[:, b])
            nz = Sx0[:, a] * Sy0[:, b] + Sx1[:, a] * Sy1[:, b]
            np.add.at(Jz, (ix + a, row), qw * vz12 * (nz >> Q))
    return Jx, Jy, Jz


def charge(ix, iy, ox, oy, qw, nx, ny):
    """Integer charge 2 qw S_x S_y on nodes -1..N+1 (index node + 1), all rows."""
    ix = np.asarray(ix, dtype=np.int64)
    iy = np.asarray(iy, dtype=np.int64)
    qw = np.broadcast_to(np.asarray(qw, dtype=np.int64), ix.shape)
    qx, qy = quantise(ox), quantise(oy)
    rho = np.zeros((nx + 3, ny), dtype=np.int64)
    for a, wa in ((0, ONE - qx), (1, qx)):
        for b, wb in ((0, ONE - qy), (1, qy)):
            np.add.at(rho, (ix + a + 1, np.mod(iy + b, ny)), 2 * qw * wa * wb)
    return rho


def divergence(Jx, Jy):
    """Integer divergence on nodes -1..N+1 (index node + 1), all rows:
    (Jx[i + 1/2] - Jx[i - 1/2]) + (Jy[g = iy] - Jy[g = iy - 1])."""
    ny = Jy.shape[1]
    # node i (index i + 1) has faces h = i (left) and h = i + 1 (right); no
    # current crosses the faces beyond the guards
    Jxp = np.concatenate([np.zeros((1, ny), np.int64), Jx, np.zeros((1, ny), np.int64)])
    return (Jxp[1:] - Jxp[:-1]) + (Jy - np.roll(Jy, 1, axis=1))
