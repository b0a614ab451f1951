"""Plain 2D3V particle-in-cell loop in double precision.

TEST INFRASTRUCTURE ONLY (see package header).

Section 4 remarks that the momentum space of the 1D code is already three
dimensional, so the same pusher serves a multi-dimensional code unchanged.
This module is that code in two dimensions (x, y; fields and momenta keep
all three components): the pusher is ``pusher.push`` exactly as in the 1D
loop, now with a non-zero B_x.

Readings (the paper gives no multi-dimensional scheme):
* Grid: 2D Yee, dx = dy, periodic in y (ny cells), x as in the 1D loop.
  Staggering (node i at x = i dx, half-node h at x = (h - 1/2) dx; row j at
  y = j dy, half-row g at y = (g + 1/2) dy):
      E_z          node i (0..N),      row j
      E_y, B_x     node i (0..N),      half-row g
      E_x, B_y     half-node h (0..N+1), row j
      B_z          half-node h (0..N+1), half-row g
  h = 0 and h = N + 1 are the boundary guards of the 1D loop.
* Maxwell (normalised, d/dz = 0):
      dBx/dt = -dEz/dy,  dBy/dt = dEz/dx,  dBz/dt = -(dEy/dx - dEx/dy),
      dEx/dt = dBz/dy - Jx,  dEy/dt = -dBz/dx - Jy,
      dEz/dt = dBy/dx - dBx/dy - Jz;
  B in two half steps around the E step, as in 1D.
* Boundaries: per row, the 1D first-order Silver-Mueller guards at both x
  ends (laser injection at x = 0 through the incoming characteristic);
  particles leaving [0, N dx) are removed; y is periodic for fields and
  particles.
* Laser: the 1D incident field times a transverse profile
  exp(-((y - L_y/2) / W)^2) (W = waist; plane wave when W = 0), evaluated at
  the y of each field row.
* Shape: linear in x and y (bilinear gather at each component's position).
* Current: Esirkepov's charge-conserving decomposition for J_x, J_y (the
  2D rule, Esirkepov, Comput. Phys. Commun. 135 (2001) 144): with old and new
  1D weights S^0, S^1 on the 4 x 4 nodes around the old cell,
      W_x = (S^1_x - S^0_x) (S^0_y + S^1_y) / 2,
      W_y = (S^1_y - S^0_y) (S^0_x + S^1_x) / 2,
      J_x(face a + 1/2, row b) = -(q w / (dt dy)) sum_{a' <= a} W_x(a', b),
      J_y(node a, face b + 1/2) = -(q w / (dt dx)) sum_{b' <= b} W_y(a, b');
  J_z = q w v_z (S^0_x S^0_y + S^1_x S^1_y) / (2 dx dy), the average of the
  old and new 2D shapes (the 1D rule for J_y, J_z extended).  Weight
  w = n0 dx dy / ppc.
* Quiet start: ppc = ppc_x ppc_y particles per cell per species on a lattice
  with seeded jitter, electrons and protons co-located (zero charge).
  Particle i of the foil (cells enumerated column by column, rows fastest;
  k = i mod ppc, kx = k div ppc_y, ky = k mod ppc_y) sits at offsets
  ((kx + 1/2) + jitter (U_{2i} - 1/2)) / ppc_x and
  ((ky + 1/2) + jitter (U_{2i+1} - 1/2)) / ppc_y, U_m the SplitMix64 draw m.
* Energies per unit length in z: field sum of field^2 / 2 dx dy (node
  columns with trapezoid end weights, half-node columns 1..N), kinetic
  sum of w M (gamma - 1), radiated and boundary fluxes as in 1D, summed over
  rows times dy.

Pins (tests/test_oracle_pic2d.py): a y-uniform run equals the 1D loop; the
y-directed vacuum modes follow the Yee dispersion; charge continuity of the
deposit on brute-forced moves (including the periodic seam); Gauss's law
after many steps; exact bilinear gather of linear fields; energy balance
without RR.
"""
from __future__ import annotations

import math

import numpy as np

from .pic import envelope, TWO_PI
from .pusher import push, rr_coefficient, gamma_of
from .rng import uniform24


def _hat(o, shift):
    """1D linear weights on the 4 nodes (old cell - 1) .. (old cell + 2) of a
    particle at offset o in cell (old cell + shift), shape (n, 4)."""
    n = o.size
    S = np.zeros((n, 4))
    r = np.arange(n)
    S[r, 1 + shift] = 1.0 - o
    S[r, 2 + shift] = o
    return S


class Pic2D:
    """2D3V laser-foil PIC in float64.  Species 0: electrons, 1: protons."""

    def __init__(self, cfg: dict, init_particles: bool = True):
        self.cfg = dict(cfg)
        cpl = int(cfg["cells_per_lambda"])
        self.dx = TWO_PI / cpl
        self.dt = cfg["cfl"] * self.dx
        self.nx = int(round(cfg["box_x"] * cpl))
        self.ny = int(round(cfg["box_y"] * cpl))
        self.eps = rr_coefficient(cfg["lambda_um"])
        self.ppc = int(cfg["ppc_x"]) * int(cfg["ppc_y"])
        self.w_ref = cfg["n0"] * self.dx * self.dx / self.ppc
        self.mass = (1.0, float(cfg["mass_ratio"]))
        self.Z = (-1.0, 1.0)
        self.qm = (-1.0, 1.0 / float(cfg["mass_ratio"]))
        self.rr = (bool(cfg["rr"]), False)
        self.a0 = float(cfg["a0"])
        self.lp = cfg["pol"] == "LP"
        self.t_env = tuple(TWO_PI * cfg[k] for k in ("t_rise", "t_flat", "t_fall"))
        self.waist = TWO_PI * float(cfg.get("waist", 0.0))
        n, m = self.nx, self.ny
        self.Ez = np.zeros((n + 1, m))
        self.Ey = np.zeros((n + 1, m))
        self.Bx = np.zeros((n + 1, m))
        self.Ex = np.zeros((n + 2, m))
        self.By = np.zeros((n + 2, m))
        self.Bz = np.zeros((n + 2, m))
        self.step_n = 0
        self.E_in = self.E_out_left = self.E_out_right = 0.0
        self.E_rad = 0.0
        self.E_esc = [0.0, 0.0]
        empty = dict(xi=np.zeros(0), eta=np.zeros(0), u=np.zeros((0, 3)), w=np.zeros(0))
        self.sp = [dict(empty) for _ in range(2)]
        if init_particles:
            self._quiet_start()

    # ------------------------------------------------------------------ setup
    def foil_cells(self):
        cpl = self.cfg["cells_per_lambda"]
        return int(round(self.cfg["x_foil"] * cpl)), int(round(self.cfg["thickness"] * cpl))

    def _quiet_start(self):
        px, py = int(self.cfg["ppc_x"]), int(self.cfg["ppc_y"])
        c0, nf = self.foil_cells()
        i = np.arange(nf * self.ny * self.ppc, dtype=np.int64)
        q, k = i // self.ppc, i % self.ppc
        kx, ky = k // py, k % py
        jit = self.cfg["jitter"]
        seed = int(self.cfg["seed"])
        ox = ((kx + 0.5) + jit * (uniform24(seed, 2 * i) - 0.5)) / px
        oy = ((ky + 0.5) + jit * (uniform24(seed, 2 * i + 1) - 0.5)) / py
        xi = (c0 + q // self.ny) + ox
        eta = (q % self.ny) + oy
        for s in range(2):
            self.sp[s] = dict(xi=xi.copy(), eta=eta.copy(), u=np.zeros((xi.size, 3)),
                              w=np.full(xi.size, self.w_ref))

    def set_particles(self, s, xi, eta, u, w):
        self.sp[s] = dict(xi=np.asarray(xi, np.float64).copy(),
                          eta=np.asarray(eta, np.float64).copy(),
                          u=np.array(u, dtype=np.float64).reshape(-1, 3),
                          w=np.array(w, dtype=np.float64))

    # ------------------------------------------------------------------ laser
    def profile(self, y):
        if self.waist <= 0.0:
            return np.ones_like(np.asarray(y, dtype=np.float64))
        yc = 0.5 * self.ny * self.dx
        return np.exp(-((np.asarray(y, dtype=np.float64) - yc) / self.waist) ** 2)

    def incident(self, t):
        """Incident (E_y on half-rows, E_z on rows) at x = 0 and time t."""
        f = self.a0 * envelope(t, *self.t_env)
        yg = (np.arange(self.ny) + 0.5) * self.dx
        yj = np.arange(self.ny) * self.dx
        if self.lp:
            return f * math.sin(t) * self.profile(yg), 0.0 * yj
        f /= math.sqrt(2.0)
        return f * math.sin(t) * self.profile(yg), f * math.cos(t) * self.profile(yj)

    # ------------------------------------------------------------------ stages
    def gather(self, xi, eta):
        """E, B (n, 3) at positions (xi, eta) in cells, bilinear weighting of
        each component at its own grid position."""
        m = self.ny
        c = np.floor(xi).astype(np.int64)
        o = xi - c
        j = np.floor(eta).astype(np.int64)
        p = eta - j
        sx = o + 0.5                       # half-node weights in x
        hb = np.floor(sx)
        fx = sx - hb
        h = c + hb.astype(np.int64)
        sy = p - 0.5                       # half-row weights in y
        gb = np.floor(sy)
        fy = sy - gb
        g = j + gb.astype(np.int64)

        def bilin(A, ix, wx, iy, wy):
            y0, y1 = iy % m, (iy + 1) % m
            return ((1 - wx) * ((1 - wy) * A[ix, y0] + wy * A[ix, y1])
                    + wx * ((1 - wy) * A[ix + 1, y0] + wy * A[ix + 1, y1]))

        Ez = bilin(self.Ez, c, o, j, p)
        Ey = bilin(self.Ey, c, o, g, fy)
        Bx = bilin(self.Bx, c, o, g, fy)
        Ex = bilin(self.Ex, h, fx, j, p)
        By = bilin(self.By, h, fx, j, p)
        Bz = bilin(self.Bz, h, fx, g, fy)
        return np.stack([Ex, Ey, Ez], axis=1), np.stack([Bx, By, Bz], axis=1)

    def deposit(self, xi0, eta0, xi1, eta1, vz, Zw, J):
        """Add the currents of moves (xi0, eta0) -> (xi1, eta1) (unwrapped in
        y) to J = (Jx, Jy, Jz): Jx[h, j] on half-nodes (0..N+1), Jy[i + 1, g]
        and Jz[i + 1, j] on nodes -1..N+1."""
        Jx, Jy, Jz = J
        m = self.ny
        c0 = np.floor(xi0).astype(np.int64)
        j0 = np.floor(eta0).astype(np.int64)
        c1 = np.floor(xi1).astype(np.int64)
        j1 = np.floor(eta1).astype(np.int64)
        Sx0 = _hat(xi0 - c0, np.zeros_like(c0))
        Sy0 = _hat(eta0 - j0, np.zeros_like(j0))
        Sx1 = _hat(xi1 - c1, c1 - c0)
        Sy1 = _hat(eta1 - j1, j1 - j0)
        Wx = (Sx1 - Sx0)[:, :, None] * (Sy0 + Sy1)[:, None, :] / 2.0
        Wy = (Sx0 + Sx1)[:, :, None] * (Sy1 - Sy0)[:, None, :] / 2.0
        Fx = -np.cumsum(Wx, axis=1)[:, :3, :]      # faces a + 1/2, a = 0..2
        Fy = -np.cumsum(Wy, axis=2)[:, :, :3]      # half-rows b + 1/2, b = 0..2
        Nz = (Sx0[:, :, None] * Sy0[:, None, :] + Sx1[:, :, None] * Sy1[:, None, :]) / 2.0
        dt, dx = self.dt, self.dx
        kx = (Zw / (dt * dx))[:, None, None]
        kz = (Zw * vz / (dx * dx))[:, None, None]
        Fx, Fy, Nz = kx * Fx, kx * Fy, kz * Nz
        for a in range(4):
            for b in range(4):
                row = (j0 - 1 + b) % m
                node = c0 - 1 + a + 1                # node index (guard offset 1)
                if a < 3:
                    np.add.at(Jx, (c0 + a, row), Fx[:, a, b])
                if b < 3:
                    np.add.at(Jy, (node, row), Fy[:, a, b])
                np.add.at(Jz, (node, row), Nz[:, a, b])

    def push_species(self, s, J):
        P = self.sp[s]
        if P["xi"].size == 0:
            return
        E, B = self.gather(P["xi"], P["eta"])
        u_new, uL = push(P["u"], E, B, self.qm[s], self.dt, self.eps, self.rr[s])
        g_new = gamma_of(u_new)
        if self.rr[s]:
            gL = gamma_of(uL)
            dg = np.sum((uL - u_new) * (uL + u_new), axis=1) / (gL + g_new)
            self.E_rad += float(np.sum(P["w"] * self.mass[s] * dg))
        v = u_new / g_new[:, None]
        xi1 = P["xi"] + v[:, 0] * self.dt / self.dx
        eta1 = P["eta"] + v[:, 1] * self.dt / self.dx
        self.deposit(P["xi"], P["eta"], xi1, eta1, v[:, 2], self.Z[s] * P["w"], J)
        gone = (xi1 < 0.0) | (xi1 >= self.nx)
        if np.any(gone):
            self.E_esc[s] += float(np.sum(P["w"][gone] * self.mass[s] * (g_new[gone] - 1.0)))
        keep = ~gone
        self.sp[s] = dict(xi=xi1[keep], eta=np.mod(eta1[keep], self.ny), u=u_new[keep],
                          w=P["w"][keep])

    def _half_b(self):
        a = 0.5 * self.dt / self.dx
        n = self.nx
        self.Bx -= a * (np.roll(self.Ez, -1, axis=1) - self.Ez)
        self.By[1:n + 1] += a * (self.Ez[1:] - self.Ez[:-1])
        self.Bz[1:n + 1] -= a * ((self.Ey[1:] - self.Ey[:-1])
                                 - (np.roll(self.Ex[1:n + 1], -1, axis=1) - self.Ex[1:n + 1]))

    def advance_fields(self, Jx, Jy, Jz):
        """Yee update with J^{n+1/2}: B half step, guards, E full step, B half
        step; Poynting bookkeeping at both x ends, row by row."""
        dt, a, n, dy = self.dt, self.dt / self.dx, self.nx, self.dx
        jy, jz = Jy[1:n + 2], Jz[1:n + 2]
        Ey0, Ez0 = self.Ey.copy(), self.Ez.copy()
        self._half_b()
        ey_in, ez_in = self.incident((self.step_n + 0.5) * dt)
        d = 1.0 + a
        self.Bz[0] = (4.0 * ey_in - 2.0 * self.Ey[0] - (1.0 - a) * self.Bz[1] + dt * jy[0]) / d
        self.By[0] = (2.0 * self.Ez[0] - (1.0 - a) * self.By[1] - dt * jz[0] - 4.0 * ez_in) / d
        self.Bz[n + 1] = (2.0 * self.Ey[n] - (1.0 - a) * self.Bz[n] - dt * jy[n]) / d
        self.By[n + 1] = (-2.0 * self.Ez[n] - (1.0 - a) * self.By[n] + dt * jz[n]) / d
        self.Ex[1:n + 1] += a * (self.Bz[1:n + 1] - np.roll(self.Bz[1:n + 1], 1, axis=1)) \
            - dt * Jx[1:n + 1]
        self.Ey -= a * (self.Bz[1:] - self.Bz[:-1]) + dt * jy
        self.Ez += a * ((self.By[1:] - self.By[:-1]) - (self.Bx - np.roll(self.Bx, 1, axis=1))) \
            - dt * jz
        eyl, ezl = 0.5 * (Ey0[0] + self.Ey[0]), 0.5 * (Ez0[0] + self.Ez[0])
        bzl, byl = 0.5 * (self.Bz[0] + self.Bz[1]), 0.5 * (self.By[0] + self.By[1])
        eyr, ezr = 0.5 * (Ey0[n] + self.Ey[n]), 0.5 * (Ez0[n] + self.Ez[n])
        bzr, byr = 0.5 * (self.Bz[n] + self.Bz[n + 1]), 0.5 * (self.By[n] + self.By[n + 1])
        self.E_in += dt * dy * float(np.sum(ey_in * ey_in + ez_in * ez_in))
        self.E_out_left += dt * dy * 0.25 * float(np.sum((eyl - bzl) ** 2 + (ezl + byl) ** 2))
        self.E_out_right += dt * dy * 0.25 * float(np.sum((eyr + bzr) ** 2 + (ezr - byr) ** 2))
        self._half_b()

    def new_currents(self):
        n, m = self.nx, self.ny
        return np.zeros((n + 2, m)), np.zeros((n + 3, m)), np.zeros((n + 3, m))

    def step(self):
        J = self.new_currents()
        for s in range(2):
            self.push_species(s, J)
        self.advance_fields(*J)
        self.step_n += 1
        return J

    def run(self, n_steps: int):
        for _ in range(n_steps):
            self.step()
        return self

    # ------------------------------------------------------------------ diagnostics
    def field_energy(self):
        """(U_Ex, U_Etrans, U_B) per unit length in z."""
        n, dx = self.nx, self.dx
        wn = np.ones(n + 1)
        wn[0] = wn[-1] = 0.5
        a2 = 0.5 * dx * dx
        ue = a2 * float(np.sum(wn[:, None] * (self.Ey ** 2 + self.Ez ** 2)))
        ux = a2 * float(np.sum(self.Ex[1:n + 1] ** 2))
        ub = a2 * float(np.sum(wn[:, None] * self.Bx ** 2)
                        + np.sum(self.By[1:n + 1] ** 2 + self.Bz[1:n + 1] ** 2))
        return ux, ue, ub

    def kinetic(self, s):
        P = self.sp[s]
        return float(np.sum(P["w"] * self.mass[s] * (gamma_of(P["u"]) - 1.0)))

    def charge_density(self):
        """rho on nodes (N + 1, ny) by bilinear weighting."""
        n, m = self.nx, self.ny
        rho = np.zeros((n + 1, m))
        for s in range(2):
            P = self.sp[s]
            c = np.floor(P["xi"]).astype(np.int64)
            j = np.floor(P["eta"]).astype(np.int64)
            o, p = P["xi"] - c, P["eta"] - j
            q = self.Z[s] * P["w"] / (self.dx * self.dx)
            for a, wa in ((0, 1 - o), (1, o)):
                for b, wb in ((0, 1 - p), (1, p)):
                    np.add.at(rho, (c + a, (j + b) % m), q * wa * wb)
        return rho

    def gauss_residual(self):
        """max |div E - rho| over nodes 1..N-1, all rows."""
        n, dx = self.nx, self.dx
        divE = ((self.Ex[2:n + 1] - self.Ex[1:n]) / dx
                + (self.Ey[1:n] - np.roll(self.Ey[1:n], 1, axis=1)) / dx)
        res = divE - self.charge_density()[1:n]
        return float(np.max(np.abs(res))) if res.size else 0.0

    def diag(self) -> dict:
        ux, ue, ub = self.field_energy()
        ke, ki = self.kinetic(0), self.kinetic(1)
        out = dict(step=self.step_n, t=self.step_n * self.dt,
                   n_alive=(self.sp[0]["xi"].size, self.sp[1]["xi"].size),
                   U_Ex=ux, U_Et=ue, U_B=ub, U_field=ux + ue + ub,
                   K_e=ke, K_i=ki, E_rad=self.E_rad, E_in=self.E_in,
                   E_out_left=self.E_out_left, E_out_right=self.E_out_right,
                   E_esc=self.E_esc[0] + self.E_esc[1],
                   gauss=self.gauss_residual())
        out["balance"] = (out["U_field"] + ke + ki + self.E_rad + self.E_out_left
                          + self.E_out_right + out["E_esc"] - self.E_in)
        return out
