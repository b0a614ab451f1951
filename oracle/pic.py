"""Plain 1D3V particle-in-cell loop in double precision.

TEST INFRASTRUCTURE ONLY (see package header).

What the paper fixes (Section 3): particles are advanced by the Boris
pusher plus the RR force of Eq. (f_r), combined by Eqs. (tot)-(pertfull),
with the mid-step estimate of Eqs. (estim1), (estimgamma) and the fields
E^(n), B^(n) at the integer step; positions follow the leapfrog
x^{n+1} = x^n + dt u^{n+1/2} / gamma^{n+1/2}.  The laser-foil problem is
Section 4 (protons and electrons, foil of density n0 and thickness l).

What the paper leaves to "a standard PIC code", and the readings taken:
* Grid: 1D Yee.  E_y, E_z, J_y, J_z on nodes x_i = i dx (i = 0..N);
  E_x, B_y, B_z, J_x on half-nodes x = (h - 1/2) dx (h = 0..N+1; h = 0 and
  h = N+1 are boundary guards).  E at integer steps; B advanced in two
  half steps so that B^n is available at integer steps for the pusher.
* Maxwell (normalised): dEx/dt = -Jx, dEy/dt = -dBz/dx - Jy,
  dEz/dt = dBy/dx - Jz, dBy/dt = dEz/dx, dBz/dt = -dEy/dx.
* Shape: linear weighting (cloud in cell) for gather and deposit.
* Current: charge-conserving 1D rule for Jx
  (Jx[m+1/2] = -(Z w / dt) sum_{k<=m} dW_k), average of old and new shape
  times v_y, v_z for Jy, Jz (divided by dx); Ex -= dt Jx.
* Boundaries: the laser enters through the left boundary, where the
  incoming characteristic E_y + B_z (resp. E_z - B_y) is set to twice the
  incident field and the outgoing one is free (a first-order
  Silver-Mueller condition written into the guard B); the right boundary
  is absorbing in the same way.  Particles leaving [0, N dx) are removed
  and their kinetic energy is booked as escaped.
* Step order: gather E^n, B^n -> push -> move -> deposit J^{n+1/2} ->
  remove escaped -> B^{n+1/2} -> guards -> E^{n+1} -> B^{n+1}.
* Radiation reaction on electrons only (Section 2 treats the electron).
* Radiated energy per step: w (gamma_L - gamma^{n+1/2}), evaluated as
  (u_L - u_new).(u_L + u_new) / (gamma_L + gamma_new).
* Kinetic energy in diagnostics uses the stored u^{n-1/2}.

Pins (tests/test_oracle_pic.py): Yee vacuum dispersion, injected laser
energy, right-boundary reflection, cold plasma oscillation at sqrt(n0),
charge continuity and Gauss's law, energy conservation without RR.
"""
from __future__ import annotations

import math

import numpy as np

from .pusher import push, rr_coefficient, gamma_of
from .rng import uniform24

TWO_PI = 2.0 * math.pi


def envelope(t, t_rise, t_flat, t_fall):
    """Amplitude envelope (times in 1/omega): sin^2 rise, flat top, sin^2 fall."""
    if t <= 0.0:
        return 0.0
    if t < t_rise:
        return math.sin(0.5 * math.pi * t / t_rise) ** 2
    t -= t_rise
    if t < t_flat:
        return 1.0
    t -= t_flat
    if t < t_fall:
        return math.cos(0.5 * math.pi * t / t_fall) ** 2
    return 0.0


class Pic1D:
    """1D3V laser-foil PIC in float64.  Species 0: electrons, 1: protons."""

    def __init__(self, cfg: dict, init_particles: bool = True):
        self.cfg = dict(cfg)
        cpl = int(cfg["cells_per_lambda"])
        self.dx = TWO_PI / cpl
        self.dt = cfg["cfl"] * self.dx
        self.nx = int(round(cfg["box_lambda"] * cpl))
        self.eps = rr_coefficient(cfg["lambda_um"])
        self.w_ref = cfg["n0"] * self.dx / cfg["ppc"]
        self.mass = (1.0, float(cfg["mass_ratio"]))
        self.Z = (-1.0, 1.0)
        self.qm = (-1.0, 1.0 / float(cfg["mass_ratio"]))
        self.rr = (bool(cfg["rr"]), False)
        self.a0 = float(cfg["a0"])
        self.lp = cfg["pol"] == "LP"
        self.t_env = tuple(TWO_PI * cfg[k] for k in ("t_rise", "t_flat", "t_fall"))
        n = self.nx
        self.Ey = np.zeros(n + 1)
        self.Ez = np.zeros(n + 1)
        self.Ex = np.zeros(n + 2)
        self.By = np.zeros(n + 2)
        self.Bz = np.zeros(n + 2)
        self.step_n = 0
        self.E_in = self.E_out_left = self.E_out_right = 0.0
        self.E_rad = 0.0
        self.E_esc = [0.0, 0.0]
        self.sp = [dict(xi=np.zeros(0), u=np.zeros((0, 3)), w=np.zeros(0)) for _ in range(2)]
        if init_particles:
            self._quiet_start()

    # ------------------------------------------------------------------ setup
    def foil_cells(self):
        cpl = self.cfg["cells_per_lambda"]
        c0 = int(round(self.cfg["x_foil"] * cpl))
        nf = int(round(self.cfg["thickness"] * cpl))
        return c0, nf

    def _quiet_start(self):
        """Cold, charge-neutral foil: ppc particles per cell at offsets
        ((k + 1/2) + jitter (U - 1/2)) / ppc, U from SplitMix64 keyed by the
        particle index; electrons and protons share positions."""
        ppc = int(self.cfg["ppc"])
        c0, nf = self.foil_cells()
        i = np.arange(nf * ppc, dtype=np.int64)
        k = i % ppc
        U = uniform24(int(self.cfg["seed"]), i)
        off = ((k + 0.5) + self.cfg["jitter"] * (U - 0.5)) / ppc
        xi = (c0 + i // ppc) + off
        for s in range(2):
            self.sp[s] = dict(xi=xi.copy(), u=np.zeros((xi.size, 3)),
                              w=np.full(xi.size, self.w_ref))

    def set_particles(self, s, cell, off, u, w):
        self.sp[s] = dict(xi=np.asarray(cell, np.float64) + np.asarray(off, np.float64),
                          u=np.array(u, dtype=np.float64).reshape(-1, 3),
                          w=np.array(w, dtype=np.float64))

    # ------------------------------------------------------------------ laser
    def incident(self, t):
        """Incident (E_y, E_z) at x = 0 and time t."""
        f = self.a0 * envelope(t, *self.t_env)
        if self.lp:
            return f * math.sin(t), 0.0
        f /= math.sqrt(2.0)
        return f * math.sin(t), f * math.cos(t)

    # ------------------------------------------------------------------ stages
    def gather(self, xi):
        """E, B (n, 3) at positions xi (in cells) by linear weighting."""
        c = np.floor(xi).astype(np.int64)
        o = xi - c
        Ey = (1.0 - o) * self.Ey[c] + o * self.Ey[c + 1]
        Ez = (1.0 - o) * self.Ez[c] + o * self.Ez[c + 1]
        sx = o + 0.5
        hb = np.floor(sx)
        fh = sx - hb
        h = c + hb.astype(np.int64)
        Ex = (1.0 - fh) * self.Ex[h] + fh * self.Ex[h + 1]
        By = (1.0 - fh) * self.By[h] + fh * self.By[h + 1]
        Bz = (1.0 - fh) * self.Bz[h] + fh * self.Bz[h + 1]
        E = np.stack([Ex, Ey, Ez], axis=1)
        B = np.stack([np.zeros_like(By), By, Bz], axis=1)
        return E, B

    def deposit(self, xi0, xi1, vy, vz, Zw, J):
        """Add the currents of moves xi0 -> xi1 to J = (Jx, Jy, Jz)."""
        Jx, Jy, Jz = J
        c0 = np.floor(xi0).astype(np.int64)
        c1 = np.floor(xi1).astype(np.int64)
        o0, o1 = xi0 - c0, xi1 - c1
        base = np.minimum(c0, c1)
        n = xi0.size
        r = np.arange(n)
        Wo = np.zeros((n, 3))
        Wn = np.zeros((n, 3))
        Wo[r, c0 - base] = 1.0 - o0
        Wo[r, c0 - base + 1] = o0
        Wn[r, c1 - base] = 1.0 - o1
        Wn[r, c1 - base + 1] = o1
        dW = Wn - Wo
        dt, dx = self.dt, self.dx
        Jx += np.bincount(base + 1, weights=-(Zw / dt) * dW[:, 0], minlength=Jx.size)
        Jx += np.bincount(base + 2, weights=-(Zw / dt) * (dW[:, 0] + dW[:, 1]),
                          minlength=Jx.size)
        for k in range(3):
            avg = 0.5 * (Wo[:, k] + Wn[:, k]) * Zw / dx
            Jy += np.bincount(base + k + 1, weights=vy * avg, minlength=Jy.size)
            Jz += np.bincount(base + k + 1, weights=vz * avg, minlength=Jz.size)

    def push_species(self, s, J):
        """Gather, push, move and deposit species s; remove escaped particles."""
        P = self.sp[s]
        if P["xi"].size == 0:
            return
        E, B = self.gather(P["xi"])
        u_old = P["u"]
        u_new, uL = push(u_old, E, B, self.qm[s], self.dt, self.eps, self.rr[s])
        g_new = gamma_of(u_new)
        if self.rr[s]:
            gL = gamma_of(uL)
            dg = np.sum((uL - u_new) * (uL + u_new), axis=1) / (gL + g_new)
            self.E_rad += float(np.sum(P["w"] * self.mass[s] * dg))
        v = u_new / g_new[:, None]
        xi1 = P["xi"] + v[:, 0] * self.dt / self.dx
        self.deposit(P["xi"], xi1, v[:, 1], v[:, 2], self.Z[s] * P["w"], J)
        gone = (xi1 < 0.0) | (xi1 >= self.nx)
        if np.any(gone):
            self.E_esc[s] += float(np.sum(P["w"][gone] * self.mass[s] * (g_new[gone] - 1.0)))
        keep = ~gone
        self.sp[s] = dict(xi=xi1[keep], u=u_new[keep], w=P["w"][keep])

    def advance_fields(self, Jx, Jy, Jz):
        """Yee update with J^{n+1/2}: B half step, guards, E full step, B half
        step; Poynting bookkeeping at both boundaries.  Jy, Jz are node arrays
        with one guard on each side (index node + 1); Jx is on half-nodes."""
        dt, a, n = self.dt, self.dt / self.dx, self.nx
        jy, jz = Jy[1:n + 2], Jz[1:n + 2]
        Ey0, Ez0 = self.Ey.copy(), self.Ez.copy()
        self.Bz[1:n + 1] -= 0.5 * a * (self.Ey[1:] - self.Ey[:-1])
        self.By[1:n + 1] += 0.5 * a * (self.Ez[1:] - self.Ez[:-1])
        t_half = (self.step_n + 0.5) * dt
        ey_in, ez_in = self.incident(t_half)
        d = 1.0 + a
        self.Bz[0] = (4.0 * ey_in - 2.0 * self.Ey[0] - (1.0 - a) * self.Bz[1] + dt * jy[0]) / d
        self.By[0] = (2.0 * self.Ez[0] - (1.0 - a) * self.By[1] - dt * jz[0] - 4.0 * ez_in) / d
        self.Bz[n + 1] = (2.0 * self.Ey[n] - (1.0 - a) * self.Bz[n] - dt * jy[n]) / d
        self.By[n + 1] = (-2.0 * self.Ez[n] - (1.0 - a) * self.By[n] + dt * jz[n]) / d
        self.Ey -= a * (self.Bz[1:] - self.Bz[:-1]) + dt * jy
        self.Ez += a * (self.By[1:] - self.By[:-1]) - dt * jz
        self.Ex -= dt * Jx
        # boundary fluxes at t_{n+1/2}: split into right- and left-going parts
        eyl, ezl = 0.5 * (Ey0[0] + self.Ey[0]), 0.5 * (Ez0[0] + self.Ez[0])
        bzl, byl = 0.5 * (self.Bz[0] + self.Bz[1]), 0.5 * (self.By[0] + self.By[1])
        eyr, ezr = 0.5 * (Ey0[n] + self.Ey[n]), 0.5 * (Ez0[n] + self.Ez[n])
        bzr, byr = 0.5 * (self.Bz[n] + self.Bz[n + 1]), 0.5 * (self.By[n] + self.By[n + 1])
        self.E_in += dt * (ey_in * ey_in + ez_in * ez_in)
        self.E_out_left += dt * 0.25 * ((eyl - bzl) ** 2 + (ezl + byl) ** 2)
        self.E_out_right += dt * 0.25 * ((eyr + bzr) ** 2 + (ezr - byr) ** 2)
        self.Bz[1:n + 1] -= 0.5 * a * (self.Ey[1:] - self.Ey[:-1])
        self.By[1:n + 1] += 0.5 * a * (self.Ez[1:] - self.Ez[:-1])

    def step(self):
        n = self.nx
        J = (np.zeros(n + 2), np.zeros(n + 3), np.zeros(n + 3))
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
        """(U_Ex, U_Etrans, U_B): sum of field^2 / 2 dx over [0, N dx] (nodes
        with trapezoid end weights, half-nodes 1..N)."""
        n, dx = self.nx, self.dx
        wn = np.ones(n + 1)
        wn[0] = wn[-1] = 0.5
        ue = 0.5 * dx * float(np.sum(wn * (self.Ey ** 2 + self.Ez ** 2)))
        ux = 0.5 * dx * float(np.sum(self.Ex[1:n + 1] ** 2))
        ub = 0.5 * dx * float(np.sum(self.By[1:n + 1] ** 2 + self.Bz[1:n + 1] ** 2))
        return ux, ue, ub

    def kinetic(self, s):
        P = self.sp[s]
        return float(np.sum(P["w"] * self.mass[s] * (gamma_of(P["u"]) - 1.0)))

    def gauss_residual(self):
        """max |(Ex[i+1/2] - Ex[i-1/2]) / dx - rho_i| over nodes 1..N-1."""
        n = self.nx
        rho = np.zeros(n + 3)
        for s in range(2):
            P = self.sp[s]
            c = np.floor(P["xi"]).astype(np.int64)
            o = P["xi"] - c
            rho += np.bincount(c + 1, weights=self.Z[s] * P["w"] * (1 - o), minlength=n + 3)
            rho += np.bincount(c + 2, weights=self.Z[s] * P["w"] * o, minlength=n + 3)
        rho /= self.dx
        res = (self.Ex[2:n + 1] - self.Ex[1:n]) / self.dx - rho[2:n + 1]
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
