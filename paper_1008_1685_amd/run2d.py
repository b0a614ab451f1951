"""Python handle over one 2D3V run of the C ABI in include/pic2d.h
(argument marshalling only; every computation runs in the library's kernels)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N

_CFG_KEYS = ("lambda_um", "cells_per_lambda", "ppc_x", "ppc_y", "box_x", "box_y", "cfl", "a0",
             "waist", "t_rise", "t_flat", "t_fall", "n0", "x_foil", "thickness", "mass_ratio",
             "sort_interval", "seed", "jitter")


FIELD_KERNELS = {"auto": 0, "tiles": 1, "strips": 2}


def make_config(cfg: dict, capacity: int = 0) -> N.Pic2dConfig:
    c = N.Pic2dConfig()
    c.struct_size = C.sizeof(N.Pic2dConfig)
    c.precision = N.PIC_FP64 if cfg.get("precision", "fp32") == "fp64" else N.PIC_FP32
    for k in _CFG_KEYS:
        setattr(c, k, type(getattr(c, k))(cfg[k]))
    c.pol = N.PIC_CP if cfg["pol"] == "CP" else N.PIC_LP
    c.rr = 1 if cfg["rr"] else 0
    c.rr_compensated = 1 if cfg.get("rr_compensated", True) else 0
    c.capacity = int(capacity)
    c.field_kernel = FIELD_KERNELS[cfg.get("field_kernel", "auto")]
    return c


def workspace_bytes(cfg: dict, capacity: int = 0) -> int:
    lib = N.load()
    c = make_config(cfg, capacity)
    n = C.c_size_t(0)
    N.check(lib.pic2d_workspace_bytes(C.byref(c), C.byref(n)), "pic2d_workspace_bytes")
    return int(n.value)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Run2D:
    """One 2D laser-foil run resident on the GPU."""

    FIELDS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")

    def __init__(self, cfg: dict, capacity: int = 0, device: str = "cuda"):
        import torch

        self.lib = N.load()
        self.cfg = dict(cfg)
        self._c = make_config(cfg, capacity)
        self.ws_bytes = workspace_bytes(cfg, capacity)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self._h = C.c_void_p()
        N.check(self.lib.pic2d_init(C.byref(self._c), C.c_void_p(self.ws.data_ptr()),
                                    C.c_size_t(self.ws_bytes), self._stream(), C.byref(self._h)),
                "pic2d_init")
        self.info = self.get_info()
        self.rdt = np.float32 if self.info["precision"] == N.PIC_FP32 else np.float64

    def _stream(self):
        import torch

        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def close(self):
        if self._h:
            self.lib.pic2d_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ stepping
    def step(self, n: int = 1):
        N.check(self.lib.pic2d_step(self._h, int(n), self._stream()), "pic2d_step")

    def push_deposit(self):
        N.check(self.lib.pic2d_push_deposit(self._h, self._stream()), "pic2d_push_deposit")

    def field_advance(self):
        N.check(self.lib.pic2d_field_advance(self._h, self._stream()), "pic2d_field_advance")

    def sort(self):
        N.check(self.lib.pic2d_sort(self._h, self._stream()), "pic2d_sort")

    # ------------------------------------------------------------ inspection
    def get_info(self) -> dict:
        o = N.Pic2dInfo()
        N.check(self.lib.pic2d_get_info(self._h, C.byref(o)), "pic2d_get_info")
        return dict(nx=o.nx, ny=o.ny, y_shift=o.y_shift, precision=o.precision, dx=o.dx, dt=o.dt,
                    eps_rr=o.eps_rr, w_ref=o.w_ref, capacity=o.capacity,
                    n_init=(o.n_init[0], o.n_init[1]), step=o.step, tile=o.tile,
                    lds_slots=o.lds_slots,
                    field_kernel={1: "tiles", 2: "strips"}.get(o.field_kernel, o.field_kernel),
                    field_blocks=o.field_blocks, sort_block_shift=(o.sort_block_x_shift,
                                                                   o.sort_block_y_shift))

    def diag(self) -> dict:
        o = N.PicDiagOut()
        N.check(self.lib.pic2d_diag(self._h, C.byref(o), self._stream()), "pic2d_diag")
        d = {k: getattr(o, k) for k, _ in N.PicDiagOut._fields_ if k != "reserved"}
        d["n_alive"] = (o.n_alive[0], o.n_alive[1])
        return d

    def _shapes(self):
        nx, ny = self.info["nx"], self.info["ny"]
        return dict(Ex=(nx + 2, ny), Ey=(nx + 1, ny), Ez=(nx + 1, ny), Bx=(nx + 1, ny),
                    By=(nx + 2, ny), Bz=(nx + 2, ny), Jx_int=(nx + 2, ny), Jy_int=(nx + 3, ny),
                    Jz_int=(nx + 3, ny), charge_int=(nx + 1, ny))

    def decode(self, cell):
        """(ix, iy) of cell indices."""
        c = np.asarray(cell, dtype=np.int64)
        sh = self.info["y_shift"]
        return c >> sh, c & ((1 << sh) - 1)

    def encode(self, ix, iy):
        return ((np.asarray(ix, np.int64) << self.info["y_shift"]) | np.asarray(iy, np.int64)).astype(np.int32)

    def get_state(self, particles: bool = True, residuals: bool = True) -> dict:
        """Fields (2D arrays [column, row]), currents, running charge and
        (unless particles=False) the alive particles."""
        self.info = self.get_info()
        cap, rdt = self.info["capacity"], self.rdt
        st = N.Pic2dState()
        keep = {}
        if particles:
            for s in range(2):
                arrs = dict(cell=np.empty(cap, np.int32))
                for k in ("ox", "oy", "ux", "uy", "uz", "w"):
                    arrs[k] = np.empty(cap, rdt)
                if s == 0 and residuals and self.cfg["rr"] and self.cfg.get("rr_compensated", True) \
                        and rdt == np.float32:
                    for k in ("rx", "ry", "rz"):
                        arrs[k] = np.empty(cap, np.float32)
                for k, a in arrs.items():
                    setattr(st.sp[s], k, _ptr(a))
                keep[s] = arrs
        grids = {}
        for k, shp in self._shapes().items():
            dt = np.int64 if k.endswith("_int") else rdt
            grids[k] = np.empty(shp, dt)
            setattr(st, k, _ptr(grids[k]))
        N.check(self.lib.pic2d_get_state(self._h, C.byref(st), self._stream()), "pic2d_get_state")
        res = dict(grids)
        res["step"] = st.step
        res["budget"] = N.budget_to_dict(st.budget)
        if particles:
            for s in range(2):
                cnt = st.sp[s].count
                res[f"sp{s}"] = {k: a[:cnt].copy() for k, a in keep[s].items()}
        return res

    def set_state(self, particles: dict | None = None, fields: dict | None = None,
                  step: int = -1, budget: dict | None = None):
        """particles: {0: {...}, 1: {...}} with cell, ox, oy, ux, uy, uz, w (+ rx, ry, rz);
        fields: any of Ex, Ey, Ez, Bx, By, Bz, Jx_int, Jy_int, Jz_int, charge_int;
        budget: the "budget" dict of get_state."""
        st = N.Pic2dState()
        keep = []
        for s in range(2):
            p = (particles or {}).get(s)
            if p is None:
                st.sp[s].count = 0
                continue
            st.sp[s].count = len(p["cell"])
            for k in ("cell", "ox", "oy", "ux", "uy", "uz", "w", "rx", "ry", "rz"):
                if k not in p:
                    continue
                if len(p[k]) != st.sp[s].count:
                    raise ValueError(f"species {s}: {k} has {len(p[k])} entries")
                dt = np.int32 if k == "cell" else (np.float32 if k in ("rx", "ry", "rz") else self.rdt)
                a = np.ascontiguousarray(p[k], dtype=dt)
                keep.append(a)
                setattr(st.sp[s], k, _ptr(a))
        shapes = self._shapes()
        for k, v in (fields or {}).items():
            if k not in shapes:
                raise KeyError(f"unknown field {k!r}")
            dt = np.int64 if k.endswith("_int") else self.rdt
            a = np.ascontiguousarray(v, dtype=dt)
            if a.shape != shapes[k]:
                raise ValueError(f"{k} must have shape {shapes[k]}, got {a.shape}")
            keep.append(a)
            setattr(st, k, _ptr(a))
        st.step = int(step)
        if budget is not None:
            st.budget = N.budget_from_dict(budget)
        N.check(self.lib.pic2d_set_state(self._h, C.byref(st), self._stream()), "pic2d_set_state")
        self.info = self.get_info()

    # ------------------------------------------------------------ timing
    def timing(self, period):
        N.check(self.lib.pic2d_timing_enable(self._h, int(period)), "pic2d_timing_enable")

    def timing_read(self):
        ms = (C.c_double * 3)()
        nl = (C.c_int64 * 3)()
        N.check(self.lib.pic2d_timing_read(self._h, ms, nl, self._stream()), "pic2d_timing_read")
        return {k: (ms[i], nl[i]) for i, k in enumerate(("push", "field", "sort"))}
