"""Python handle over one simulation run of the C ABI (argument marshalling only).

Device memory comes from torch (one uint8 workspace tensor per run) and
work is enqueued on torch's current HIP stream; every computation happens
in the library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N

_CFG_KEYS = ("lambda_um", "cells_per_lambda", "ppc", "box_lambda", "cfl", "a0", "t_rise",
             "t_flat", "t_fall", "n0", "x_foil", "thickness", "mass_ratio", "sort_interval",
             "seed", "jitter")


def make_config(cfg: dict, capacity: int = 0) -> N.PicConfig:
    c = N.PicConfig()
    c.struct_size = C.sizeof(N.PicConfig)
    c.precision = N.PIC_FP64 if cfg.get("precision", "fp32") == "fp64" else N.PIC_FP32
    for k in _CFG_KEYS:
        setattr(c, k, type(getattr(c, k))(cfg[k]))
    c.pol = N.PIC_CP if cfg["pol"] == "CP" else N.PIC_LP
    c.rr = 1 if cfg["rr"] else 0
    c.rr_compensated = 1 if cfg.get("rr_compensated", True) else 0
    c.capacity = int(capacity)
    return c


def workspace_bytes(cfg: dict, capacity: int = 0) -> int:
    lib = N.load()
    c = make_config(cfg, capacity)
    n = C.c_size_t(0)
    N.check(lib.pic_workspace_bytes(C.byref(c), C.byref(n)), "pic_workspace_bytes")
    return int(n.value)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Run:
    """One laser-foil run resident on the GPU."""

    def __init__(self, cfg: dict, capacity: int = 0, device: str = "cuda", workspace=None,
                 stream=None):
        """stream: a torch.cuda.Stream for every call of this run (default: the
        current stream at each call)."""
        import torch

        self.lib = N.load()
        self.stream = stream
        self.cfg = dict(cfg)
        self._c = make_config(cfg, capacity)
        self.ws_bytes = workspace_bytes(cfg, capacity)
        if workspace is None:
            if stream is not None:
                with torch.cuda.stream(stream):
                    workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
            else:
                workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        elif workspace.numel() * workspace.element_size() < self.ws_bytes:
            raise ValueError("workspace tensor too small")
        self.ws = workspace
        self._h = C.c_void_p()
        N.check(self.lib.pic_init(C.byref(self._c), C.c_void_p(self.ws.data_ptr()),
                                  C.c_size_t(self.ws_bytes), self._stream(), C.byref(self._h)),
                "pic_init")
        self.info = self.get_info()
        self.rdt = np.float32 if self.info["precision"] == N.PIC_FP32 else np.float64

    def _stream(self):
        import torch

        st = self.stream if self.stream is not None else torch.cuda.current_stream()
        return C.c_void_p(st.cuda_stream)

    def close(self):
        if self._h:
            self.lib.pic_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ stepping
    def step(self, n: int = 1):
        N.check(self.lib.pic_step(self._h, int(n), self._stream()), "pic_step")

    def push_deposit(self):
        N.check(self.lib.pic_push_deposit(self._h, self._stream()), "pic_push_deposit")

    def field_advance(self):
        N.check(self.lib.pic_field_advance(self._h, self._stream()), "pic_field_advance")

    def sort(self):
        N.check(self.lib.pic_sort(self._h, self._stream()), "pic_sort")

    def set_max_grid(self, max_workgroups: int):
        """Split the push and sort passes into launches of at most
        max_workgroups work-groups (0: one launch per pass)."""
        N.check(self.lib.pic_set_max_grid(self._h, int(max_workgroups)), "pic_set_max_grid")

    # ------------------------------------------------------------ inspection
    def get_info(self) -> dict:
        o = N.PicInfo()
        N.check(self.lib.pic_get_info(self._h, C.byref(o)), "pic_get_info")
        return dict(n_cells=o.n_cells, precision=o.precision, dx=o.dx, dt=o.dt, eps_rr=o.eps_rr,
                    w_ref=o.w_ref, capacity=o.capacity, n_init=(o.n_init[0], o.n_init[1]),
                    step=o.step, tile=o.tile, lds_slots=o.lds_slots)

    def diag(self, allow_nonfinite: bool = False) -> dict:
        o = N.PicDiagOut()
        st = self.lib.pic_diag(self._h, C.byref(o), self._stream())
        if not (allow_nonfinite and st == N.PIC_ENONFINITE):
            N.check(st, "pic_diag")
        d = {k: getattr(o, k) for k, _ in N.PicDiagOut._fields_ if k != "reserved"}
        d["n_alive"] = (o.n_alive[0], o.n_alive[1])
        return d

    def has_residuals(self) -> bool:
        return (self.rdt == np.float32 and bool(self.cfg["rr"])
                and bool(self.cfg.get("rr_compensated", True)))

    def get_state(self, residuals: bool = True, particles: bool = True) -> dict:
        """Fields, currents and (unless particles=False) the alive particles."""
        info = self.get_info()
        n, cap, rdt = info["n_cells"], info["capacity"], self.rdt
        if not particles:
            cap = 0
        st = N.PicState()
        out = {}
        keep = []
        for s in range(2):
            if not particles:
                out[s] = {}
                continue
            arrs = dict(cell=np.empty(cap, np.int32), off=np.empty(cap, rdt), ux=np.empty(cap, rdt),
                        uy=np.empty(cap, rdt), uz=np.empty(cap, rdt), w=np.empty(cap, rdt))
            # residuals exist for FP32 electrons under compensated RR only
            if s == 0 and residuals and self.has_residuals():
                for k in ("rx", "ry", "rz"):
                    arrs[k] = np.empty(cap, np.float32)
            sp = st.sp[s]
            for k, a in arrs.items():
                setattr(sp, k, _ptr(a))
            out[s] = arrs
            keep.append(arrs)
        f = dict(Ex=np.empty(n + 2, rdt), Ey=np.empty(n + 1, rdt), Ez=np.empty(n + 1, rdt),
                 By=np.empty(n + 2, rdt), Bz=np.empty(n + 2, rdt), Ex_int=np.empty(n + 2, np.int64),
                 Jx_int=np.empty(n + 2, np.int64), Jy_int=np.empty(n + 3, np.int64),
                 Jz_int=np.empty(n + 3, np.int64))
        for k, a in f.items():
            setattr(st, k, _ptr(a))
        N.check(self.lib.pic_get_state(self._h, C.byref(st), self._stream()), "pic_get_state")
        res = dict(f)
        res["step"] = st.step
        res["budget"] = N.budget_to_dict(st.budget)
        if particles:
            for s in range(2):
                cnt = st.sp[s].count
                res[f"sp{s}"] = {k: a[:cnt].copy() for k, a in out[s].items()}
        return res

    def get_particles(self, species: int, first: int, count: int, residuals: bool = False,
                      keys=("cell", "off", "ux", "uy", "uz", "w")) -> dict:
        """Raw slots first .. first + count - 1 of a species (no compaction;
        removed particles have cell = INT32_MIN); stable between sorts."""
        rdt = self.rdt
        dt = dict(cell=np.int32, off=rdt, ux=rdt, uy=rdt, uz=rdt, w=rdt)
        arrs = {k: np.empty(count, dt[k]) for k in keys}
        if residuals and species == 0 and self.has_residuals():
            for k in ("rx", "ry", "rz"):
                arrs[k] = np.empty(count, np.float32)
        sp = N.PicSpeciesState()
        for k, a in arrs.items():
            setattr(sp, k, _ptr(a))
        N.check(self.lib.pic_get_particles(self._h, int(species), int(first), int(count), C.byref(sp),
                                           self._stream()), "pic_get_particles")
        return {k: a[: sp.count] for k, a in arrs.items()}

    def set_state(self, particles: dict | None = None, fields: dict | None = None,
                  step: int = -1, budget: dict | None = None):
        """particles: {0: {...}, 1: {...}} with cell, off, ux, uy, uz, w (+ rx, ry, rz);
        fields: any of Ex, Ey, Ez, By, Bz, Ex_int, Jx_int, Jy_int, Jz_int; budget: the
        "budget" dict of get_state (cumulative budget terms and the non-finite flag)."""
        st = N.PicState()
        keep = []
        for s in range(2):
            sp = st.sp[s]
            p = (particles or {}).get(s)
            if p is None:
                sp.count = 0
                continue
            sp.count = len(p["cell"])
            for k in ("cell", "off", "ux", "uy", "uz", "w", "rx", "ry", "rz"):
                if k not in p:
                    continue
                if len(p[k]) != sp.count:
                    raise ValueError(f"species {s}: {k} has {len(p[k])} entries, cell has {sp.count}")
                dt = np.int32 if k == "cell" else (np.float32 if k in ("rx", "ry", "rz") else self.rdt)
                a = np.ascontiguousarray(p[k], dtype=dt)
                keep.append(a)
                setattr(sp, k, _ptr(a))
        n = self.info["n_cells"]
        need = dict(Ex=n + 2, Ey=n + 1, Ez=n + 1, By=n + 2, Bz=n + 2, Ex_int=n + 2,
                    Jx_int=n + 2, Jy_int=n + 3, Jz_int=n + 3)
        for k, v in (fields or {}).items():
            if k not in need:
                raise KeyError(f"unknown field {k!r}")
            dt = np.int64 if k in ("Ex_int", "Jx_int", "Jy_int", "Jz_int") else self.rdt
            a = np.ascontiguousarray(v, dtype=dt)
            if a.shape != (need[k],):
                raise ValueError(f"{k} must have shape ({need[k]},), got {a.shape}")
            keep.append(a)
            setattr(st, k, _ptr(a))
        st.step = int(step)
        if budget is not None:
            st.budget = N.budget_from_dict(budget)
        N.check(self.lib.pic_set_state(self._h, C.byref(st), self._stream()), "pic_set_state")

    def spectrum(self, bins: int, e_max_mev: float) -> np.ndarray:
        h = np.zeros(bins, np.float64)
        N.check(self.lib.pic_spectrum(self._h, int(bins), float(e_max_mev),
                                      h.ctypes.data_as(C.POINTER(C.c_double)), self._stream()),
                "pic_spectrum")
        return h

    def friction(self, bins: int, log10_lo: float, log10_hi: float):
        """Friction coefficient d of every electron (Eq. (damping)): its
        histogram in log10 d (electron weight per bin) and dict(max, mean,
        below, above) (mean weighted; below/above: weight outside the range)."""
        h = np.zeros(bins, np.float64)
        st = np.zeros(4, np.float64)
        N.check(self.lib.pic_friction(self._h, int(bins), float(log10_lo), float(log10_hi),
                                      h.ctypes.data_as(C.POINTER(C.c_double)),
                                      st.ctypes.data_as(C.POINTER(C.c_double)), self._stream()),
                "pic_friction")
        return h, dict(max=st[0], mean=st[1], below=st[2], above=st[3])

    def spectrum_static(self, bins: int, e_max_mev: float) -> np.ndarray:
        """As spectrum(), through the entry point that keeps its counters in
        the library's fixed device array (no device memory of its own)."""
        h = np.zeros(bins, np.float64)
        N.check(self.lib.pic_spectrum_static(self._h, int(bins), float(e_max_mev),
                                             h.ctypes.data_as(C.POINTER(C.c_double)), self._stream()),
                "pic_spectrum_static")
        return h

    # ------------------------------------------------------------ timing
    def timing(self, period):
        """Time every ``period``-th launch of each kernel kind (True: every
        launch, False or 0: off)."""
        N.check(self.lib.pic_timing_enable(self._h, int(period)), "pic_timing_enable")

    def timing_read(self):
        ms = (C.c_double * 3)()
        nl = (C.c_int64 * 3)()
        N.check(self.lib.pic_timing_read(self._h, ms, nl, self._stream()), "pic_timing_read")
        return {k: (ms[i], nl[i]) for i, k in enumerate(("push", "field", "sort"))}
