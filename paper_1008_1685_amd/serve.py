"""Serving form: continuous batching of independent laser-foil runs.

``Batch`` wraps the C batch entry points (argument marshalling only).
``Server`` is the request loop: requests arrive over wall-clock time, are
admitted in arrival order while a batch slot and the device-memory budget
allow, are advanced together one captured quantum at a time, and are
retired (diagnostics, memory freed) as soon as they reach their step count.
"""
from __future__ import annotations

import collections
import ctypes as C
import time

import numpy as np

from . import _native as N
from .run import Run, workspace_bytes


class Batch:
    def __init__(self, precision: str = "fp32", max_slots: int = 64, quantum: int = 16,
                 max_particles: int = 4 * 10 ** 7, max_cells: int = 10 ** 6, stream=None):
        import torch

        self.lib = N.load()
        self.prec = N.PIC_FP64 if precision == "fp64" else N.PIC_FP32
        self.max_slots, self.quantum = int(max_slots), int(quantum)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        n = C.c_size_t()
        N.check(self.lib.pic_batch_workspace_bytes(self.prec, self.max_slots, C.byref(n)),
                "pic_batch_workspace_bytes")
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        self._h = C.c_void_p()
        N.check(self.lib.pic_batch_create(self.prec, self.max_slots, self.quantum, int(max_particles),
                                          int(max_cells), C.c_void_p(self.ws.data_ptr()),
                                          C.c_size_t(n.value), self._st(), C.byref(self._h)),
                "pic_batch_create")
        self._steps = (C.c_int64 * self.max_slots)()

    def _st(self):
        return C.c_void_p(self.stream.cuda_stream)

    def admit(self, run: Run, n_steps: int) -> int:
        slot = C.c_int32(-1)
        N.check(self.lib.pic_batch_admit(self._h, run._h, int(n_steps), self._st(), C.byref(slot)),
                "pic_batch_admit")
        return slot.value

    def fits(self, cfg: dict):
        """(now, ever): whether a run of ``cfg`` would be admitted at this
        moment, and whether it fits an empty batch at all."""
        from .run import make_config

        c = make_config(cfg)
        now, ever = C.c_int32(0), C.c_int32(0)
        N.check(self.lib.pic_batch_fits(self._h, C.byref(c), C.byref(now), C.byref(ever)),
                "pic_batch_fits")
        return bool(now.value), bool(ever.value)

    def step(self, n_quanta: int = 1):
        N.check(self.lib.pic_batch_step(self._h, int(n_quanta), self._st()), "pic_batch_step")

    def drain(self) -> int:
        """Advance every resident run to its step target; returns the number
        of quanta enqueued."""
        q = C.c_int64(0)
        N.check(self.lib.pic_batch_drain(self._h, C.byref(q), self._st()), "pic_batch_drain")
        return q.value

    def set_persistent(self, on):
        """Launch each quantum's steps as one persistent launch (True) or as
        one push and one field launch per step (False, the default); 2 is the
        persistent form with its barrier waits cut to zero (the error path)."""
        mode = on if isinstance(on, int) and not isinstance(on, bool) else (1 if on else 0)
        N.check(self.lib.pic_batch_set_persistent(self._h, mode), "pic_batch_set_persistent")

    def poll(self) -> np.ndarray:
        N.check(self.lib.pic_batch_poll(self._h, self._steps, self._st()), "pic_batch_poll")
        return np.frombuffer(self._steps, dtype=np.int64).copy()

    def poll_async(self):
        """Queue a poll of the step counters behind the queued replays."""
        N.check(self.lib.pic_batch_poll_async(self._h, self._st()), "pic_batch_poll_async")

    def poll_wait(self) -> np.ndarray:
        """Steps of the queued poll (-1: free, or admitted or released since)."""
        N.check(self.lib.pic_batch_poll_wait(self._h, self._steps), "pic_batch_poll_wait")
        return np.frombuffer(self._steps, dtype=np.int64).copy()

    def release(self, slot: int):
        N.check(self.lib.pic_batch_release(self._h, int(slot), self._st()), "pic_batch_release")

    def close(self):
        if self._h:
            self.lib.pic_batch_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_steps(cfg: dict) -> int:
    """Steps of a request: its periods at dt = cfl dx, dx = lambda / cells_per_lambda."""
    return int(round(cfg["periods"] * cfg["cells_per_lambda"] / cfg["cfl"]))


class Server:
    """Continuous-batching request loop over one or more Batches.

    budget_bytes bounds the summed run workspaces resident at once; quantum
    is the steps of one captured replay, and every request's sort_interval
    must equal it (the sort opens each replay); quanta_per_poll is how many
    captured quanta are enqueued between two checks for finished runs;
    persistent selects the batches' launch form (Batch.set_persistent).
    groups > 1 splits the max_slots slots over that
    many batches, each on a stream of its own: their launches overlap on the
    device, so one batch's short launches fill the ramp and tail of the
    other's.  A request joins the group with the least resident work that
    admits it.  The persistent form takes one group: its launch must have the
    device to itself."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, quantum: int = 16,
                 max_particles: int = 4 * 10 ** 7, max_cells: int = 2 * 10 ** 6,
                 quanta_per_poll: int = 2, precision: str = "fp32", persistent: bool = False,
                 groups: int = 1):
        self.budget = int(budget_bytes)
        if int(groups) < 1:
            raise ValueError("groups must be >= 1")
        if persistent and int(groups) > 1:
            # its work-groups wait for each other at grid barriers, so they
            # must all be resident at once, beside no other batch's launches
            raise ValueError("the persistent form runs as one group")
        groups = min(int(groups), int(max_slots))
        per = [max_slots // groups + (1 if g < max_slots % groups else 0) for g in range(groups)]
        self.batches = [Batch(precision, n, quantum, max_particles, max_cells) for n in per]
        for b in self.batches:
            b.set_persistent(persistent)
        self.quanta_per_poll = int(quanta_per_poll)
        self.peak_bytes = 0

    @property
    def batch(self):
        return self.batches[0]

    def serve(self, requests, keep_runs: bool = False, clock=time.perf_counter):
        """requests: list of dict(arrival=seconds, cfg=...), sorted by arrival.
        Returns one record per request: arrival, admitted, done, latency
        (seconds, wall clock from the start of serve), steps, particles and
        final diagnostics (and the Run itself with keep_runs)."""
        G = len(self.batches)
        pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
        queue = collections.deque()
        active = {}  # (group, slot) -> record
        load = [0] * G  # resident workspace bytes per group
        used = 0
        out = []
        inflight = [False] * G  # a poll is queued behind the group's replays
        t0 = clock()
        while pending or queue or active:
            now = clock() - t0
            while pending and pending[0]["arrival"] <= now:
                queue.append(pending.popleft())
            while queue:
                req = queue[0]
                need = workspace_bytes(req["cfg"])
                if used + need > self.budget and active:
                    break  # (a request larger than the whole budget runs alone)
                chosen, ever = None, False
                for g in sorted(range(G), key=lambda g: load[g]):
                    fits_now, fits_ever = self.batches[g].fits(req["cfg"])
                    ever = ever or fits_ever
                    if fits_now:
                        chosen = g
                        break
                if not ever:
                    raise ValueError(f"request {req['cfg'].get('name', '')!r} exceeds the batch's "
                                     "work capacity (max_particles / max_cells)")
                if chosen is None:
                    break
                # the request is admitted: only now is its memory set aside
                b = self.batches[chosen]
                run = Run(req["cfg"], stream=b.stream)
                steps = run_steps(req["cfg"])
                slot = b.admit(run, steps)
                queue.popleft()
                used += need
                load[chosen] += need
                self.peak_bytes = max(self.peak_bytes, used)
                active[(chosen, slot)] = dict(req=req, run=run, steps=steps, need=need,
                                              admitted=clock() - t0)
            if not active:
                for g in range(G):
                    if inflight[g]:
                        self.batches[g].poll_wait()
                        inflight[g] = False
                if pending:
                    time.sleep(max(0.0, pending[0]["arrival"] - (clock() - t0)))
                continue
            busy = {g for g, _ in active}
            # every busy group's next round is queued before the host waits
            # for the previous round's polls, so the device never idles on
            # the round trip
            for g in sorted(busy):
                self.batches[g].step(self.quanta_per_poll)
            done = []
            for g in range(G):
                if not (inflight[g] or g in busy):
                    continue
                b = self.batches[g]
                steps_now = b.poll_wait() if inflight[g] else None
                inflight[g] = g in busy
                if inflight[g]:
                    b.poll_async()
                if steps_now is not None:
                    done += [(g, s) for (gg, s), a in active.items()
                             if gg == g and 0 <= steps_now[s] and steps_now[s] >= a["steps"]]
            if not done:
                continue
            t_done = clock() - t0
            for key in done:
                g, slot = key
                a = active.pop(key)
                self.batches[g].release(slot)
                d = a["run"].diag(allow_nonfinite=True)
                rec = dict(name=a["req"]["cfg"].get("name", ""), arrival=a["req"]["arrival"],
                           admitted=a["admitted"], done=t_done,
                           latency=t_done - a["req"]["arrival"], steps=a["steps"],
                           particles=int(sum(a["run"].info["n_init"])), diag=d)
                if keep_runs:
                    rec["run"] = a["run"]
                else:
                    a["run"].close()
                out.append(rec)
                used -= a["need"]
                load[g] -= a["need"]
        for g in range(G):
            if inflight[g]:
                self.batches[g].poll_wait()
        return out
