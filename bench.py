"""Throughput benchmark of the PIC hot path on one MI355X.

One step = push-deposit (gather, Boris, RR, move, integer deposit), field
advance, the periodic cell sort, and (every --diag-every steps) the FP64
energy budget and Gauss check.  Prints one JSON line.

Workload (default): laser-foil run at the precision-form scale - LP a0 = 500,
200 cells per wavelength, 100 wavelengths (20,000 cells), hydrogen foil of
1 wavelength at n0 = 100 n_c with 25,000 particles per cell per species
(1e7 particles), FP32 particles with compensated RR, FP64 reductions.

Timed window.  Every timed run is first stepped, untimed, to 10 laser
periods (4,000 steps; the pulse reaches the foil after 8 periods), so the
window lies inside the laser-foil interaction whatever --steps and --warmup
are; --warmup adds steps on top.  The cell sort runs every I steps (I = 64),
and a sort costs more than its own kernel: the push after it has no cell
ranges from the previous push and scans its tiles first.  The headline
window therefore charges the sort at its configured rate, 1/I per step,
from the same run: with s0 the first sort step after the lead-in and
m = I/2, the wall time of the m steps [s0 - m, s0) (no sort) and of the m
steps [s0, s0 + m) (one sort) give the cost of one sort, C; the K timed steps
[s0 + m, s0 + m + K) hold n sorts; the time per step is
(wall - n C + (K/I) C) / K.  The raw wall time is reported beside it.  Side
runs time whole sort intervals that open with a sort, which hold the
configured share of sorts by themselves.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# per-kernel durations come from HIP events recorded by every
# TIMING_PERIOD-th launch of each kernel kind at its start and end
TIMING_PERIOD = 8


KERNEL_SOURCES = {"k_push": ("kernels.hpp", "pic_lib.hip"),
                  "k_push2": ("kernels.hpp", "kernels2d.hpp", "pic2d_host.inc")}


def kernel_hash(kernel: str = "k_push") -> str:
    """SHA-256 of the device source a push kernel is built from."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_1008_1685_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def stored_traffic(path: str, workload: str, kernel: str):
    """HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (calibrated
    on a plain copy), only for the kernel source the counters were taken on."""
    if not os.path.exists(path):
        return None
    try:
        tj = json.load(open(path))
        if tj.get("workload") == workload and tj.get("kernel_sha256") == kernel_hash(kernel):
            return tj.get("bytes_per_launch")
    except Exception:
        pass
    return None


def alg_bytes_per_push(precision: str, compensated: bool, rr: bool):
    """Algorithmic HBM bytes of one push (electron, ion): read cell, offset,
    3 momenta, weight; write cell, offset, 3 momenta; compensated RR also
    reads and writes 3 FP32 residuals per electron."""
    r = 4 if precision == "fp32" else 8
    ion = (4 + 5 * r) + (4 + 4 * r)
    ele = ion + (24 if (precision == "fp32" and compensated and rr) else 0)
    return ele, ion


# untimed lead-in of every timed run: into the laser-foil interaction
T_START_PERIODS = 10.0


def window_start(cfg, warmup, t_start=T_START_PERIODS):
    """First timed step: t_start periods plus `warmup` steps, rounded up to a
    step at which the cell sort runs (multiples of the sort interval)."""
    from workloads import periods_to_steps

    lead = periods_to_steps(dict(cfg, periods=t_start)) + max(int(warmup), 0)
    k = cfg["sort_interval"]
    return -(-lead // k) * k


def sorts_in_window(start, steps, interval):
    """Sorts that run inside steps [start, start + steps): one at the start of
    every step that is a positive multiple of the sort interval."""
    first = max(start, 1)
    return max((start + steps - 1) // interval - (first - 1) // interval, 0)


def time_run(cfg, steps, warmup, diag_every, timing=TIMING_PERIOD, t_start=T_START_PERIODS,
             keep_state=False, sort_cost=False):
    """Time `steps` steps of `cfg` after the lead-in to t_start periods plus
    `warmup` steps.  sort_cost=False: the window opens at a sort step and its
    wall time is taken as is.  sort_cost=True: the sort is charged at
    1/sort_interval per step with its cost measured in the same run (the
    module docstring)."""
    import torch

    from paper_1008_1685_amd import Run

    run = Run(cfg)
    interval = cfg["sort_interval"]
    s0 = window_start(cfg, warmup, t_start)
    m = max(interval // 2, 1)

    def wall(k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        run.step(k)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    # host-side work (diagnostics, the state copy) comes before the last untimed
    # steps, so the device is busy again when the window opens
    if sort_cost:
        run.step(s0 - m)
        d0 = run.diag()
        state = run.get_state() if keep_state else None
        t_plain = wall(m)   # [s0 - m, s0): no sort
        t_sort = wall(m)    # [s0, s0 + m): the sort at s0 and the push after it
        c_sort = max(t_sort - t_plain, 0.0)
        start = s0 + m
    else:
        run.step(s0 - m)
        d0 = run.diag()
        state = run.get_state() if keep_state else None
        run.step(m)
        c_sort = None
        start = s0
    torch.cuda.synchronize()
    run.timing(timing)
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(diag_every, steps - done)
        run.step(k)
        done += k
        if done % diag_every == 0 and done < steps:
            run.diag()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = run.timing_read()
    run.timing(0)
    d1 = run.diag()
    n_e = 0.5 * (d0["n_alive"][0] + d1["n_alive"][0])
    n_i = 0.5 * (d0["n_alive"][1] + d1["n_alive"][1])
    sorts = sorts_in_window(start, steps, interval)
    raw = t1 - t0
    seconds = raw if c_sort is None else raw - sorts * c_sort + steps / interval * c_sort
    out = dict(seconds=seconds, raw_seconds=raw, sorts_in_window=sorts, sort_cost_s=c_sort,
               start=start, n_e=n_e, n_i=n_i, kernels=kt, diag0=d0, diag1=d1,
               info=run.get_info(), state=state)
    run.close()
    del run
    torch.cuda.empty_cache()
    return out


def pushes_per_s(r, steps):
    return (r["n_e"] + r["n_i"]) * steps / r["seconds"]


def alg_bytes_per_push_2d(precision: str, compensated: bool, rr: bool):
    """As alg_bytes_per_push with the second offset: read cell, 2 offsets, 3
    momenta, weight; write cell, 2 offsets, 3 momenta (+ 24 B of residuals
    per compensated FP32 electron)."""
    r = 4 if precision == "fp32" else 8
    ion = (4 + 6 * r) + (4 + 5 * r)
    ele = ion + (24 if (precision == "fp32" and compensated and rr) else 0)
    return ele, ion


def time_run_2d(cfg, steps, warmup, timing=TIMING_PERIOD):
    import torch

    from paper_1008_1685_amd.run2d import Run2D

    run = Run2D(cfg)
    run.step(warmup)
    d0 = run.diag()
    torch.cuda.synchronize()
    run.timing(timing)
    t0 = time.perf_counter()
    run.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = run.timing_read()
    run.timing(0)
    d1 = run.diag()
    out = dict(seconds=t1 - t0, n_e=0.5 * (d0["n_alive"][0] + d1["n_alive"][0]),
               n_i=0.5 * (d0["n_alive"][1] + d1["n_alive"][1]), kernels=kt, diag1=d1,
               info=run.get_info())
    run.close()
    del run
    torch.cuda.empty_cache()
    return out


def bench_2d(warmup=1280, steps=400, side_runs=True, traffic_json=None):
    """The 2D3V form (2,560 x 1,024 cells, 8.4e6 particles, LP a0 = 500 with
    a 4-wavelength waist), timed from the pulse's arrival at the foil: one
    step = push-deposit, the field advance, the cell sort every 24 steps.
    The push kernel's roofline is reported as for the 1D path."""
    from workloads import preset2d

    cfg = preset2d("d2")
    r = time_run_2d(cfg, steps, warmup)
    value = (r["n_e"] + r["n_i"]) * steps / r["seconds"]
    be, bi = alg_bytes_per_push_2d(cfg["precision"], cfg["rr_compensated"], cfg["rr"])
    push_ms, push_n = r["kernels"]["push"]
    avg = push_ms * 1e-3 / max(push_n, 1)
    nbytes = be * r["n_e"] + bi * r["n_i"]
    out = dict(workload=f"d2: 2D3V, LP a0={cfg['a0']:g} waist {cfg['waist']:g} wavelengths, "
                        f"{r['info']['nx']} x {r['info']['ny']} cells, "
                        f"{int(r['n_e'] + r['n_i'])} particles, fp32 + compensated RR",
               pushes_per_s=value, ms_per_step=r["seconds"] * 1e3 / steps, steps=steps,
               warmup=warmup,
               roofline=dict(bound="hbm", achieved=nbytes / avg / 1e9, peak=PEAK_HBM_GBS, unit="GB/s",
                             frac=nbytes / avg / 1e9 / PEAK_HBM_GBS, kernel="k_push2",
                             traffic=stored_traffic(traffic_json or os.path.join(
                                 ROOT, "profiles", "traffic_d2.json"), "d2", "k_push2"),
                             bytes_per_launch=nbytes, avg_launch_us=avg * 1e6,
                             alg_bytes_per_push=dict(electron=be, ion=bi)),
               kernel_us_per_launch={k: v[0] * 1e3 / max(v[1], 1) for k, v in r["kernels"].items()},
               gauss_int=r["diag1"]["gauss_int"], gauss=r["diag1"]["gauss"],
               energy_balance=r["diag1"]["balance"] / max(r["diag1"]["E_in"], 1e-300))
    if not side_runs:
        return out
    side = max(steps // 2, 100)
    r_off = time_run_2d(dict(cfg, rr=False), side, warmup, timing=0)
    r_64 = time_run_2d(dict(cfg, precision="fp64"), side, warmup, timing=0)
    v_off = (r_off["n_e"] + r_off["n_i"]) * side / r_off["seconds"]
    v_64 = (r_64["n_e"] + r_64["n_i"]) * side / r_64["seconds"]
    out["rr_cost"] = dict(pushes_per_s_rr_off=v_off, overhead=v_off / value - 1.0)
    out["fp64_path"] = dict(pushes_per_s=v_64, speedup_fp32_over_fp64=value / v_64)
    return out


def side_by_side_c2(warmup=3200, steps=2000):
    """The plain method at scale (12,000 cells, 4e5 particles, LP a0 = 300):
    FP32 and FP64, RR on and off, each timed over the same window at the
    start of the laser-foil interaction."""
    out = {}
    from workloads import preset

    for prec in ("fp64", "fp32"):
        for rr in (True, False):
            cfg = preset("c2", precision=prec, rr=rr)
            r = time_run(cfg, steps, warmup, steps, t_start=0.0)
            out[f"{prec}_rr_{'on' if rr else 'off'}"] = pushes_per_s(r, steps)
    out["speedup_fp32_over_fp64"] = out["fp32_rr_on"] / out["fp64_rr_on"]
    out["rr_overhead_fp64"] = out["fp64_rr_off"] / out["fp64_rr_on"] - 1.0
    out["workload"] = "c2: LP a0=300, 12000 cells, 400000 particles, steps 3200-5200, pushes/s"
    return out


def copy_ceiling(nbytes=2 ** 31, reps=20):
    """The measured STREAM-copy ceiling of the roofline: GB/s (bytes read +
    bytes written) of a plain device copy of `nbytes` by the hand-written
    copy kernel (libstreamcopy.so, one 16-byte element per thread), and for
    comparison by torch's copy_, each timed with events over `reps` copies
    after three untimed ones."""
    import ctypes as C

    import torch

    path = os.path.join(ROOT, "paper_1008_1685_amd", "libstreamcopy.so")
    if not os.path.exists(path):  # a measurement aid: built here when missing
        from paper_1008_1685_amd.build import build_stream_copy
        build_stream_copy()
    lib = C.CDLL(path)
    lib.stream_copy.restype = C.c_int
    lib.stream_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    a = torch.arange(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()

    def hip_copy():
        rc = lib.stream_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), nbytes,
                             C.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"stream_copy failed ({rc})")

    def gbs(copy):
        for _ in range(3):
            copy()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            copy()
        e1.record()
        e1.synchronize()
        return 2 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9

    b.zero_()
    hip = gbs(hip_copy)
    if not torch.equal(a, b):
        raise RuntimeError("stream_copy copied wrong data")
    ref = gbs(lambda: b.copy_(a))
    del a, b
    torch.cuda.empty_cache()
    return dict(gbs=hip, torch_copy_gbs=ref,
                what=f"device copy of {nbytes / 2 ** 30:g} GiB by stream_copy (one 16-byte element per "
                     f"thread), read + written bytes over the mean of {reps} copies")


def small_runs():
    """Whole runs of the small workloads through pic_step (two sort intervals
    per graph replay): c1 (12,800 particles, 2,000 cells, 6,000 steps) and
    c1w (102,400 particles), wall clock from the first step to the last;
    launch latency, not bandwidth, bounds them."""
    import torch

    from paper_1008_1685_amd import Run
    from workloads import periods_to_steps, preset

    out = {}
    for name in ("c1", "c1w"):
        cfg = preset(name)
        n = periods_to_steps(cfg)
        run = Run(cfg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.step(n)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        d = run.diag()
        pushes = 0.5 * (sum(run.get_info()["n_init"]) + sum(d["n_alive"])) * n  # (few leave)
        out[name] = dict(pushes_per_s=pushes / dt, us_per_step=dt / n * 1e6, steps=n,
                         particles=int(sum(run.get_info()["n_init"])), alive_end=list(d["n_alive"]))
        run.close()
    return out


def cpu_baseline(cfg, state, budget_s=20.0, max_steps=12):
    """The FP64 oracle, as is, on a bounded sample of the same workload: a few
    steps from the state at which the GPU's timed window starts (particles,
    fields and the laser clock taken from the GPU run, promoted to FP64)."""
    import numpy as np

    from oracle import pic as opic

    sim = opic.Pic1D(cfg, init_particles=False)
    for k in ("Ex", "Ey", "Ez", "By", "Bz"):
        getattr(sim, k)[:] = np.asarray(state[k], dtype=np.float64)
    for s in range(2):
        p = state[f"sp{s}"]
        u = np.stack([np.asarray(p[k], np.float64) for k in ("ux", "uy", "uz")], 1)
        sim.set_particles(s, p["cell"], p["off"], u, p["w"])
    sim.step_n = int(state["step"])
    n = sim.sp[0]["xi"].size + sim.sp[1]["xi"].size
    t0 = time.perf_counter()
    rates = []  # each step is one repetition
    pushes = 0
    while len(rates) < max_steps and (len(rates) < 3 or (time.perf_counter() - t0) < budget_s):
        m = sim.sp[0]["xi"].size + sim.sp[1]["xi"].size
        ts = time.perf_counter()
        sim.step()
        rates.append(m / (time.perf_counter() - ts))
        pushes += m
    dt = time.perf_counter() - t0
    k = len(rates)
    t_p = int(state["step"]) * sim.dt / (2.0 * 3.141592653589793)
    return dict(value=float(np.median(rates)), unit="pushes/s", cores=1, host_cpu_count=os.cpu_count(),
                kind="oracle", repetitions=k, mean=pushes / dt,
                sample=f"{k} oracle steps ({pushes} pushes, {dt:.1f} s) from the GPU run's state at "
                       f"step {int(state['step'])} (t = {t_p:.2f} periods, {n} particles), "
                       "where the timed window starts; the median of the steps' rates; numpy, "
                       "one thread")


# batches the serving slots are split over (streams of their own); the
# persistent form and the stress run's co-scheduling use one
SERVE_GROUPS = 3
# steps per captured quantum of the serving batch: the requests' sort interval
SERVE_QUANTUM = 32


def serve_bench(n_runs=256, rate=20.0, seed=0, max_slots=64, budget_gb=64.0, persistent=False,
                groups=SERVE_GROUPS, saturated=False):
    """Serving form: a Poisson stream of independent laser-foil requests
    (a0, polarisation, density, thickness, size and length randomised),
    continuously batched; latency = completion - arrival.  persistent: each
    quantum's steps as one persistent launch rather than a push and a field
    launch per step; groups: the slots split over that many batches on
    streams of their own; saturated: every request queued at time 0 (the
    batch's throughput with no idle slot, rather than the stream's latency)."""
    import numpy as np

    from paper_1008_1685_amd.serve import Server, run_steps
    from workloads import poisson_stream

    if persistent:
        groups = 1  # the persistent launch needs the device to itself
    reqs = poisson_stream(seed, n_runs=n_runs, rate=rate)
    if saturated:
        reqs = [dict(r, arrival=0.0) for r in reqs]
    max_p = max(2 * r["cfg"]["ppc"] * round(r["cfg"]["thickness"] * r["cfg"]["cells_per_lambda"])
                for r in reqs)
    max_c = max(round(r["cfg"]["box_lambda"] * r["cfg"]["cells_per_lambda"]) for r in reqs)
    srv = Server(budget_bytes=int(budget_gb * 2 ** 30), max_slots=max_slots, quantum=SERVE_QUANTUM,
                 max_particles=max_slots * max_p, max_cells=max_slots * (max_c + 8),
                 persistent=persistent, groups=groups)
    t0 = time.perf_counter()
    recs = srv.serve(reqs)
    wall = time.perf_counter() - t0
    lat = np.array([r["latency"] for r in recs])
    pushes = sum(r["particles"] * r["steps"] for r in recs)
    # algorithmic bytes of those pushes (electrons and ions in equal numbers)
    be, bi = alg_bytes_per_push("fp32", True, True)
    bad = sum(1 for r in recs if r["diag"]["gauss_int"] != 0 or r["diag"]["nonfinite"])
    return dict(workload=f"{n_runs} Poisson requests at {rate:g}/s (seed {seed}); a0 U[50,500], "
                         "LP/CP, n0 U[50,150], thickness U[0.5,2], 1e4-1e6 particles, 30-80 periods",
                requests=len(recs), p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()), wall_s=wall,
                pushes=float(pushes), pushes_per_s=pushes / wall,
                push_bytes_per_s_frac=pushes / wall * (be + bi) / 2 / (PEAK_HBM_GBS * 1e9),
                peak_resident_bytes=srv.peak_bytes, max_slots=max_slots, groups=len(srv.batches),
                failed_checks=bad,
                launch_form="one persistent launch per quantum" if persistent
                else "a push and a field launch per step")


def stress_bench(serve_kwargs, t_start=8.5, window=200, chunk=8, max_grid=512):
    """The stress run (2e8 particles, 80,000 cells, LP a0 = 800), stepped from
    the pulse's arrival at the foil on a stream of its own, its push and sort
    passes split into launches of at most `max_grid` work-groups
    (pic_set_max_grid; 0: whole passes): its throughput alone, then while a
    second host thread steps it without pause and the serving stream is
    served on the same GPU.  Both streams have the default priority; the
    requests' kernels are dispatched between the stress run's pieces."""
    import threading

    import torch

    from paper_1008_1685_amd import Run
    from workloads import preset

    cfg = preset("c5")
    st = torch.cuda.Stream()
    run = Run(cfg, stream=st)
    run.set_max_grid(max_grid)
    n = sum(run.get_info()["n_init"])
    warm = window_start(cfg, 0, t_start)  # the pulse reaches the foil after 8 periods
    run.step(warm)
    st.synchronize()
    t0 = time.perf_counter()
    run.step(window)
    st.synchronize()
    alone = n * window / (time.perf_counter() - t0)
    stop = threading.Event()
    done = [0]

    def loop():
        while not stop.is_set():
            run.step(chunk)
            st.synchronize()
            done[0] += chunk

    th = threading.Thread(target=loop, daemon=True)
    t1 = time.perf_counter()
    th.start()
    try:
        serving = serve_bench(**serve_kwargs)
    finally:
        stop.set()
        th.join()
    el = time.perf_counter() - t1
    d = run.diag()
    run.close()
    return dict(workload=f"c5: LP a0={cfg['a0']:g}, {run.info['n_init'][0] + run.info['n_init'][1]} particles, "
                         f"80000 cells, fp32 + compensated RR, stepped from step {warm} "
                         f"({warm / 800:.2f} periods, in the laser-foil interaction)",
                max_grid=max_grid, pushes_per_s_alone=alone,
                pushes_per_s_with_serving=n * done[0] / el,
                share=n * done[0] / el / alone,  # the stress run's rate beside the requests / alone
                steps_with_serving=done[0],
                gauss_int=d["gauss_int"], serving_under_load=serving)


def write_traffic(fetch, write, cfetch, cwrite, out_path, kernel="k_push", workload="c3",
                  match="k_push", last=50):
    """A traffic record (profiles/traffic.json, profiles/traffic_d2.json) from
    rocprofv3 counter_collection.csv files: FETCH_SIZE and WRITE_SIZE of the
    last `last` launches whose name contains `match` (c3: the 50 timed steps of
    --steps 50 --warmup 0 --no-side-runs --no-serve; d2: the 400 timed steps of
    --only-2d --no-side-runs) and of a plain 1 GiB device copy (torch
    b.copy_(a), the calibration of bytes reported per byte moved)."""
    import csv

    import numpy as np

    def kib(path, name, last=50):
        rows = [r for r in csv.DictReader(open(path)) if name in r["Kernel_Name"]]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return float(np.mean([float(r["Counter_Value"]) for r in rows][-last:])), len(rows)

    f_copy, _ = kib(cfetch, "copyBuffer")
    w_copy, _ = kib(cwrite, "copyBuffer")
    f_factor, w_factor = 2 ** 30 / (f_copy * 1024), 2 ** 30 / (w_copy * 1024)
    f_push, nf = kib(fetch, match, last)
    w_push, nw = kib(write, match, last)
    out = dict(workload=workload, kernel=kernel, kernel_sha256=kernel_hash(kernel),
               fetch_kib=f_push, write_kib=w_push, fetch_factor=f_factor, write_factor=w_factor,
               read_bytes=f_push * 1024 * f_factor, write_bytes=w_push * 1024 * w_factor,
               bytes_per_launch=f_push * 1024 * f_factor + w_push * 1024 * w_factor,
               launches_averaged=min(last, nf, nw))
    json.dump(out, open(out_path, "w"), indent=1)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=0,
                    help="steps on top of the untimed lead-in to 10 periods")
    ap.add_argument("--diag-every", type=int, default=1000)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-side-runs", action="store_true",
                    help="skip the RR-off and FP64 comparison runs and the CPU baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-form measurement")
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the stress run and the serving measurement under its load")
    ap.add_argument("--stress-only", type=int, default=0, metavar="N",
                    help="only run the stress run with the first N serving requests beside it")
    ap.add_argument("--stress-grid", type=int, default=512,
                    help="work-groups per launch of the stress run's push and sort passes (0: whole)")
    ap.add_argument("--only-2d", action="store_true",
                    help="only run the 2D3V measurement (with --no-side-runs: without its RR-off "
                         "and FP64 runs)")
    ap.add_argument("--traffic-2d", action="store_true",
                    help="with --write-traffic: the 2D push kernel on d2 (profiles/traffic_d2.json)")
    ap.add_argument("--serve-only", type=int, default=0, metavar="N",
                    help="only run the serving measurement, on the first N requests")
    ap.add_argument("--serve-persistent", action="store_true",
                    help="with --serve-only: each quantum's steps as one persistent launch")
    ap.add_argument("--serve-saturated", action="store_true",
                    help="with --serve-only: every request queued at time 0")
    ap.add_argument("--serve-groups", type=int, default=SERVE_GROUPS, metavar="G",
                    help="with --serve-only: the slots split over G batches on streams of their own")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                         "COPY_WRITE_CSV"),
                    help="write --traffic-json from rocprofv3 counter files and exit")
    args = ap.parse_args()
    if args.write_traffic:
        if args.traffic_2d:
            path = args.traffic_json
            if path == os.path.join(ROOT, "profiles", "traffic.json"):
                path = os.path.join(ROOT, "profiles", "traffic_d2.json")
            write_traffic(*args.write_traffic, path, kernel="k_push2", workload="d2",
                          match="k_push2<float>", last=400)
        else:
            write_traffic(*args.write_traffic, args.traffic_json)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU particle decomposition is a design note, not built)", flush=True)
        sys.exit(2)

    import torch

    from workloads import preset

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.serve_only:
        print(json.dumps(dict(serving=serve_bench(n_runs=args.serve_only,
                                                  persistent=args.serve_persistent,
                                                  groups=args.serve_groups,
                                                  saturated=args.serve_saturated))), flush=True)
        return
    if args.only_2d:
        print(json.dumps(dict(pic2d=bench_2d(side_runs=not args.no_side_runs))), flush=True)
        return
    if args.stress_only:
        print(json.dumps(dict(stress=stress_bench(dict(n_runs=args.stress_only, groups=1),
                                                     max_grid=args.stress_grid))),
              flush=True)
        return
    cfg = preset(args.workload)
    res = time_run(cfg, args.steps, args.warmup, args.diag_every,
                   keep_state=not args.no_side_runs, sort_cost=True)
    value = pushes_per_s(res, args.steps)
    be, bi = alg_bytes_per_push(cfg["precision"], cfg["rr_compensated"], cfg["rr"])
    push_ms, push_n = res["kernels"]["push"]
    avg_push_s = push_ms * 1e-3 / max(push_n, 1)
    bytes_per_launch = be * res["n_e"] + bi * res["n_i"]
    achieved = bytes_per_launch / avg_push_s / 1e9
    # HBM bytes per push launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (calibrated
    # on a plain copy); only valid for the kernel source the counters were taken on
    traffic = stored_traffic(args.traffic_json, args.workload, "k_push")

    line = dict(
        metric="particle-pushes/s incl. RR+gather+deposit (% HBM roofline); p50/p99 run latency",
        value=value, unit="pushes/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=res["seconds"] * 1e3 / args.steps, higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32" if cfg["precision"] == "fp32" else "f64",
        data="synthetic (seeded quiet-start foil, analytic laser)",
        config=dict(workload=f"{args.workload}: LP a0={cfg['a0']:g}, {res['info']['n_cells']} cells, "
                             f"{int(res['n_e'] + res['n_i'])} particles "
                             f"({cfg['ppc']} per cell per species), "
                             f"{cfg['precision']} + compensated RR, FP64 budgets",
                    n_cells=res["info"]["n_cells"], particles=int(res["n_e"] + res["n_i"]),
                    sort_interval=cfg["sort_interval"], diag_every=args.diag_every,
                    t_start_periods=res["start"] * res["info"]["dt"] / (2 * 3.141592653589793),
                    window_steps=[res["start"], res["start"] + args.steps],
                    parallelism="single GPU"),
        window=dict(raw_ms_per_step=res["raw_seconds"] * 1e3 / args.steps,
                    sorts_in_window=res["sorts_in_window"], sort_cost_ms=res["sort_cost_s"] * 1e3,
                    method=f"time per step = (wall - {res['sorts_in_window']} C + steps/"
                           f"{cfg['sort_interval']} C) / steps; C, the cost of one sort (its kernels "
                           "and the push after it), is the wall time of the half interval that "
                           "opens with the sort before the window minus that of the half interval "
                           "before it, in the same run"),
        roofline=dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
                      frac=achieved / PEAK_HBM_GBS, traffic=traffic,
                      kernel="k_push", bytes_per_launch=bytes_per_launch,
                      avg_launch_us=avg_push_s * 1e6, alg_bytes_per_push=dict(electron=be, ion=bi)),
        kernel_us_per_launch={k: v[0] * 1e3 / max(v[1], 1) for k, v in res["kernels"].items()},
        kernel_ms_per_step={k: v[0] / max(v[1], 1) * (1.0 / cfg["sort_interval"] if k == "sort" else 1.0)
                            for k, v in res["kernels"].items()},
        kernel_launches_timed={k: v[1] for k, v in res["kernels"].items()},
        timing=f"HIP start/end events of every {TIMING_PERIOD}th launch of each kernel",
        energy_balance=res["diag1"]["balance"] / max(res["diag1"]["E_in"], 1e-300),
        gauss_int=res["diag1"]["gauss_int"],
    )
    if not args.no_side_runs:
        cc = copy_ceiling()
        line["roofline"]["copy_ceiling"] = cc
        line["roofline"]["frac_of_copy"] = achieved / cc["gbs"]
        # side runs over the same window (the same lead-in, at least 256 steps)
        # (a whole number of sort intervals: the sorts in the window are the configured share)
        side = max(-(-args.steps // cfg["sort_interval"]) * cfg["sort_interval"], 256)
        def best(c, reps=2):
            # side runs repeat: single short windows vary by several percent
            # from run to run on one box; the faster of the repeats is kept
            return max(pushes_per_s(time_run(c, side, args.warmup, args.diag_every, timing=0), side)
                       for _ in range(reps))

        v_on = best(cfg)
        v_off = best(dict(cfg, rr=False))
        v_nc = best(dict(cfg, rr_compensated=False))
        v_64 = best(dict(cfg, precision="fp64"), 1)
        # the RR arithmetic alone (no residual arrays: 44 B per push like RR
        # off) and with the compensated accumulation (+24 B per electron)
        line["rr_cost"] = dict(pushes_per_s_rr_on=v_on, pushes_per_s_rr_off=v_off,
                               overhead=v_off / v_on - 1.0,
                               pushes_per_s_rr_on_uncompensated=v_nc,
                               overhead_uncompensated=v_off / v_nc - 1.0, steps=side,
                               paper="about +10% compute time with RR (Section 3)")
        line["fp64_path"] = dict(pushes_per_s=v_64, pushes_per_s_fp32=v_on,
                                 speedup_fp32_over_fp64=v_on / v_64, steps=side)
        # the other polarisation and amplitude of the precision-form workload
        variants = {}
        for pol, a0 in (("CP", 500.0), ("CP", 200.0), ("LP", 200.0)):
            r_v = time_run(dict(cfg, pol=pol, a0=a0), side, args.warmup, args.diag_every, timing=0)
            variants[f"{pol}_a0_{a0:g}"] = dict(pushes_per_s=pushes_per_s(r_v, side),
                                                energy_balance=r_v["diag1"]["balance"] / r_v["diag1"]["E_in"],
                                                gauss_int=r_v["diag1"]["gauss_int"])
        variants["LP_a0_500"] = dict(pushes_per_s=v_on)
        variants["steps"] = side
        line["c3_variants"] = variants
        line["plain_method_scale"] = side_by_side_c2()
        line["small_runs"] = small_runs()
        line["pic2d"] = bench_2d()
        line["cpu_baseline"] = cpu_baseline(cfg, res["state"])
    if not args.no_serve:
        line["serving"] = serve_bench()
        # the same stream with each quantum's steps in one persistent launch
        # (measured slower; the default keeps a push and a field launch per step)
        per = serve_bench(persistent=True, groups=1)
        line["serving_persistent_form"] = {k: per[k] for k in ("p50_s", "p99_s", "mean_s", "wall_s",
                                                               "pushes_per_s", "failed_checks",
                                                               "launch_form")}
        # the same 256 requests all queued at time 0: the served batch's
        # throughput when no slot idles (its whole pipeline: sorts, pushes,
        # field passes and the host's admissions), as a fraction of the
        # HBM peak by the pushes' algorithmic bytes
        sat = serve_bench(saturated=True)
        line["serving_saturated"] = {k: sat[k] for k in ("wall_s", "pushes", "pushes_per_s",
                                                         "push_bytes_per_s_frac", "groups",
                                                         "failed_checks", "p50_s", "p99_s")}
        if not args.no_stress:
            line["stress"] = stress_bench(dict(groups=1), max_grid=args.stress_grid)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
