"""bench.py's host-side arithmetic and contract, without a GPU: algorithmic
bytes per push, the timed window's start, the traffic record written from
counter files and its source check, and the one-GPU refusal."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from workloads import preset  # noqa: E402


def test_algorithmic_bytes_per_push():
    # FP32: read cell, offset, 3 momenta, weight (24 B), write cell, offset,
    # 3 momenta (20 B); compensated RR adds 3 FP32 residuals each way (24 B)
    assert bench.alg_bytes_per_push("fp32", True, True) == (68, 44)
    assert bench.alg_bytes_per_push("fp32", False, True) == (44, 44)
    assert bench.alg_bytes_per_push("fp32", True, False) == (44, 44)
    # FP64: int32 cell, FP64 offset, momenta and weight: read 44, write 36
    assert bench.alg_bytes_per_push("fp64", True, True) == (80, 80)


def test_window_starts_in_the_interaction_at_a_sort_step():
    cfg = preset("c3")  # 400 steps per period, a sort every 64 steps
    assert bench.window_start(cfg, 0) == 4032       # 10 periods = 4,000 steps, rounded up
    assert bench.window_start(cfg, 5) == 4032
    assert bench.window_start(cfg, 40) == 4096
    c5 = preset("c5")  # 800 steps per period, a sort every 32 steps
    assert bench.window_start(c5, 0, 8.5) == 6816
    assert all(bench.window_start(cfg, w) % cfg["sort_interval"] == 0 for w in range(0, 200, 7))


def test_sorts_in_the_window():
    # 20 timed steps after the sort-cost half intervals: steps 4,064-4,083, no sort
    assert bench.sorts_in_window(4064, 20, 64) == 0
    assert bench.sorts_in_window(4032, 20, 64) == 1   # opens with the sort at 4,032
    assert bench.sorts_in_window(4032, 256, 64) == 4
    assert bench.sorts_in_window(1, 64, 64) == 1
    assert bench.sorts_in_window(0, 64, 64) == 0      # step 0 has no sort
    for start in range(0, 300, 13):
        for steps in (1, 20, 64, 100):
            brute = sum(1 for k in range(start, start + steps) if k > 0 and k % 64 == 0)
            assert bench.sorts_in_window(start, steps, 64) == brute


def _counter_file(path, name, counter, values):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, v in enumerate(values):
            w.writerow([i + 1, name, counter, v])


def test_traffic_record_from_counter_files(tmp_path):
    # the copy kernel moves 1 GiB each way: FETCH_SIZE reports half of it (x2
    # calibration), WRITE_SIZE all of it (x1)
    gib_kib = 2 ** 30 / 1024
    _counter_file(tmp_path / "cf.csv", "__amd_rocclr_copyBuffer", "FETCH_SIZE", [gib_kib / 2] * 4)
    _counter_file(tmp_path / "cw.csv", "__amd_rocclr_copyBuffer", "WRITE_SIZE", [gib_kib] * 4)
    # 60 push launches; the last 50 average 1000 / 2000 KiB
    _counter_file(tmp_path / "f.csv", "void pic::k_push<float>(pic::PushArgs<float>)", "FETCH_SIZE",
                  [5.0] * 10 + [1000.0] * 50)
    _counter_file(tmp_path / "w.csv", "void pic::k_push<float>(pic::PushArgs<float>)", "WRITE_SIZE",
                  [7.0] * 10 + [2000.0] * 50)
    out = tmp_path / "traffic.json"
    bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                        str(tmp_path / "cw.csv"), str(out))
    t = json.load(open(out))
    assert t["fetch_factor"] == pytest.approx(2.0) and t["write_factor"] == pytest.approx(1.0)
    assert t["read_bytes"] == pytest.approx(2000.0 * 1024)
    assert t["write_bytes"] == pytest.approx(2000.0 * 1024)
    assert t["launches_averaged"] == 50
    # reported only for the sources it was taken on
    assert bench.stored_traffic(str(out), "c3", "k_push") == pytest.approx(4000.0 * 1024)
    assert bench.stored_traffic(str(out), "d2", "k_push") is None
    t["kernel_sha256"] = "0" * 64
    json.dump(t, open(out, "w"))
    assert bench.stored_traffic(str(out), "c3", "k_push") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_serving_bench_passes_its_launch_form_and_groups(monkeypatch):
    # serve_bench builds its Server with the requested groups, except that the
    # persistent form always runs as one group, and with the requests' sort
    # interval as its quantum; a saturated stream queues every request at time 0
    import paper_1008_1685_amd.serve as S

    made = []

    class FakeServer:
        def __init__(self, budget_bytes, max_slots, quantum, max_particles, max_cells, persistent, groups):
            made.append(dict(persistent=persistent, groups=groups, quantum=quantum))
            self.batches = [None] * groups
            self.peak_bytes = 0

        def serve(self, reqs):
            made[-1]["arrivals"] = [r["arrival"] for r in reqs]
            # the batch takes runs whose sort interval is its quantum
            assert all(r["cfg"]["sort_interval"] == made[-1]["quantum"] for r in reqs)
            return [dict(latency=1.0, particles=10, steps=5, diag=dict(gauss_int=0, nonfinite=0))
                    for _ in reqs]

    monkeypatch.setattr(S, "Server", FakeServer)
    r = bench.serve_bench(n_runs=4)
    assert made[-1]["groups"] == bench.SERVE_GROUPS and not made[-1]["persistent"]
    assert r["groups"] == bench.SERVE_GROUPS and r["pushes"] == 4 * 50
    bench.serve_bench(n_runs=4, persistent=True)
    assert made[-1]["groups"] == 1 and made[-1]["persistent"]
    bench.serve_bench(n_runs=4, saturated=True, groups=2)
    assert made[-1]["groups"] == 2 and made[-1]["arrivals"] == [0.0] * 4
    assert max(made[0]["arrivals"]) > 0
