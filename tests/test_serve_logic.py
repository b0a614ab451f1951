"""Host logic of the serving loop (no GPU): admission order, device-memory
budget, slot capacity and reuse, completion bookkeeping.  The batch and
runs are replaced by stand-ins that count steps like the device does."""
import numpy as np
import pytest

import paper_1008_1685_amd.serve as S
from workloads import poisson_stream, preset


class FakeRun:
    made = 0

    def __init__(self, cfg, stream=None, **kw):
        FakeRun.made += 1
        self.cfg = cfg
        self.info = dict(n_init=(10, 10))
        self._h = object()
        self.closed = False

    def diag(self, allow_nonfinite=False):
        return dict(step=self.step, gauss_int=0)

    def close(self):
        self.closed = True


class FakeBatch:
    def __init__(self, precision, max_slots, quantum, max_particles, max_cells):
        self.max_slots, self.quantum = max_slots, quantum
        self.slots = [None] * max_slots
        self.stream = None
        self.admitted = []

    def fits(self, cfg):
        # work capacity of the stand-in: runs of more than 1e4 particles never fit
        ever = cfg.get("ppc", 0) <= 10 ** 4
        return ever and any(s is None for s in self.slots), ever

    def admit(self, run, n_steps):
        for i, s in enumerate(self.slots):
            if s is None:
                run.step, run.target = 0, n_steps
                self.slots[i] = run
                self.admitted.append(run.cfg["name"])
                return i
        raise AssertionError("admit called without a free slot")

    def set_persistent(self, on):
        self.persistent = on

    def step(self, n):
        for r in self.slots:
            if r is not None:
                r.step = min(r.target, r.step + n * self.quantum)

    def poll(self):
        return np.array([-1 if r is None else r.step for r in self.slots], np.int64)

    def poll_async(self):
        # the counters as queued behind the replays; a slot whose run changes
        # before the wait reads -1, as the library reports it
        self._snap = [(r, -1 if r is None else r.step) for r in self.slots]

    def poll_wait(self):
        out = [v if r is not None and r is self.slots[i] else -1 for i, (r, v) in enumerate(self._snap)]
        self._snap = None
        return np.array(out, np.int64)

    def release(self, slot):
        self.slots[slot] = None


@pytest.fixture
def fakes(monkeypatch):
    monkeypatch.setattr(S, "Run", FakeRun)
    monkeypatch.setattr(S, "Batch", FakeBatch)
    sizes = {}
    monkeypatch.setattr(S, "workspace_bytes", lambda cfg, capacity=0: sizes.get(cfg["name"], 100))
    return sizes


def _reqs(n, steps_periods=(1.0, 2.0, 3.0)):
    out = []
    for i in range(n):
        cfg = dict(preset("c1", periods=steps_periods[i % len(steps_periods)]), name=f"r{i}")
        out.append(dict(arrival=0.0, cfg=cfg))
    return out


def test_every_request_completes_in_arrival_order_of_admission(fakes):
    srv = S.Server(budget_bytes=10 ** 9, max_slots=2)
    reqs = _reqs(5)
    recs = srv.serve(reqs)
    assert sorted(r["name"] for r in recs) == [f"r{i}" for i in range(5)]
    assert srv.batch.admitted == [f"r{i}" for i in range(5)]
    for r in recs:
        assert r["diag"]["step"] == r["steps"] == S.run_steps(reqs[int(r["name"][1:])]["cfg"])
        assert r["done"] >= r["admitted"] >= r["arrival"]


def test_memory_budget_bounds_resident_runs(fakes):
    for i in range(6):
        fakes[f"r{i}"] = 400
    srv = S.Server(budget_bytes=1000, max_slots=8)
    recs = srv.serve(_reqs(6))
    assert len(recs) == 6
    assert srv.peak_bytes <= 1000 and srv.peak_bytes == 800


def test_a_run_larger_than_the_budget_runs_alone(fakes):
    fakes["r0"] = 5000
    srv = S.Server(budget_bytes=1000, max_slots=8)
    recs = srv.serve(_reqs(3))
    assert len(recs) == 3
    assert srv.peak_bytes == 5000  # admitted only into an empty batch


def test_runs_are_built_only_when_admission_succeeds(fakes):
    # two slots, five requests: every Run built is admitted at once (none is
    # built, then freed again, while the batch is full)
    FakeRun.made = 0
    srv = S.Server(budget_bytes=10 ** 9, max_slots=2)
    recs = srv.serve(_reqs(5))
    assert len(recs) == 5 and FakeRun.made == 5


def test_a_request_that_can_never_fit_raises(fakes):
    reqs = _reqs(2)
    reqs[1]["cfg"]["ppc"] = 10 ** 5
    srv = S.Server(budget_bytes=10 ** 9, max_slots=2)
    with pytest.raises(ValueError, match="work capacity"):
        srv.serve(reqs)


def test_poisson_stream_shape():
    runs = poisson_stream(0, n_runs=256, rate=20.0)
    t = np.array([r["arrival"] for r in runs])
    assert np.all(np.diff(t) > 0)
    assert 256 / t[-1] == pytest.approx(20.0, rel=0.2)
    n = np.array([2 * r["cfg"]["ppc"] * round(r["cfg"]["thickness"] * 100) for r in runs])
    assert n.min() >= 0.9e4 and n.max() <= 1.1e6
    assert {r["cfg"]["pol"] for r in runs} == {"LP", "CP"}
    assert all(30 <= r["cfg"]["periods"] <= 80 for r in runs)


def test_a_poll_queued_before_an_admission_does_not_release_the_new_run(fakes):
    # one slot: the long run finishes (600 steps), the short one (200 steps)
    # takes its slot while a poll queued before the admission still holds the
    # long run's 600; the short run must be released only at its own target
    srv = S.Server(budget_bytes=10 ** 9, max_slots=1)
    reqs = _reqs(2, steps_periods=(3.0, 1.0))
    recs = srv.serve(reqs)
    assert [r["name"] for r in recs] == ["r0", "r1"]
    for r in recs:
        assert r["diag"]["step"] == r["steps"] == S.run_steps(reqs[int(r["name"][1:])]["cfg"])


def test_groups_split_the_slots_and_share_the_requests(fakes):
    srv = S.Server(budget_bytes=10 ** 9, max_slots=5, groups=2)
    assert [b.max_slots for b in srv.batches] == [3, 2]
    reqs = _reqs(7)
    recs = srv.serve(reqs)
    assert sorted(r["name"] for r in recs) == [f"r{i}" for i in range(7)]
    for r in recs:
        assert r["diag"]["step"] == r["steps"] == S.run_steps(reqs[int(r["name"][1:])]["cfg"])
    assert all(b.admitted for b in srv.batches)
    assert sorted(sum((b.admitted for b in srv.batches), [])) == sorted(r["name"] for r in recs)


def test_a_request_joins_the_group_with_the_least_resident_work(fakes):
    fakes.update(r0=400, r1=100, r2=100)
    srv = S.Server(budget_bytes=10 ** 9, max_slots=4, groups=2)
    srv.serve(_reqs(3))
    # r0 (400) takes group 0; r1 and r2 go to group 1, which then holds 200
    assert srv.batches[0].admitted == ["r0"] and srv.batches[1].admitted == ["r1", "r2"]


def test_the_persistent_form_runs_as_one_group(fakes):
    with pytest.raises(ValueError, match="one group"):
        S.Server(budget_bytes=10 ** 9, max_slots=4, groups=2, persistent=True)
    with pytest.raises(ValueError):
        S.Server(budget_bytes=10 ** 9, max_slots=4, groups=0)
    assert len(S.Server(budget_bytes=10 ** 9, max_slots=2, groups=3).batches) == 2
