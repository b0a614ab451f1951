"""Serving form on the GPU: continuous batching gives each run the result it
gets alone and the oracle's result, admits by device-memory budget, reuses
slots, and confines a failing run's error to that run."""
import numpy as np
import pytest

from workloads import preset

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def _req_cfgs():
    # uneven sizes, both polarisations; step counts not multiples of the quantum
    return [
        dict(preset("c1", ppc=8, box_lambda=4.0, x_foil=1.5, pol="LP", a0=150.0, periods=1.5, seed=1), name="a"),
        dict(preset("c1", ppc=24, box_lambda=6.0, x_foil=2.0, pol="CP", a0=250.0, periods=3.0, seed=2), name="b"),
        dict(preset("c1", ppc=16, box_lambda=5.0, x_foil=1.0, pol="LP", a0=300.0, periods=2.2, seed=3), name="c"),
    ]


def _alone(cfg):
    from paper_1008_1685_amd import Run
    from paper_1008_1685_amd.serve import run_steps

    run = Run(cfg)
    run.step(run_steps(cfg))
    return run.get_state(), run.diag()


def _same(sa, da, sb, db):
    for k in ("Ex_int", "Ey", "Ez", "By", "Bz", "Ex"):
        assert np.array_equal(sa[k], sb[k]), k
    for s in range(2):
        keys = ("cell", "off", "ux", "uy", "uz")
        A = np.stack([sa[f"sp{s}"][k].astype(np.float64) for k in keys], 1)
        B = np.stack([sb[f"sp{s}"][k].astype(np.float64) for k in keys], 1)
        assert np.array_equal(A[np.lexsort(A.T[::-1])], B[np.lexsort(B.T[::-1])])
    assert da["step"] == db["step"] and da["n_alive"] == db["n_alive"]
    for k in ("E_in", "E_out_left", "E_out_right", "U_field"):
        assert da[k] == db[k], k
    # FP64 sums over particles depend on particle order (the sort order within
    # a cell is not fixed): rounding only
    for k in ("K_e", "K_i"):
        assert da[k] == pytest.approx(db[k], rel=1e-12, abs=1e-300), k
    # RR and escape losses are summed per thread in FP32 before the FP64 sums
    for k in ("E_rad", "E_esc"):
        assert da[k] == pytest.approx(db[k], rel=1e-6, abs=1e-300), k


@pytest.mark.parametrize("persistent,groups", [(False, 1), (True, 1), (False, 2)],
                         ids=["per-pass-launches", "persistent", "two-groups"])
def test_each_run_is_the_same_alone_and_in_the_mix(persistent, groups):
    from paper_1008_1685_amd.serve import Server

    cfgs = _req_cfgs()
    alone = [_alone(c) for c in cfgs]
    # staggered arrivals: runs join while others are already on the GPU; with
    # two groups, two batches on streams of their own step at the same time
    reqs = [dict(arrival=0.002 * i, cfg=c) for i, c in enumerate(cfgs)]
    srv = Server(budget_bytes=1 << 34, max_slots=4, max_particles=2 * 10 ** 6, max_cells=10 ** 5,
                 persistent=persistent, groups=groups)
    recs = srv.serve(reqs, keep_runs=True)
    assert len(recs) == 3
    by = {r["name"]: r for r in recs}
    for (sa, da), c in zip(alone, cfgs):
        r = by[c["name"]]
        _same(sa, da, r["run"].get_state(), r["diag"])
        assert r["diag"]["gauss_int"] == 0


def test_budget_and_slot_reuse():
    from paper_1008_1685_amd import workspace_bytes
    from paper_1008_1685_amd.serve import Server

    cfgs = [dict(c, name=f"{c['name']}{k}", seed=10 * k + i)
            for k in range(3) for i, c in enumerate(_req_cfgs())]
    need = max(workspace_bytes(c) for c in cfgs)
    budget = 2 * need + 1  # at most two runs resident by memory, three slots
    srv = Server(budget_bytes=budget, max_slots=3, max_particles=2 * 10 ** 6, max_cells=10 ** 5)
    recs = srv.serve([dict(arrival=0.0, cfg=c) for c in cfgs])
    assert len(recs) == len(cfgs)
    assert srv.peak_bytes <= budget
    for r in recs:
        assert r["diag"]["gauss_int"] == 0
        assert r["diag"]["step"] == r["steps"]
        assert r["latency"] >= r["done"] - r["admitted"] >= 0


@pytest.mark.parametrize("persistent,groups", [(False, 1), (True, 1), (False, 3)],
                         ids=["per-pass-launches", "persistent", "three-groups"])
def test_every_run_of_a_request_stream_conserves_charge(persistent, groups):
    # many uneven runs sharing the batch through admission, sorts and slot
    # reuse: each run's integer Gauss law must hold exactly at the end
    from paper_1008_1685_amd.serve import Server
    from workloads import poisson_stream

    reqs = poisson_stream(0, n_runs=48, rate=20.0)
    max_p = max(2 * r["cfg"]["ppc"] * round(r["cfg"]["thickness"] * r["cfg"]["cells_per_lambda"])
                for r in reqs)
    max_c = max(round(r["cfg"]["box_lambda"] * r["cfg"]["cells_per_lambda"]) for r in reqs)
    srv = Server(budget_bytes=16 * 2 ** 30, max_slots=64, quantum=reqs[0]["cfg"]["sort_interval"],
                 max_particles=64 * max_p,
                 max_cells=64 * (max_c + 8), persistent=persistent, groups=groups)
    recs = srv.serve(reqs)
    assert len(recs) == len(reqs)
    bad = [(r["name"], r["diag"]["gauss_int"], r["diag"]["nonfinite"]) for r in recs
           if r["diag"]["gauss_int"] != 0 or r["diag"]["nonfinite"]]
    assert not bad, bad


_ORACLE_ROWS = {}


def _oracle_rows(c):
    # the oracle's diagnostics of a configuration over three seeds (computed
    # once per configuration for every test that needs them)
    from oracle import pic as opic
    from paper_1008_1685_amd.serve import run_steps

    if c["name"] not in _ORACLE_ROWS:
        n = run_steps(c)
        _ORACLE_ROWS[c["name"]] = [opic.Pic1D(dict(c, seed=c["seed"] + 100 * k)).run(n).diag()
                                   for k in range(3)]
    return _ORACLE_ROWS[c["name"]]


@pytest.mark.parametrize("groups", [1, 3], ids=["one-group", "three-groups"])
def test_served_runs_match_the_oracle(groups):
    # every served request against the FP64 oracle on its own configuration,
    # at the tolerances of the short runs: each energy term within 2e-3 of the
    # injected energy plus twice the oracle's own seed-to-seed spread (LP heats
    # the electrons chaotically), the balance within 1e-3, alive counts exact;
    # with three groups the requests step in batches on separate streams
    from paper_1008_1685_amd.serve import Server

    keys = ("U_field", "K_e", "K_i", "E_rad", "E_out_left", "E_out_right", "E_esc")
    cfgs = _req_cfgs()
    reqs = [dict(arrival=0.002 * i, cfg=c) for i, c in enumerate(cfgs)]
    srv = Server(budget_bytes=1 << 34, max_slots=4, max_particles=2 * 10 ** 6, max_cells=10 ** 5,
                 groups=groups)
    recs = {r["name"]: r for r in srv.serve(reqs)}
    for c in cfgs:
        d = recs[c["name"]]["diag"]
        rows = _oracle_rows(c)
        ref = rows[0]
        e_in = ref["E_in"]
        assert d["E_in"] == pytest.approx(e_in, rel=1e-6)
        assert d["gauss_int"] == 0
        for k in keys:
            vals = np.array([r[k] for r in rows])
            tol = (2e-3 + 2 * np.ptp(vals) / e_in) * e_in
            print(f"[{c['name']}] {k}: served {d[k] / e_in:.5f} oracle {vals.mean() / e_in:.5f} "
                  f"tol {tol / e_in:.5f} (fraction of E_in)", flush=True)
            assert abs(d[k] - vals.mean()) <= tol, (c["name"], k, d[k], vals)
        assert abs(d["balance"] - ref["balance"]) <= 1e-3 * e_in


def test_a_non_finite_request_flags_only_itself():
    # a request whose state holds a NaN momentum shares the batch with three
    # others: only it reports PIC_ENONFINITE (the particle dropped), and every
    # other run ends bit for bit as it does alone
    from paper_1008_1685_amd import PicError, Run
    from paper_1008_1685_amd.serve import Batch, run_steps

    cfgs = _req_cfgs()
    alone = [_alone(c) for c in cfgs]
    bad = dict(cfgs[1], name="nan", seed=7)
    batch = Batch(max_slots=4, quantum=16, max_particles=2 * 10 ** 6, max_cells=10 ** 5)
    entries = []
    for c in (cfgs[0], bad, cfgs[1], cfgs[2]):
        run = Run(c, stream=batch.stream)
        if c is bad:
            st = run.get_state()
            n0 = st["sp0"]["cell"].size
            st["sp0"]["ux"][n0 // 2] = np.nan
            run.set_state({0: st["sp0"], 1: st["sp1"]}, step=0)
        entries.append((c, run, batch.admit(run, run_steps(c))))
    while True:
        batch.step(2)
        now = batch.poll()
        if all(now[slot] >= run_steps(c) for c, _, slot in entries):
            break
    for c, run, slot in entries:
        batch.release(slot)
    for c, run, slot in entries:
        if c is bad:
            with pytest.raises(PicError, match="PIC_ENONFINITE"):
                run.diag()
            d = run.diag(allow_nonfinite=True)
            # (the dropped particle's charge leaves without a current, so this
            # run's Gauss law no longer closes: its result is flagged invalid)
            assert d["nonfinite"] == 1 and d["n_alive"][1] == n0
            assert d["n_alive"][0] <= n0 - 1
            continue
        k = [x["name"] for x in cfgs].index(c["name"])
        d = run.diag()
        assert d["nonfinite"] == 0
        _same(*alone[k], run.get_state(), d)
    batch.close()


def test_persistent_form_limits():
    from paper_1008_1685_amd.serve import Batch

    b = Batch(max_slots=129, quantum=16, max_particles=10 ** 5, max_cells=10 ** 4)
    with pytest.raises(RuntimeError, match="at most 128 slots"):
        b.set_persistent(True)
    b.set_persistent(False)
    b.close()


@pytest.mark.parametrize("persistent", [False, True], ids=["per-pass-launches", "persistent"])
def test_drain_runs_every_resident_run_to_its_target(persistent):
    from paper_1008_1685_amd import Run
    from paper_1008_1685_amd.serve import Batch, run_steps

    cfgs = _req_cfgs()[:2]
    alone = [_alone(c) for c in cfgs]
    b = Batch(max_slots=4, quantum=16, max_particles=2 * 10 ** 6, max_cells=10 ** 5)
    b.set_persistent(persistent)
    runs, slots = [], []
    for c in cfgs:
        r = Run(c, stream=b.stream)
        runs.append(r)
        slots.append(b.admit(r, run_steps(c)))
    q = b.drain()
    steps = b.poll()
    assert q >= max(run_steps(c) for c in cfgs) // 16
    for r, sl, c, (sa, da) in zip(runs, slots, cfgs, alone):
        assert steps[sl] == run_steps(c)
        b.release(sl)
        _same(sa, da, r.get_state(), r.diag())
    assert b.drain() == 0  # nothing resident
    b.close()


@pytest.mark.parametrize("persistent", [False, True], ids=["per-pass-launches", "persistent"])
def test_fp64_batch_runs_are_the_same_alone_and_in_the_mix(persistent):
    # the plain FP64 path through both batch launch forms
    from paper_1008_1685_amd.serve import Server

    cfgs = [dict(c, precision="fp64") for c in _req_cfgs()]
    alone = [_alone(c) for c in cfgs]
    reqs = [dict(arrival=0.0, cfg=c) for c in cfgs]
    srv = Server(budget_bytes=1 << 34, max_slots=4, max_particles=2 * 10 ** 6, max_cells=10 ** 5,
                 precision="fp64", persistent=persistent)
    recs = srv.serve(reqs, keep_runs=True)
    by = {r["name"]: r for r in recs}
    for (sa, da), c in zip(alone, cfgs):
        r = by[c["name"]]
        _same(sa, da, r["run"].get_state(), r["diag"])
        assert r["diag"]["gauss_int"] == 0


def test_async_poll_reports_only_runs_resident_when_it_was_queued():
    from paper_1008_1685_amd import Run
    from paper_1008_1685_amd._native import PicError
    from paper_1008_1685_amd.serve import Batch, run_steps

    cfgs = _req_cfgs()[:2]
    b = Batch(max_slots=4, quantum=16, max_particles=2 * 10 ** 6, max_cells=10 ** 5)
    ra = Run(cfgs[0], stream=b.stream)
    sa = b.admit(ra, run_steps(cfgs[0]))
    b.step(2)
    b.poll_async()
    with pytest.raises(PicError):
        b.poll_async()  # one queued poll at a time
    rb = Run(cfgs[1], stream=b.stream)
    sb = b.admit(rb, run_steps(cfgs[1]))  # admitted after the poll was queued
    steps = b.poll_wait()
    assert steps[sa] == 32 and steps[sb] == -1
    assert all(steps[s] == -1 for s in range(4) if s not in (sa, sb))
    with pytest.raises(PicError):
        b.poll_wait()  # nothing queued
    b.step(1)
    b.poll_async()
    steps = b.poll_wait()
    assert steps[sa] == 48 and steps[sb] == 16
    b.release(sa)
    b.release(sb)
    b.close()


def test_persistent_barrier_timeout_is_reported():
    # every grid-barrier wait of the persistent launch cut to zero from the
    # host (set_persistent(2)): the launch still ends (every wait is bounded)
    # and the next poll reports the error instead of steps
    from paper_1008_1685_amd import Run
    from paper_1008_1685_amd._native import PicError
    from paper_1008_1685_amd.serve import Batch, run_steps

    cfgs = _req_cfgs()
    b = Batch(max_slots=4, quantum=16, max_particles=2 * 10 ** 6, max_cells=10 ** 5)
    b.set_persistent(2)
    runs = []
    for c in cfgs:
        r = Run(c, stream=b.stream)
        runs.append(r)
        b.admit(r, run_steps(c))
    b.step(1)
    with pytest.raises(PicError, match="timed out"):
        b.poll()
    b.close()
    for r in runs:
        r.close()
