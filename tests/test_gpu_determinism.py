"""Repeated runs reproduce bit for bit.

Every particle's update depends only on its own data and on the fields; the
current is summed in exact integers and the fields from it, so two runs of
the same configuration must end in identical states.  Only the order of
particles within a cell after a sort is left open (the sort claims
positions by atomics), so particle arrays are compared in a canonical order.
"""
import hashlib

import numpy as np
import pytest

from workloads import preset, preset2d

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def _digest(st, particle_keys, grid_keys):
    h = hashlib.sha256()
    for k in grid_keys:
        h.update(np.ascontiguousarray(st[k]).tobytes())
    for s in (0, 1):
        p = st[f"sp{s}"]
        order = np.lexsort([p[k] for k in reversed(particle_keys)])
        for k in particle_keys:
            h.update(np.ascontiguousarray(p[k][order]).tobytes())
    return h.hexdigest()


def _run1d(cfg, steps):
    from paper_1008_1685_amd import Run

    run = Run(cfg)
    run.step(steps)
    st = run.get_state()
    out = _digest(st, ("cell", "off", "ux", "uy", "uz", "w"),
                  ("Ex_int", "Ey", "Ez", "By", "Bz", "Jx_int", "Jy_int", "Jz_int"))
    run.close()
    return out


def _run2d(cfg, steps):
    from paper_1008_1685_amd.run2d import Run2D

    run = Run2D(cfg)
    run.step(steps)
    st = run.get_state()
    out = _digest(st, ("cell", "ox", "oy", "ux", "uy", "uz", "w"),
                  ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx_int", "Jy_int", "Jz_int", "charge_int"))
    run.close()
    return out


@pytest.mark.parametrize("name,precision,steps", [
    # 4e5 particles into the laser-foil interaction (the pulse reaches the foil
    # near step 3,200), with sorts and particles leaving the box; before the
    # pulse arrives the foil sees fields of order 1e-80 and below, so a
    # rounding that depends on where a particle sits in a tile shows in the
    # momenta long before it moves a current.  c2 pushes in small tiles.
    ("c2", "fp32", 3500), ("c2", "fp64", 3500),
    # 1e7 particles in the large tiles of the benchmark, into the interaction
    ("c3", "fp32", 4500)])
def test_1d_runs_repeat_bit_for_bit(name, precision, steps):
    cfg = preset(name, precision=precision)
    assert _run1d(cfg, steps) == _run1d(cfg, steps)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_2d_runs_repeat_bit_for_bit(precision):
    cfg = preset2d("d1", precision=precision)
    assert _run2d(cfg, 384) == _run2d(cfg, 384)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_sort_interval_and_launch_split_leave_the_run_unchanged(precision):
    # the integer currents, the fields and every particle (as a set, with its
    # RR residuals) are independent of the particle order the sort leaves and
    # of how a pass is split over launches: the same run with a sort every
    # 8, 16 or 48 steps, and with its push and sort passes split into
    # launches of 3 work-groups, ends in the same state
    from paper_1008_1685_amd import Run

    cfg = preset("c1", ppc=16, x_foil=2.0, box_lambda=6.0, pol="LP", a0=200.0, precision=precision)
    steps = 1200  # the pulse reaches the foil after about 400 steps

    def digest(interval, max_grid=0):
        run = Run(dict(cfg, sort_interval=interval))
        if max_grid:
            run.set_max_grid(max_grid)
        run.step(steps)
        st = run.get_state()
        keys = ["cell", "off", "ux", "uy", "uz", "w"] + [k for k in ("rx", "ry", "rz") if k in st["sp0"]]
        h = hashlib.sha256()
        for k in ("Ex_int", "Ey", "Ez", "By", "Bz", "Jx_int", "Jy_int", "Jz_int"):
            h.update(np.ascontiguousarray(st[k]).tobytes())
        for s in (0, 1):
            p = st[f"sp{s}"]
            alive = p["cell"] != np.iinfo(np.int32).min  # removed slots stay until the next sort
            ks = [k for k in keys if k in p]
            q = {k: p[k][alive] for k in ks}
            order = np.lexsort([q[k] for k in reversed(ks)])
            for k in ks:
                h.update(np.ascontiguousarray(q[k][order]).tobytes())
        d = run.diag()
        run.close()
        assert d["gauss_int"] == 0
        return h.hexdigest()

    ref = digest(16)
    assert digest(8) == ref
    assert digest(48) == ref
    assert digest(16, max_grid=3) == ref


def _state_digest(run):
    # integer currents, fields and every alive particle (as a set, with its
    # RR residuals) of a run
    st = run.get_state()
    keys = ["cell", "off", "ux", "uy", "uz", "w"] + [k for k in ("rx", "ry", "rz") if k in st["sp0"]]
    h = hashlib.sha256()
    for k in ("Ex_int", "Ey", "Ez", "By", "Bz", "Jx_int", "Jy_int", "Jz_int"):
        h.update(np.ascontiguousarray(st[k]).tobytes())
    for s in (0, 1):
        p = st[f"sp{s}"]
        alive = p["cell"] != np.iinfo(np.int32).min
        ks = [k for k in keys if k in p]
        q = {k: p[k][alive] for k in ks}
        order = np.lexsort([q[k] for k in reversed(ks)])
        for k in ks:
            h.update(np.ascontiguousarray(q[k][order]).tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_push_tile_size_leaves_the_run_unchanged(precision):
    # one state in the laser-foil interaction, stepped alone in the single-run
    # push's 5,120-particle tiles (four particles' loads in flight) and in a
    # serving batch's 1,024-particle tiles (two in flight): the tiling decides
    # only which lanes push which particles, so both end in the same state
    from paper_1008_1685_amd import Run
    from paper_1008_1685_amd.serve import Batch

    cfg = preset("c2", ppc=8000, precision=precision)  # 1.6e6 particles per species
    src = Run(cfg)
    src.step(3264)  # the pulse reaches the foil near step 3,200
    st = src.get_state()
    src.close()
    parts = {0: st["sp0"], 1: st["sp1"]}
    fields = {k: st[k] for k in ("Ex", "Ey", "Ez", "By", "Bz", "Ex_int", "Jx_int", "Jy_int", "Jz_int")}
    steps = 64  # three sorts (every 16 steps)

    alone = Run(cfg)
    assert alone.get_info()["tile"] == 5120
    alone.set_state(parts, fields, step=0)
    start = _state_digest(alone)
    alone.step(steps)
    ref = _state_digest(alone)
    assert ref != start  # the steps move particles and currents
    assert alone.diag()["gauss_int"] == 0
    alone.close()

    batch = Batch(precision=precision, max_slots=1, quantum=cfg["sort_interval"],
                  max_particles=4 * 10 ** 6, max_cells=2 * 10 ** 4)
    run = Run(cfg, stream=batch.stream)
    run.set_state(parts, fields, step=0)
    slot = batch.admit(run, steps)
    batch.drain()
    assert batch.poll()[slot] == steps
    batch.release(slot)
    assert _state_digest(run) == ref
    assert run.diag()["gauss_int"] == 0
    run.close()
    batch.close()
