"""pic_step replays two sort intervals at a time as one captured graph.
Every replay must leave the state that the same steps give when launched one
kernel at a time (the stage entry points): fields, integer currents and
particles (in a canonical order: the sort leaves the order within a cell
open) bit for bit, with eager work and synchronisation (diagnostics, state
reads) between the replays, across step counts that start and end between
sort steps, with per-kernel timing switched on in between (which steps
without graphs), and after the particle state is replaced."""
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


G = ("Ex_int", "Ex", "Ey", "Ez", "By", "Bz", "Jx_int", "Jy_int", "Jz_int")
P = ("cell", "off", "ux", "uy", "uz", "w", "rx", "ry", "rz")


def _same(a, b, where):
    for k in G:
        assert np.array_equal(a[k], b[k]), (where, k)
    for s in (0, 1):
        pa, pb = a[f"sp{s}"], b[f"sp{s}"]
        keys = [k for k in P if k in pa]
        assert pa["cell"].size == pb["cell"].size, (where, s)
        oa = np.lexsort([pa[k] for k in reversed(keys)])
        ob = np.lexsort([pb[k] for k in reversed(keys)])
        for k in keys:
            assert np.array_equal(pa[k][oa], pb[k][ob]), (where, s, k)


def _eager(run, n, interval):
    for _ in range(n):
        if run.info["step"] > 0 and run.info["step"] % interval == 0:
            run.sort()
        run.push_deposit()
        run.field_advance()
        run.info["step"] += 1


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_graph_replays_match_kernel_by_kernel_steps(precision):
    from paper_1008_1685_amd import Run

    interval = 16
    cfg = preset("c1", ppc=16, x_foil=2.0, box_lambda=6.0, pol="LP", a0=300.0,
                 precision=precision, sort_interval=interval)
    g, e = Run(cfg), Run(cfg)
    e.info["step"] = 0
    for i, n in enumerate((5, 100, 64, 33, 7, 200, 96, 1, 640, 130, 900)):
        if i == 4:
            g.timing(1)   # steps with per-kernel events go launch by launch
        if i == 6:
            g.timing(0)
        g.step(n)
        _eager(e, n, interval)
        dg, de = g.diag(), e.diag()
        assert dg["step"] == de["step"] and dg["n_alive"] == de["n_alive"], i
        for k in ("E_in", "E_out_left", "E_out_right", "U_field", "gauss_int"):
            assert dg[k] == de[k], (i, k)
        _same(g.get_state(), e.get_state(), i)
    assert dg["E_rad"] > 0 and dg["n_alive"][0] < 1600  # through the interaction
    # replacing the particles drops the recorded graphs (launch grids change)
    st = g.get_state()
    keep = {s: {k: v[: v.size // 2] for k, v in st[f"sp{s}"].items()} for s in (0, 1)}
    g.set_state(keep)
    e.set_state(keep)
    g.step(200)
    _eager(e, 200, interval)
    _same(g.get_state(), e.get_state(), "after set_state")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_split_launches_give_the_same_run(precision):
    # the push and sort passes split into launches of 3 work-groups (graph
    # replays and launch by launch) end in the state of whole-pass launches
    from paper_1008_1685_amd import Run

    cfg = preset("c1", ppc=64, x_foil=2.0, box_lambda=6.0, pol="LP", a0=300.0,
                 precision=precision, sort_interval=16)
    whole, split = Run(cfg), Run(cfg)
    split.set_max_grid(3)
    for n in (5, 300, 1, 1500):
        whole.step(n)
        split.step(n)
        _same(whole.get_state(), split.get_state(), n)
    dw, ds = whole.diag(), split.diag()
    for k in ("E_in", "U_field", "gauss_int", "n_alive"):
        assert dw[k] == ds[k], k
    assert dw["E_rad"] == pytest.approx(ds["E_rad"], rel=1e-6)
