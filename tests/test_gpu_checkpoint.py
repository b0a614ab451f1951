"""Checkpoint and resume: a state taken with get_state and set into a fresh
run continues exactly as the uninterrupted run.

Every particle's update depends only on its own data and the fields, the
current is summed in exact integers, and the boundary energies are summed
in step order, so the particles (compared in a canonical order, since the
sort leaves the order within a cell open), fields, integer currents,
boundary energies and every integer diagnostic must repeat bit for bit.
FP64 sums over particles follow the particle order within a cell: the
kinetic energies agree to rounding (1e-12), the radiated and escaped
energies, summed per thread in FP32 first, to 1e-6, as between two
uninterrupted runs."""
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


def _same_state(a, b, particle_keys, grid_keys):
    """Grids equal bit for bit, and particles equal bit for bit in a canonical
    order (whichever of ``particle_keys`` each species has); the message
    names every array that differs."""
    diffs = []
    for k in grid_keys:
        if not np.array_equal(a[k], b[k]):
            diffs.append(f"{k}: {int(np.sum(a[k] != b[k]))} entries")
    for s in (0, 1):
        pa, pb = a[f"sp{s}"], b[f"sp{s}"]
        keys = [k for k in particle_keys if k in pa]
        if pa["cell"].size != pb["cell"].size:
            diffs.append(f"species {s}: {pa['cell'].size} against {pb['cell'].size} particles")
            continue
        oa = np.lexsort([pa[k] for k in reversed(keys)])
        ob = np.lexsort([pb[k] for k in reversed(keys)])
        for k in keys:
            if not np.array_equal(pa[k][oa], pb[k][ob]):
                diffs.append(f"species {s} {k}: {int(np.sum(pa[k][oa] != pb[k][ob]))} particles")
    assert not diffs, "; ".join(diffs)


EXACT = ("step", "n_alive", "gauss_int", "n_stiff", "nonfinite", "E_in", "E_out_left",
         "E_out_right", "U_Ex", "U_Et", "U_B", "U_field")


def _compare_diag(da, db, exact=EXACT):
    for k in exact:
        assert da[k] == db[k], (k, da[k], db[k])
    for k in ("K_e", "K_i"):
        assert da[k] == pytest.approx(db[k], rel=1e-12, abs=1e-300), k
    for k in ("E_rad", "E_esc"):
        assert da[k] == pytest.approx(db[k], rel=1e-6, abs=1e-300), k
    assert da["balance"] == pytest.approx(db["balance"], abs=1e-9 * da["E_in"])


P1 = ("cell", "off", "ux", "uy", "uz", "w", "rx", "ry", "rz")
G1 = ("Ex_int", "Ex", "Ey", "Ez", "By", "Bz", "Jx_int", "Jy_int", "Jz_int")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_1d_checkpoint_resumes_bit_for_bit(precision):
    from paper_1008_1685_amd import Run

    # LP into the interaction: RR radiates and particles leave the box; the
    # checkpoint falls between two sorts (every 500 steps) after electrons
    # have left, so the state it takes is compacted around removed slots
    cfg = preset("c1", ppc=16, x_foil=2.0, box_lambda=6.0, pol="LP", a0=300.0,
                 precision=precision, sort_interval=500)
    k, n = 1795, 2400
    whole = Run(cfg)
    whole.step(n)
    sw, dw = whole.get_state(), whole.diag()

    first = Run(cfg)
    first.step(k)
    cp = first.get_state()
    assert cp["budget"]["E_in"] > 0 and cp["budget"]["E_rad"] > 0 and cp["budget"]["E_esc"][0] > 0
    assert cp["sp0"]["cell"].size < 1600
    first.close()
    resumed = Run(cfg)
    resumed.set_state({0: cp["sp0"], 1: cp["sp1"]},
                      fields={g: cp[g] for g in G1}, step=cp["step"], budget=cp["budget"])
    assert resumed.get_state(particles=False)["budget"]["E_in"] == cp["budget"]["E_in"]
    resumed.step(n - k)
    sr, dr = resumed.get_state(), resumed.diag()
    assert dw["n_alive"][0] < cp["sp0"]["cell"].size  # more left after the checkpoint
    _same_state(sw, sr, P1, G1)
    _compare_diag(dw, dr)


def test_1d_resume_without_the_budget_restarts_it():
    # the budget is part of the checkpoint: leaving it out restarts the
    # cumulative terms from zero (the energy balance no longer closes)
    from paper_1008_1685_amd import Run

    cfg = preset("c1", ppc=8, x_foil=2.0, box_lambda=6.0, pol="CP", a0=200.0)
    first = Run(cfg)
    first.step(900)
    cp = first.get_state()
    resumed = Run(cfg)
    resumed.set_state({0: cp["sp0"], 1: cp["sp1"]}, fields={g: cp[g] for g in G1},
                      step=cp["step"])
    d = resumed.diag()
    assert d["E_in"] == 0.0 and abs(d["balance"]) > 0.1 * cp["budget"]["E_in"]
    resumed.set_state(step=cp["step"], budget=cp["budget"])
    d = resumed.diag()
    assert d["E_in"] == cp["budget"]["E_in"] and abs(d["balance"]) < 1e-2 * d["E_in"]


P2 = ("cell", "ox", "oy", "ux", "uy", "uz", "w", "rx", "ry", "rz")
G2 = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx_int", "Jy_int", "Jz_int", "charge_int")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_2d_checkpoint_resumes_bit_for_bit(precision):
    from paper_1008_1685_amd.run2d import Run2D

    cfg = preset2d("d1", precision=precision)
    k, n = 203, 384
    whole = Run2D(cfg)
    whole.step(n)
    sw, dw = whole.get_state(), whole.diag()
    first = Run2D(cfg)
    first.step(k)
    cp = first.get_state()
    first.close()
    resumed = Run2D(cfg)
    resumed.set_state({0: cp["sp0"], 1: cp["sp1"]}, fields={g: cp[g] for g in G2},
                      step=cp["step"], budget=cp["budget"])
    resumed.step(n - k)
    sr, dr = resumed.get_state(), resumed.diag()
    _same_state(sw, sr, P2, G2)
    # the boundary energies are per-row sums: the restored totals sit in row 0,
    # so their sums agree to rounding
    exact = tuple(k for k in EXACT if k not in ("E_in", "E_out_left", "E_out_right"))
    _compare_diag(dw, dr, exact)
    for k in ("E_in", "E_out_left", "E_out_right"):
        assert dr[k] == pytest.approx(dw[k], rel=1e-12, abs=1e-300), k
