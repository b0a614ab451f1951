"""The allocation-free spectrum entry point (pic_spectrum_static) against
pic_spectrum, which takes its counters from the run's workspace: the same
histogram, exactly (integer counts), on two calls in a row, the second on a
smaller run with fewer bins, so counts the first call left in the shared
array would show."""
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


def _run(**kw):
    from paper_1008_1685_amd import Run

    cfg = preset("c1", **kw)
    run = Run(cfg)
    run.step(2400)  # into the laser-foil interaction: a spread of proton energies
    return run


def test_static_spectrum_matches_the_workspace_spectrum():
    from paper_1008_1685_amd import PicError

    big = _run(ppc=64, pol="LP", a0=300.0)
    small = _run(ppc=8, x_foil=4.0, a0=150.0, seed=3)
    h_ref = big.spectrum(4096, 80.0)
    h = big.spectrum_static(4096, 80.0)
    assert h_ref.sum() > 0 and np.count_nonzero(h_ref) > 20
    assert np.array_equal(h, h_ref)
    # second call: fewer particles, fewer bins, another range
    h_ref2 = small.spectrum(300, 40.0)
    h2 = small.spectrum_static(300, 40.0)
    assert h_ref2.sum() > 0
    assert np.array_equal(h2, h_ref2)
    # and the first again, after the smaller call
    assert np.array_equal(big.spectrum_static(4096, 80.0), h_ref)
    # the fixed array bounds the bin count
    with pytest.raises(PicError, match="PIC_EINVAL"):
        big.spectrum_static(65537, 80.0)
    big.close()
    small.close()
