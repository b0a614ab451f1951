"""The move arithmetic of the deposition contract needs correctly rounded
square roots and reciprocals.  The push kernel computes them from hardware
estimates plus FMA corrections; this compares them, for every finite float
>= 1, with the compiler's correctly rounded sqrtf and 1.0f / x (the
reciprocal below 2^126).  Any difference would break the bit-exact cell and
current contract against the oracle."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu


def test_move_sqrt_and_reciprocal_are_correctly_rounded_everywhere():
    import torch

    from paper_1008_1685_amd import _native as N

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print("\n[gpu] exhaustive rounding check, floats in [1, 2^128)", flush=True)
    lib = N.load()
    bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    first, last = 0x3F800000, 0x7F7FFFFF  # 1.0 .. largest finite float
    N.check(lib.pic_check_rounding(first, last - first + 1, C.c_void_p(bad.data_ptr()), stream),
            "pic_check_rounding")
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
