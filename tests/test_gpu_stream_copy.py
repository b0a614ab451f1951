"""The copy kernel behind the roofline's measured ceiling copies exactly,
including a size that leaves a partial last work-group, and refuses sizes
and alignments it does not take before launching anything."""
import ctypes as C
import os

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    lib = C.CDLL(os.path.join(ROOT, "paper_1008_1685_amd", "libstreamcopy.so"))
    lib.stream_copy.restype = C.c_int
    lib.stream_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    return lib


def test_stream_copy_is_exact_and_checks_its_arguments():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print("\n[gpu] stream_copy", flush=True)
    lib = _lib()
    st = torch.cuda.current_stream()
    n = 4 * 1000003  # int32 words: 1,000,003 16-byte elements, a partial last work-group
    a = torch.randint(-2 ** 31, 2 ** 31 - 1, (n + 4,), dtype=torch.int32, device="cuda")
    b = torch.full((n + 4,), 7, dtype=torch.int32, device="cuda")
    assert lib.stream_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), 4 * n,
                           C.c_void_p(st.cuda_stream)) == 0
    torch.cuda.synchronize()
    assert torch.equal(a[:n], b[:n])
    assert torch.all(b[n:] == 7)  # nothing past the end
    assert lib.stream_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), 0,
                           C.c_void_p(st.cuda_stream)) == 0
    # a size that is not a multiple of 16 and a misaligned pointer are refused
    assert lib.stream_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), 4 * n - 4,
                           C.c_void_p(st.cuda_stream)) == 1
    assert lib.stream_copy(C.c_void_p(a.data_ptr() + 4), C.c_void_p(b.data_ptr()), 64,
                           C.c_void_p(st.cuda_stream)) == 1
    torch.cuda.synchronize()
    assert torch.all(b[n:] == 7)
