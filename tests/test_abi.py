"""The C-ABI library loads and exports every entry point include/*.h declares
(no GPU needed: nothing here launches a kernel)."""
import ctypes as C
import os
import re

import pytest

from paper_1008_1685_amd import _native as N
from workloads import preset

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    inc = os.path.join(ROOT, "include")
    txt = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc))
                  if f.endswith(".h"))
    return sorted(set(re.findall(r"\b(pic(?:2d)?_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = N.load()
    names = _declared()
    assert len(names) >= 30
    assert "pic2d_push_deposit" in names
    for n in names:
        assert hasattr(lib, n), n
        assert n in N.SIGNATURES, f"{n} not declared in the binding"


def test_struct_layouts_match_header_sizes():
    # pic_config: validated by struct_size; a wrong layout is rejected
    lib = N.load()
    c = N.PicConfig()
    c.struct_size = C.sizeof(N.PicConfig) + 8
    n = C.c_size_t()
    assert lib.pic_workspace_bytes(C.byref(c), C.byref(n)) == N.PIC_EINVAL
    assert b"struct_size" in lib.pic_last_error()


def test_workspace_bytes_and_validation_on_host():
    from paper_1008_1685_amd.run import make_config
    lib = N.load()
    sizes = {}
    for name in ("c1", "c2", "c3"):
        c = make_config(preset(name))
        n = C.c_size_t()
        assert lib.pic_workspace_bytes(C.byref(c), C.byref(n)) == N.PIC_OK
        sizes[name] = n.value
    assert sizes["c1"] < sizes["c2"] < sizes["c3"]
    # c3: 5e6 particles per species, two buffers, 24 B + 12 B residuals (electrons)
    assert sizes["c3"] > 2 * 5e6 * (24 + 12 + 24)
    for bad in (dict(cfl=0.6), dict(ppc=0), dict(x_foil=99.0), dict(cells_per_lambda=2)):
        c = make_config(preset("c1", **bad))
        assert lib.pic_workspace_bytes(C.byref(c), C.byref(n)) == N.PIC_EINVAL


def test_null_arguments_are_rejected_without_a_gpu():
    lib = N.load()
    assert lib.pic_check_rounding(0x3F800000, 16, None, None) == N.PIC_EINVAL
    cnt = C.c_ulonglong(0)
    assert lib.pic_check_rounding(0xFFFFFFF0, 32, C.byref(cnt), None) == N.PIC_EINVAL
    assert lib.pic_step(None, 1, None) == N.PIC_EINVAL
    assert lib.pic_diag(None, None, None) == N.PIC_EINVAL
    c = N.PicConfig()
    h = C.c_void_p()
    from paper_1008_1685_amd.run import make_config
    c = make_config(preset("c1"))
    assert lib.pic_init(C.byref(c), None, 0, None, C.byref(h)) == N.PIC_EINVAL


def test_track_and_particle_reads_validate_on_the_host():
    lib = N.load()
    w = N.PicWave(10.0, 0.0, 0.0)
    x = (C.c_double * 4)()
    args = lambda **k: dict(dict(wave=C.byref(w), scheme=0, rr=1, prec=N.PIC_FP64, lam=0.8, dt=0.01,
                                 t0=0.0, steps=10, n=4, p=C.cast(x, C.c_void_p)), **k)

    def call(a):
        return lib.pic_track(a["wave"], a["scheme"], a["rr"], a["prec"], a["lam"], a["dt"], a["t0"],
                             a["steps"], a["n"], a["p"], a["p"], a["p"], a["p"], None)

    assert call(args(wave=None)) == N.PIC_EINVAL
    assert call(args(scheme=7)) == N.PIC_EINVAL
    assert call(args(rr=3)) == N.PIC_EINVAL
    assert call(args(prec=5)) == N.PIC_EINVAL
    assert call(args(dt=0.0)) == N.PIC_EINVAL
    assert call(args(lam=-1.0)) == N.PIC_EINVAL
    assert call(args(steps=-1)) == N.PIC_EINVAL
    assert call(args(p=None)) == N.PIC_EINVAL
    assert call(args(t0=float("nan"))) == N.PIC_EINVAL
    w.a_y = float("inf")
    assert call(args()) == N.PIC_EINVAL
    # nothing to do: no launch, no device needed
    w.a_y = 10.0
    assert call(args(n=0, p=None)) == N.PIC_OK
    sp = N.PicSpeciesState()
    assert lib.pic_get_particles(None, 0, 0, 1, C.byref(sp), None) == N.PIC_EINVAL


def test_2d_config_validation_on_host():
    from paper_1008_1685_amd.run2d import make_config
    from workloads import preset2d
    lib = N.load()
    n = C.c_size_t()
    sizes = {}
    for name in ("d1", "d2"):
        c = make_config(preset2d(name))
        assert lib.pic2d_workspace_bytes(C.byref(c), C.byref(n)) == N.PIC_OK
        sizes[name] = n.value
    # d2: 4.2e6 particles per species in two buffers, 40 B each (electrons), plus grids
    assert sizes["d2"] > 2 * 4.19e6 * (28 + 40) and sizes["d1"] < sizes["d2"]
    for bad in (dict(cfl=0.6), dict(ppc_x=0), dict(x_foil=99.0), dict(box_y=0.01),
                dict(waist=-1.0), dict(cells_per_lambda=2)):
        c = make_config(preset2d("d1", **bad))
        assert lib.pic2d_workspace_bytes(C.byref(c), C.byref(n)) == N.PIC_EINVAL, bad
    # field kernel choice: unknown values, and column strips over a period
    # longer than one work-group (1,024 rows in FP32, 512 in FP64)
    c = make_config(preset2d("d1"))
    c.field_kernel = 3
    assert lib.pic2d_workspace_bytes(C.byref(c), C.byref(n)) == N.PIC_EINVAL
    for prec, rows, ok in (("fp32", 1024, True), ("fp32", 1056, False), ("fp64", 512, True),
                           ("fp64", 544, False)):
        c = make_config(preset2d("d1", precision=prec, box_y=rows / 32, field_kernel="strips"))
        want = N.PIC_OK if ok else N.PIC_EINVAL
        assert lib.pic2d_workspace_bytes(C.byref(c), C.byref(n)) == want, (prec, rows)
        c = make_config(preset2d("d1", precision=prec, box_y=rows / 32))  # automatic: any period
        assert lib.pic2d_workspace_bytes(C.byref(c), C.byref(n)) == N.PIC_OK
    c = make_config(preset2d("d1"))
    c.struct_size = C.sizeof(N.Pic2dConfig) - 8
    assert lib.pic2d_workspace_bytes(C.byref(c), C.byref(n)) == N.PIC_EINVAL
    assert b"struct_size" in lib.pic_last_error()
    h = C.c_void_p()
    c = make_config(preset2d("d1"))
    assert lib.pic2d_init(C.byref(c), None, 0, None, C.byref(h)) == N.PIC_EINVAL
    assert lib.pic2d_step(None, 1, None) == N.PIC_EINVAL
    assert lib.pic2d_diag(None, None, None) == N.PIC_EINVAL
    assert lib.pic2d_get_state(None, None, None) == N.PIC_EINVAL
    assert lib.pic2d_timing_enable(None, 1) == N.PIC_EINVAL


def test_the_copy_ceiling_library_exports_its_entry_point():
    # stream_copy (include/stream_copy.h): the measured copy ceiling of the
    # roofline, built beside the main library
    lib = C.CDLL(os.path.join(ROOT, "paper_1008_1685_amd", "libstreamcopy.so"))
    assert hasattr(lib, "stream_copy")
    txt = open(os.path.join(ROOT, "include", "stream_copy.h")).read()
    assert "int stream_copy(const void* src, void* dst, size_t bytes, void* stream);" in txt
