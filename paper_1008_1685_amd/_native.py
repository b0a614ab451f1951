"""ctypes declarations of the C ABI in include/pic.h and include/pic2d.h
(argument marshalling only).

The shared library is built in-tree as ``paper_1008_1685_amd/libpic.so``; a
missing library is an error, there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PIC_LIB may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("PIC_LIB") or os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EHIP, PIC_ENONFINITE, PIC_EBUSY = 0, -1, -2, -3, -4, -5
PIC_FP32, PIC_FP64 = 0, 1
PIC_LP, PIC_CP = 0, 1

STATUS_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EHIP",
                -4: "PIC_ENONFINITE", -5: "PIC_EBUSY"}


class PicConfig(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("precision", C.c_int32),
        ("lambda_um", C.c_double),
        ("cells_per_lambda", C.c_int32),
        ("ppc", C.c_int32),
        ("box_lambda", C.c_double),
        ("cfl", C.c_double),
        ("pol", C.c_int32),
        ("rr", C.c_int32),
        ("a0", C.c_double),
        ("t_rise", C.c_double),
        ("t_flat", C.c_double),
        ("t_fall", C.c_double),
        ("n0", C.c_double),
        ("x_foil", C.c_double),
        ("thickness", C.c_double),
        ("mass_ratio", C.c_double),
        ("rr_compensated", C.c_int32),
        ("sort_interval", C.c_int32),
        ("seed", C.c_uint64),
        ("jitter", C.c_double),
        ("capacity", C.c_int64),
    ]


class PicInfo(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32),
        ("precision", C.c_int32),
        ("dx", C.c_double),
        ("dt", C.c_double),
        ("eps_rr", C.c_double),
        ("w_ref", C.c_double),
        ("capacity", C.c_int64),
        ("n_init", C.c_int64 * 2),
        ("step", C.c_int64),
        ("tile", C.c_int32),
        ("lds_slots", C.c_int32),
    ]


class PicDiagOut(C.Structure):
    _fields_ = [
        ("step", C.c_int64),
        ("t", C.c_double),
        ("n_alive", C.c_int64 * 2),
        ("U_Ex", C.c_double),
        ("U_Et", C.c_double),
        ("U_B", C.c_double),
        ("K_e", C.c_double),
        ("K_i", C.c_double),
        ("E_rad", C.c_double),
        ("E_in", C.c_double),
        ("E_out_left", C.c_double),
        ("E_out_right", C.c_double),
        ("E_esc", C.c_double),
        ("gauss", C.c_double),
        ("gauss_int", C.c_int64),
        ("n_stiff", C.c_int64),
        ("nonfinite", C.c_int32),
        ("reserved", C.c_int32),
        ("U_field", C.c_double),
        ("balance", C.c_double),
    ]


class PicBudgetState(C.Structure):
    _fields_ = [
        ("valid", C.c_int32),
        ("nonfinite", C.c_int32),
        ("E_in", C.c_double),
        ("E_out_left", C.c_double),
        ("E_out_right", C.c_double),
        ("E_rad", C.c_double),
        ("E_esc", C.c_double * 2),
        ("n_stiff", C.c_double),
    ]


BUDGET_KEYS = ("nonfinite", "E_in", "E_out_left", "E_out_right", "E_rad", "E_esc", "n_stiff")


def budget_to_dict(b: "PicBudgetState") -> dict:
    d = {k: getattr(b, k) for k in BUDGET_KEYS}
    d["E_esc"] = (b.E_esc[0], b.E_esc[1])
    return d


def budget_from_dict(d: dict) -> "PicBudgetState":
    b = PicBudgetState()
    b.valid = 1
    b.nonfinite = int(d["nonfinite"])
    for k in ("E_in", "E_out_left", "E_out_right", "E_rad", "n_stiff"):
        setattr(b, k, float(d[k]))
    b.E_esc[0], b.E_esc[1] = (float(x) for x in d["E_esc"])
    return b


class PicWave(C.Structure):
    _fields_ = [("a_y", C.c_double), ("a_z", C.c_double), ("psi", C.c_double)]


PIC_TRACK_LEAPFROG, PIC_TRACK_RK4 = 0, 1
PIC_RR_OFF, PIC_RR_REDUCED, PIC_RR_FULL = 0, 1, 2


class PicSpeciesState(C.Structure):
    _fields_ = [
        ("count", C.c_int64),
        ("cell", C.c_void_p),
        ("off", C.c_void_p),
        ("ux", C.c_void_p),
        ("uy", C.c_void_p),
        ("uz", C.c_void_p),
        ("w", C.c_void_p),
        ("rx", C.c_void_p),
        ("ry", C.c_void_p),
        ("rz", C.c_void_p),
    ]


class PicState(C.Structure):
    _fields_ = [
        ("sp", PicSpeciesState * 2),
        ("Ex", C.c_void_p),
        ("Ey", C.c_void_p),
        ("Ez", C.c_void_p),
        ("By", C.c_void_p),
        ("Bz", C.c_void_p),
        ("Ex_int", C.c_void_p),
        ("Jx_int", C.c_void_p),
        ("Jy_int", C.c_void_p),
        ("Jz_int", C.c_void_p),
        ("step", C.c_int64),
        ("budget", PicBudgetState),
    ]


class Pic2dConfig(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("precision", C.c_int32),
        ("lambda_um", C.c_double),
        ("cells_per_lambda", C.c_int32),
        ("ppc_x", C.c_int32),
        ("ppc_y", C.c_int32),
        ("pol", C.c_int32),
        ("box_x", C.c_double),
        ("box_y", C.c_double),
        ("cfl", C.c_double),
        ("rr", C.c_int32),
        ("rr_compensated", C.c_int32),
        ("a0", C.c_double),
        ("waist", C.c_double),
        ("t_rise", C.c_double),
        ("t_flat", C.c_double),
        ("t_fall", C.c_double),
        ("n0", C.c_double),
        ("x_foil", C.c_double),
        ("thickness", C.c_double),
        ("mass_ratio", C.c_double),
        ("sort_interval", C.c_int32),
        ("field_kernel", C.c_int32),
        ("seed", C.c_uint64),
        ("jitter", C.c_double),
        ("capacity", C.c_int64),
    ]


class Pic2dInfo(C.Structure):
    _fields_ = [
        ("nx", C.c_int32),
        ("ny", C.c_int32),
        ("y_shift", C.c_int32),
        ("precision", C.c_int32),
        ("dx", C.c_double),
        ("dt", C.c_double),
        ("eps_rr", C.c_double),
        ("w_ref", C.c_double),
        ("capacity", C.c_int64),
        ("n_init", C.c_int64 * 2),
        ("step", C.c_int64),
        ("tile", C.c_int32),
        ("lds_slots", C.c_int32),
        ("field_kernel", C.c_int32),
        ("field_blocks", C.c_int32),
        ("sort_block_x_shift", C.c_int32),
        ("sort_block_y_shift", C.c_int32),
        ("reserved_info", C.c_int32),
    ]


class Pic2dSpeciesState(C.Structure):
    _fields_ = [
        ("count", C.c_int64),
        ("cell", C.c_void_p),
        ("ox", C.c_void_p),
        ("oy", C.c_void_p),
        ("ux", C.c_void_p),
        ("uy", C.c_void_p),
        ("uz", C.c_void_p),
        ("w", C.c_void_p),
        ("rx", C.c_void_p),
        ("ry", C.c_void_p),
        ("rz", C.c_void_p),
    ]


class Pic2dState(C.Structure):
    _fields_ = [
        ("sp", Pic2dSpeciesState * 2),
        ("Ex", C.c_void_p),
        ("Ey", C.c_void_p),
        ("Ez", C.c_void_p),
        ("Bx", C.c_void_p),
        ("By", C.c_void_p),
        ("Bz", C.c_void_p),
        ("Jx_int", C.c_void_p),
        ("Jy_int", C.c_void_p),
        ("Jz_int", C.c_void_p),
        ("charge_int", C.c_void_p),
        ("step", C.c_int64),
        ("budget", PicBudgetState),
    ]


# exported symbols: name -> (restype, argtypes)
SIGNATURES = {
    "pic_workspace_bytes": (C.c_int, [C.POINTER(PicConfig), C.POINTER(C.c_size_t)]),
    "pic_init": (C.c_int, [C.POINTER(PicConfig), C.c_void_p, C.c_size_t, C.c_void_p,
                           C.POINTER(C.c_void_p)]),
    "pic_step": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    "pic_diag": (C.c_int, [C.c_void_p, C.POINTER(PicDiagOut), C.c_void_p]),
    "pic_get_info": (C.c_int, [C.c_void_p, C.POINTER(PicInfo)]),
    "pic_free": (None, [C.c_void_p]),
    "pic_last_error": (C.c_char_p, []),
    "pic_push_deposit": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pic_field_advance": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pic_sort": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pic_get_state": (C.c_int, [C.c_void_p, C.POINTER(PicState), C.c_void_p]),
    "pic_set_state": (C.c_int, [C.c_void_p, C.POINTER(PicState), C.c_void_p]),
    "pic_check_rounding": (C.c_int, [C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p]),
    "pic_track": (C.c_int, [C.POINTER(PicWave), C.c_int32, C.c_int32, C.c_int32, C.c_double,
                            C.c_double, C.c_double, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_void_p]),
    "pic_get_particles": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64,
                                    C.POINTER(PicSpeciesState), C.c_void_p]),
    "pic_spectrum": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double),
                               C.c_void_p]),
    "pic_spectrum_static": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double),
                                      C.c_void_p]),
    "pic_friction": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.c_void_p]),
    "pic_set_max_grid": (C.c_int, [C.c_void_p, C.c_int32]),
    "pic_timing_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "pic_timing_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                  C.c_void_p]),
    "pic_batch_workspace_bytes": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "pic_batch_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_int64,
                                   C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pic_batch_admit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.POINTER(C.c_int32)]),
    "pic_batch_fits": (C.c_int, [C.c_void_p, C.POINTER(PicConfig), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]),
    "pic_batch_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "pic_batch_poll": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_void_p]),
    "pic_batch_release": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "pic_batch_set_persistent": (C.c_int, [C.c_void_p, C.c_int32]),
    "pic_batch_drain": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_void_p]),
    "pic_batch_poll_async": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pic_batch_poll_wait": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "pic_batch_free": (None, [C.c_void_p]),
    "pic2d_workspace_bytes": (C.c_int, [C.POINTER(Pic2dConfig), C.POINTER(C.c_size_t)]),
    "pic2d_init": (C.c_int, [C.POINTER(Pic2dConfig), C.c_void_p, C.c_size_t, C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    "pic2d_step": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    "pic2d_push_deposit": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pic2d_field_advance": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pic2d_sort": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pic2d_diag": (C.c_int, [C.c_void_p, C.POINTER(PicDiagOut), C.c_void_p]),
    "pic2d_get_info": (C.c_int, [C.c_void_p, C.POINTER(Pic2dInfo)]),
    "pic2d_free": (None, [C.c_void_p]),
    "pic2d_get_state": (C.c_int, [C.c_void_p, C.POINTER(Pic2dState), C.c_void_p]),
    "pic2d_set_state": (C.c_int, [C.c_void_p, C.POINTER(Pic2dState), C.c_void_p]),
    "pic2d_timing_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "pic2d_timing_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                    C.c_void_p]),
}

_lib = None


class PicError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the library (once) and declare every exported entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with paper_1008_1685_amd.build.build() "
            "(no CPU fallback exists)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, where):
    if status != PIC_OK:
        msg = load().pic_last_error().decode(errors="replace")
        raise PicError(status, where, msg)

