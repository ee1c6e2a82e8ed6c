"""ctypes declarations of libtffr's C ABI (include/tffr.h, include/tffr_debug.h).

Loading fails loudly when the library has not been built: there is no fallback path.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtffr.so")

TFFR_OK = 0
STATUS_NAMES = {0: "TFFR_OK", 1: "TFFR_ERR_ARG", 2: "TFFR_ERR_EVANESCENT", 3: "TFFR_ERR_NONMONOTONE",
                4: "TFFR_ERR_LAYOUT", 5: "TFFR_ERR_UNSUPPORTED", 6: "TFFR_ERR_SINGULAR", 7: "TFFR_ERR_NOMEM",
                8: "TFFR_ERR_HIP", 9: "TFFR_ERR_SCRATCH"}
TFFR_ERR_SCRATCH = 9
SCRATCH_BYTES = 32 << 20

W_NONE, W_QUAD, W_FFR, W_TFFR, W_USER = 0, 1, 2, 3, 4
THRESH_LITERAL, THRESH_CORRELATION = 0, 1
C64, C128, C64_FP16IN = 0, 1, 2
GRID_ES, GRID_LITERAL = 0, 1


class Params(ctypes.Structure):
    _fields_ = [
        ("n_pulses", ctypes.c_int32),
        ("n_freq", ctypes.c_int32),
        ("mx", ctypes.c_int32),
        ("my", ctypes.c_int32),
        ("fov_x", ctypes.c_double),
        ("fov_y", ctypes.c_double),
        ("weighting", ctypes.c_int32),
        ("window_a", ctypes.c_double),
        ("q", ctypes.c_double),
        ("band_r", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("thresh_mode", ctypes.c_int32),
        ("kernel_width", ctypes.c_int32),
        ("upsampfac", ctypes.c_double),
        ("dtype", ctypes.c_int32),
        ("gridding", ctypes.c_int32),
    ]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_PROTOS = {
    "tffr_default_params": (None, [ctypes.POINTER(Params)]),
    "tffr_validate": (ctypes.c_int, [ctypes.POINTER(Params), _dp, _dp]),
    "tffr_plan_create": (ctypes.c_int, [ctypes.POINTER(Params), _dp, _dp, ctypes.POINTER(_vp)]),
    "tffr_validate_xy": (ctypes.c_int, [ctypes.POINTER(Params), _dp, _dp]),
    "tffr_plan_create_xy": (ctypes.c_int, [ctypes.POINTER(Params), _dp, _dp, ctypes.POINTER(_vp)]),
    "tffr_plan_destroy": (None, [_vp]),
    "tffr_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "tffr_plan_info": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      _dp, ctypes.POINTER(ctypes.c_int32)]),
    "tffr_weights": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "tffr_kept_count": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _vp]),
    "tffr_forward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_adjoint": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_entropy": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_entropy_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_entropy_step_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_row_phase_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_coord_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_rma_front_end": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "tffr_rma_range_fft": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "tffr_rma_front_end_pos": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_double,
                                              ctypes.POINTER(ctypes.c_double), ctypes.c_double, _vp, _vp]),
    "tffr_stolt_image": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "tffr_debug_fft": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      _vp, _vp, _vp]),
    "tffr_debug_rows": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_debug_cols": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "tffr_debug_ent_cols": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "tffr_debug_ent_adj_rows": (ctypes.c_int, [_vp] * 11),
    "tffr_debug_step_kernel_times": (ctypes.c_int, [_vp] * 12 + [ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                                                ctypes.POINTER(ctypes.c_int32),
                                                                ctypes.POINTER(ctypes.c_char_p)]),
    "tffr_debug_step_kernel_marginal_times": (ctypes.c_int, [_vp] * 12 + [ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                                                         ctypes.POINTER(ctypes.c_int32),
                                                                         ctypes.POINTER(ctypes.c_char_p)]),
    "tffr_debug_ffr_route": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "tffr_debug_plan_config": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)]),
}

_lib = None


def load():
    """Load libtffr.so (built by paper_1910_10908_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtffr.so not built at {LIB_PATH}; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, what=""):
    if status != TFFR_OK:
        msg = load().tffr_status_string(status).decode()
        raise RuntimeError(f"{what}: {msg}" if what else msg)
