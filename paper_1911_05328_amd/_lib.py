"""ctypes binding of libstarmm.so (the C ABI declared in include/starmm.h).

Argument marshalling only: every step of a product runs in the library's HIP
kernels.  The library is loaded from this package directory; if it is
missing, loading raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# STARMM_LIBRARY names another build of the same library (e.g. the
# host-sanitizer build of build.py --sanitize)
LIB_PATH = os.environ.get("STARMM_LIBRARY") or os.path.join(_HERE, "libstarmm.so")

MM_OK, MM_ERR_INVALID_ARG, MM_ERR_UNSUPPORTED, MM_ERR_WORKSPACE, MM_ERR_HIP, MM_ERR_INCOMPLETE = 0, -1, -2, -3, -4, -5
PLUS_TIMES, MIN_PLUS, MAX_PLUS, MAX_MIN, OR_AND = 0, 1, 2, 3, 4
DT_I32, DT_F32, DT_BF16, DT_F16 = 0, 1, 2, 3
PREC_F32, PREC_BF16X3, PREC_BF16X3_HIACC, PREC_BF16, PREC_FP16X3, PREC_FP16X3_HIACC = 0, 1, 2, 3, 4, 5
CLASSIC, WINOGRAD = 0, 1
FLAG_NONDETERMINISTIC = 1
FLAG_SPLIT_IN_KERNEL = 2
FLAG_PERSISTENT = 4
FLAG_CHECKED_RANGE = 8
FLAG_OVERWRITE_C = 16
PERSIST_SLOTS = 2048
STATIC_SCRATCH_BYTES = 64 << 20
STRASSEN_LAYOUT_GIVEN = 0x100


class Schedule(ctypes.Structure):
    _fields_ = [
        ("tile", ctypes.c_int32),
        ("split_k", ctypes.c_int32),
        ("star_depth", ctypes.c_int32),
        ("strassen_depth", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("band_rows", ctypes.c_int64),
        ("flags", ctypes.c_int32),
        ("strassen_layout", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("sched", Schedule),
        ("tile_k", ctypes.c_int32),
        ("tar_levels", ctypes.c_int32),
        ("sar_levels", ctypes.c_int32),
        ("bands", ctypes.c_int64),
        ("tiles_m", ctypes.c_int64),
        ("tiles_n", ctypes.c_int64),
        ("workgroups", ctypes.c_int64),
        ("temp_elems", ctypes.c_int64),
        ("ws_bytes", ctypes.c_int64),
        ("leaf_m", ctypes.c_int64),
        ("leaf_n", ctypes.c_int64),
        ("leaf_k", ctypes.c_int64),
        ("leaves", ctypes.c_int64),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "sched"}
        d["sched"] = self.sched.as_dict()
        return d


class TunedEntry(ctypes.Structure):
    _fields_ = [
        ("semiring", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
        ("sched", Schedule),
        ("ms", ctypes.c_double),
    ]


class Problem(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
        ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
        ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
        ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64),
    ]


BILINEAR_MAX_GRID = 4
BILINEAR_MAX_PRODUCTS = 64
BILINEAR_CLASSICAL, BILINEAR_STRASSEN = 0, 1
_BL_N = BILINEAR_MAX_PRODUCTS * BILINEAR_MAX_GRID * BILINEAR_MAX_GRID


class BilinearScheme(ctypes.Structure):
    """mm_bilinear_scheme: grid g, R products, alpha[r*g*g + p],
    beta[r*g*g + q], gamma[c*R + r] (int8)."""
    _fields_ = [
        ("g", ctypes.c_int32),
        ("products", ctypes.c_int32),
        ("alpha", ctypes.c_int8 * _BL_N),
        ("beta", ctypes.c_int8 * _BL_N),
        ("gamma", ctypes.c_int8 * _BL_N),
    ]


class StarmmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status}) {last_error()}")


_lib = None


def lib():
    """The loaded library (raises OSError if libstarmm.so is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is not built; run paper_1911_05328_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        L.mm_semiring.argtypes = [I32, I32, I64, I64, I64, P, I64, P, I64, P, I64, P, SZ,
                                  ctypes.POINTER(Schedule), P]
        L.mm_semiring.restype = I32
        L.mm_semiring_static.argtypes = [I32, I32, I64, I64, I64, P, I64, P, I64, P, I64,
                                         ctypes.POINTER(Schedule), P]
        L.mm_semiring_static.restype = I32
        L.mm_strassen.argtypes = [I64, I64, I64, P, I64, P, I64, P, I64, I32, I32, I32, P, SZ, P]
        L.mm_strassen.restype = I32
        L.mm_strassen_workspace_bytes.argtypes = [I64, I64, I64, I32, I32, I32]
        L.mm_strassen_workspace_bytes.restype = SZ
        L.mm_plan.argtypes = [I32, I32, I64, I64, I64, SZ, ctypes.POINTER(Schedule),
                              ctypes.POINTER(PlanInfo)]
        L.mm_plan.restype = I32
        L.mm_workspace_bytes.argtypes = [I32, I32, I64, I64, I64, ctypes.POINTER(Schedule)]
        L.mm_workspace_bytes.restype = SZ
        L.mm_persistent_status.argtypes = [P, SZ, P]
        L.mm_persistent_status.restype = I32
        L.mm_status_string.argtypes = [I32]
        L.mm_status_string.restype = ctypes.c_char_p
        L.mm_last_error.argtypes = []
        L.mm_last_error.restype = ctypes.c_char_p
        L.mm_version.argtypes = []
        L.mm_version.restype = I32
        I64P = ctypes.POINTER(ctypes.c_int64)
        L.mm_tile_order.argtypes = [I64, I64, I64P, I64P]
        L.mm_tile_order.restype = I32
        L.mm_microbench.argtypes = [I32, I64, P, P, I64, ctypes.POINTER(ctypes.c_double), P]
        L.mm_microbench.restype = I32
        L.mm_profile_enable.argtypes = [I32]
        L.mm_profile_enable.restype = None
        L.mm_profile_reset.argtypes = []
        L.mm_profile_reset.restype = None
        L.mm_profile_summary.argtypes = [ctypes.c_char_p, SZ]
        L.mm_profile_summary.restype = I64
        I8P = ctypes.POINTER(ctypes.c_int8)
        L.mm_strassen_coefficients.argtypes = [I32, I8P, I8P, I8P]
        L.mm_strassen_coefficients.restype = I32
        BSP = ctypes.POINTER(BilinearScheme)
        L.mm_bilinear_builtin.argtypes = [I32, I32, BSP]
        L.mm_bilinear_builtin.restype = I32
        L.mm_bilinear_product.argtypes = [BSP, BSP, BSP]
        L.mm_bilinear_product.restype = I32
        L.mm_bilinear_scheme_check.argtypes = [BSP]
        L.mm_bilinear_scheme_check.restype = I32
        L.mm_bilinear_workspace_bytes.argtypes = [I64, I64, I64, BSP, I32]
        L.mm_bilinear_workspace_bytes.restype = SZ
        L.mm_bilinear.argtypes = [I64, I64, I64, P, I64, P, I64, P, I64, BSP, I32, P, SZ, P]
        L.mm_bilinear.restype = I32
        F = ctypes.c_float
        L.mm_mlp_linear_forward.argtypes = [I64, I64, I64, P, P, P, P, I32, P]
        L.mm_mlp_linear_forward.restype = I32
        L.mm_mlp_linear_backward.argtypes = [I64, I64, I64, P, P, P, P, P, P, P, P, I32, P]
        L.mm_mlp_linear_backward.restype = I32
        L.mm_mlp_masked_mse.argtypes = [I64, P, P, P, P, P, P]
        L.mm_mlp_masked_mse.restype = I32
        L.mm_mlp_adam.argtypes = [I64, P, P, P, P, F, F, F, F, I32, P]
        L.mm_mlp_adam.restype = I32
        PP, SP = ctypes.POINTER(Problem), ctypes.POINTER(Schedule)
        L.mm_batched_workspace_bytes.argtypes = [I32, PP, I32, SP]
        L.mm_batched_workspace_bytes.restype = SZ
        L.mm_batched.argtypes = [I32, PP, I32, SP, P, SZ, P]
        L.mm_batched.restype = I32
        L.mm_batched_graph_create.argtypes = [I32, PP, I32, SP, P, SZ, P, ctypes.POINTER(ctypes.c_void_p)]
        L.mm_batched_graph_create.restype = I32
        L.mm_batched_graph_launch.argtypes = [P, P]
        L.mm_batched_graph_launch.restype = I32
        L.mm_batched_graph_destroy.argtypes = [P]
        L.mm_batched_graph_destroy.restype = None
        L.mm_domain_violations.argtypes = [I32, I32, P, I64, I64, I64, P, P]
        L.mm_domain_violations.restype = I32
        L.mm_cost_model_param_count.argtypes = []
        L.mm_cost_model_param_count.restype = I64
        L.mm_cost_model_load.argtypes = [ctypes.POINTER(ctypes.c_float), I64]
        L.mm_cost_model_load.restype = I32
        L.mm_tuned_load.argtypes = [ctypes.POINTER(TunedEntry), I64]
        L.mm_tuned_load.restype = I32
        L.mm_schedule_selection_clear.argtypes = []
        L.mm_schedule_selection_clear.restype = None
        DP = ctypes.POINTER(ctypes.c_double)
        L.mm_propose_schedule.argtypes = [I32, I32, I64, I64, I64, SZ, SP, DP]
        L.mm_propose_schedule.restype = I32
        L.mm_tuned_lookup.argtypes = [I32, I32, I64, I64, I64, SZ, SP, DP]
        L.mm_tuned_lookup.restype = I32
        _lib = L
    return _lib


def status_string(st: int) -> str:
    return lib().mm_status_string(st).decode()


def last_error() -> str:
    return lib().mm_last_error().decode()


def make_schedule(tile=0, split_k=0, star_depth=0, strassen_depth=0, variant=WINOGRAD,
                  precision=PREC_F32, band_rows=0, flags=0, strassen_layout=0) -> Schedule:
    return Schedule(tile, split_k, star_depth, strassen_depth, variant, precision, band_rows, flags,
                    strassen_layout)


def strassen_layout(depth_first_mask: int) -> int:
    """The schedule's strassen_layout value making levels with their bit set
    (bit 0 = the top level) depth-first (MM_STRASSEN_LAYOUT)."""
    return STRASSEN_LAYOUT_GIVEN | depth_first_mask


def _sched_ptr(s):
    return ctypes.byref(s) if s is not None else None
