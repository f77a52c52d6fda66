"""starmm: space-bounded divide-and-conquer matrix multiplication on MI355X.

Python face of the C ABI in include/starmm.h.  The functions here take torch
tensors only to read their device pointers and the current HIP stream; all
arithmetic runs in the library's HIP kernels (libstarmm.so in this
directory).  Nothing here computes a product on the host.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (CLASSIC, DT_BF16, DT_F16, DT_F32, DT_I32, FLAG_CHECKED_RANGE, FLAG_OVERWRITE_C, FLAG_NONDETERMINISTIC, FLAG_PERSISTENT, FLAG_SPLIT_IN_KERNEL, MAX_MIN, PERSIST_SLOTS, STATIC_SCRATCH_BYTES,
                   MAX_PLUS, MIN_PLUS, OR_AND, MM_ERR_HIP, MM_ERR_INVALID_ARG, MM_ERR_UNSUPPORTED,
                   MM_ERR_WORKSPACE, MM_ERR_INCOMPLETE, MM_OK, PLUS_TIMES, PREC_BF16, PREC_BF16X3,
                   PREC_BF16X3_HIACC, PREC_F32, PREC_FP16X3, PREC_FP16X3_HIACC, WINOGRAD, PlanInfo, Schedule,
                   StarmmError, TunedEntry, BilinearScheme, BILINEAR_CLASSICAL, BILINEAR_STRASSEN,
                   BILINEAR_MAX_GRID, BILINEAR_MAX_PRODUCTS, make_schedule, strassen_layout)

INF = 1 << 30

__all__ = [
    "semiring_mm", "semiring_mm_static", "STATIC_SCRATCH_BYTES", "strassen_mm", "persistent_status", "MM_ERR_INCOMPLETE", "plan", "workspace_bytes", "strassen_workspace_bytes",
    "make_schedule", "strassen_layout", "Schedule", "PlanInfo", "StarmmError", "INF",
    "PLUS_TIMES", "MIN_PLUS", "MAX_PLUS", "MAX_MIN", "OR_AND", "DT_I32", "DT_F32", "DT_BF16", "DT_F16",
    "PREC_F32", "PREC_BF16X3", "PREC_BF16X3_HIACC", "PREC_BF16", "PREC_FP16X3", "PREC_FP16X3_HIACC", "CLASSIC",
    "WINOGRAD",
    "FLAG_NONDETERMINISTIC", "profile_enable", "profile_reset", "profile_summary",
    "batched_mm", "batched_workspace_bytes", "BatchedGraph", "measured_peaks", "FLAG_SPLIT_IN_KERNEL", "FLAG_PERSISTENT", "PERSIST_SLOTS",
    "FLAG_CHECKED_RANGE", "FLAG_OVERWRITE_C", "domain_violations",
    "bilinear_mm", "bilinear_workspace_bytes", "bilinear_scheme", "bilinear_scheme_product",
    "bilinear_scheme_from_arrays", "bilinear_scheme_arrays", "bilinear_scheme_ok", "BilinearScheme",
    "BILINEAR_CLASSICAL", "BILINEAR_STRASSEN", "BILINEAR_MAX_GRID", "BILINEAR_MAX_PRODUCTS", "TunedEntry", "cost_model_load", "tuned_load", "selection_clear", "propose_schedule", "tuned_lookup",
]


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.int32:
        return DT_I32
    if t.dtype == torch.float32:
        return DT_F32
    if t.dtype == torch.bfloat16:
        return DT_BF16
    if t.dtype == torch.float16:
        return DT_F16
    raise TypeError(f"unsupported dtype {t.dtype}")


def _check_matrix(t, name):
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    # (an empty matrix or a single column reads no column neighbours, so any
    # column stride will do)
    if t.numel() > 0 and t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must be row-major (unit column stride)")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ld(t):
    return max(t.stride(0), t.shape[1], 1)


def semiring_mm(A, B, C, semiring: int = PLUS_TIMES, workspace=None, schedule: Schedule | None = None,
                stream=None, check_persistent: bool = True) -> None:
    """C <- C (+) A (x) B on the device (mm_semiring).

    A: m x k, B: k x n, C: m x n, row-major device tensors (int32 for (min,+),
    (max,+), (max, min) and Boolean (or, and) on 0/1; float32, bfloat16 or float16 A/B with float32 C for (+,x)).  ``workspace`` is
    a uint8 device tensor whose size is the space budget (None = no budget).
    A persistent launch (``FLAG_PERSISTENT`` in the schedule) is followed by
    ``persistent_status`` unless ``check_persistent`` is false: that waits
    for the stream and raises if a bounded wait gave up (C incomplete).
    """
    for t, nm in ((A, "A"), (B, "B"), (C, "C")):
        _check_matrix(t, nm)
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch")
    dt = _dtype_code(A)
    if _dtype_code(B) != dt:
        raise TypeError("A and B must share a dtype")
    ws_ptr = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = _lib.lib().mm_semiring(semiring, dt, m, n, k, ctypes.c_void_p(A.data_ptr()), _ld(A),
                                ctypes.c_void_p(B.data_ptr()), _ld(B), ctypes.c_void_p(C.data_ptr()),
                                _ld(C), ws_ptr, ws_bytes, _lib._sched_ptr(schedule),
                                _stream_handle(stream))
    if st != MM_OK:
        raise StarmmError(st, "mm_semiring")
    # (an empty product launches nothing and leaves no status word)
    if check_persistent and schedule is not None and (schedule.flags & FLAG_PERSISTENT) and m * n * k > 0:
        persistent_status(workspace, stream)


def semiring_mm_static(A, B, C, semiring: int = PLUS_TIMES, schedule: Schedule | None = None,
                       stream=None) -> None:
    """C <- C (+) A (x) B on the device with the library's static scratch as
    the workspace (mm_semiring_static): no device allocation by the call.
    Tensors as in ``semiring_mm``; a schedule needing more than
    STATIC_SCRATCH_BYTES raises (MM_ERR_WORKSPACE)."""
    for t, nm in ((A, "A"), (B, "B"), (C, "C")):
        _check_matrix(t, nm)
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch")
    dt = _dtype_code(A)
    if _dtype_code(B) != dt:
        raise TypeError("A and B must share a dtype")
    st = _lib.lib().mm_semiring_static(semiring, dt, m, n, k, ctypes.c_void_p(A.data_ptr()), _ld(A),
                                       ctypes.c_void_p(B.data_ptr()), _ld(B), ctypes.c_void_p(C.data_ptr()),
                                       _ld(C), _lib._sched_ptr(schedule), _stream_handle(stream))
    if st != MM_OK:
        raise StarmmError(st, "mm_semiring_static")


def persistent_status(workspace, stream=None) -> None:
    """Raise StarmmError(MM_ERR_INCOMPLETE) if the last persistent product that
    used ``workspace`` left C incomplete (mm_persistent_status; waits for the
    stream)."""
    ws_ptr = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = _lib.lib().mm_persistent_status(ws_ptr, ws_bytes, _stream_handle(stream))
    if st != MM_OK:
        raise StarmmError(st, "mm_persistent_status")


def bilinear_scheme(kind: int, param: int) -> "_lib.BilinearScheme":
    """A built-in bilinear scheme (mm_bilinear_builtin): BILINEAR_CLASSICAL
    with param = grid edge g, or BILINEAR_STRASSEN with param = CLASSIC or
    WINOGRAD."""
    s = _lib.BilinearScheme()
    st = _lib.lib().mm_bilinear_builtin(kind, param, ctypes.byref(s))
    if st != MM_OK:
        raise StarmmError(st, "mm_bilinear_builtin")
    return s


def bilinear_scheme_product(s1, s2) -> "_lib.BilinearScheme":
    """s1 over the coarse grid, s2 inside each block, as one flat level
    (mm_bilinear_product)."""
    s = _lib.BilinearScheme()
    st = _lib.lib().mm_bilinear_product(ctypes.byref(s1), ctypes.byref(s2), ctypes.byref(s))
    if st != MM_OK:
        raise StarmmError(st, "mm_bilinear_product")
    return s


def bilinear_scheme_from_arrays(g: int, alpha, beta, gamma) -> "_lib.BilinearScheme":
    """A scheme from nested sequences: alpha and beta R x g*g, gamma g*g x R."""
    s = _lib.BilinearScheme()
    R = len(alpha)
    if not (1 <= g <= _lib.BILINEAR_MAX_GRID and 1 <= R <= _lib.BILINEAR_MAX_PRODUCTS):
        raise ValueError("grid or product count out of range")
    s.g, s.products = g, R
    for r in range(R):
        for p in range(g * g):
            s.alpha[r * g * g + p] = int(alpha[r][p])
            s.beta[r * g * g + p] = int(beta[r][p])
    for c in range(g * g):
        for r in range(R):
            s.gamma[c * R + r] = int(gamma[c][r])
    return s


def bilinear_scheme_arrays(s):
    """(g, alpha, beta, gamma) of a scheme as nested lists (R x g*g, R x g*g,
    g*g x R)."""
    g, R = s.g, s.products
    alpha = [[s.alpha[r * g * g + p] for p in range(g * g)] for r in range(R)]
    beta = [[s.beta[r * g * g + p] for p in range(g * g)] for r in range(R)]
    gamma = [[s.gamma[c * R + r] for r in range(R)] for c in range(g * g)]
    return g, alpha, beta, gamma


def bilinear_scheme_ok(s) -> bool:
    """Whether the scheme multiplies matrices (mm_bilinear_scheme_check)."""
    return _lib.lib().mm_bilinear_scheme_check(ctypes.byref(s)) == MM_OK


def bilinear_workspace_bytes(m: int, n: int, k: int, scheme, precision: int = PREC_BF16X3) -> int:
    return int(_lib.lib().mm_bilinear_workspace_bytes(m, n, k, ctypes.byref(scheme), precision))


def bilinear_mm(A, B, C, scheme, precision: int = PREC_BF16X3, workspace=None, stream=None) -> None:
    """C <- C + A B over float32 through one level of a bilinear scheme
    (mm_bilinear)."""
    for t, nm in ((A, "A"), (B, "B"), (C, "C")):
        _check_matrix(t, nm)
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch")
    ws_ptr = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = _lib.lib().mm_bilinear(m, n, k, ctypes.c_void_p(A.data_ptr()), _ld(A), ctypes.c_void_p(B.data_ptr()), _ld(B),
                                ctypes.c_void_p(C.data_ptr()), _ld(C), ctypes.byref(scheme), precision, ws_ptr,
                                ws_bytes, _stream_handle(stream))
    if st != MM_OK:
        raise StarmmError(st, "mm_bilinear")


def strassen_mm(A, B, C, depth: int, variant: int = WINOGRAD, precision: int = PREC_BF16X3,
                workspace=None, stream=None) -> None:
    """C <- C + A B over float32 through `depth` Strassen levels (mm_strassen)."""
    for t, nm in ((A, "A"), (B, "B"), (C, "C")):
        _check_matrix(t, nm)
    m, k = A.shape
    _, n = B.shape
    ws_ptr = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = _lib.lib().mm_strassen(m, n, k, ctypes.c_void_p(A.data_ptr()), _ld(A),
                                ctypes.c_void_p(B.data_ptr()), _ld(B), ctypes.c_void_p(C.data_ptr()),
                                _ld(C), depth, variant, precision, ws_ptr, ws_bytes,
                                _stream_handle(stream))
    if st != MM_OK:
        raise StarmmError(st, "mm_strassen")


def _problems(triples):
    arr = (_lib.Problem * max(len(triples), 1))()
    dt = None
    for i, (A, B, C) in enumerate(triples):
        for t, nm in ((A, "A"), (B, "B"), (C, "C")):
            _check_matrix(t, nm)
        m, k = A.shape
        k2, n = B.shape
        if k2 != k or tuple(C.shape) != (m, n):
            raise ValueError(f"problem {i}: shape mismatch")
        d = _dtype_code(A)
        if _dtype_code(B) != d or d == DT_I32:
            raise TypeError(f"problem {i}: A and B must both be float32, both bfloat16 or both float16")
        if dt is None:
            dt = d
        elif d != dt:
            raise TypeError("all problems of a batch share one input dtype")
        arr[i] = _lib.Problem(m, n, k, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), C.data_ptr(), _ld(C))
    return arr, (DT_BF16 if dt is None else dt)


def _sched_array(schedules, count):
    if schedules is None:
        return None
    if len(schedules) != count:
        raise ValueError("one schedule per problem")
    arr = (Schedule * max(count, 1))()
    for i, s in enumerate(schedules):
        arr[i] = s
    return arr


def batched_workspace_bytes(triples, schedules=None) -> int:
    arr, dt = _problems(triples)
    return int(_lib.lib().mm_batched_workspace_bytes(len(triples), arr, dt, _sched_array(schedules, len(triples))))


def batched_mm(triples, schedules=None, workspace=None, stream=None) -> None:
    """C_i += A_i B_i for every (A_i, B_i, C_i) in one persistent launch (mm_batched)."""
    arr, dt = _problems(triples)
    ws_ptr = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = _lib.lib().mm_batched(len(triples), arr, dt, _sched_array(schedules, len(triples)), ws_ptr, ws_bytes,
                               _stream_handle(stream))
    if st != MM_OK:
        raise StarmmError(st, "mm_batched")


class BatchedGraph:
    """A batch captured once as a hipGraph of the persistent kernel (mm_batched_graph_*)."""

    def __init__(self, triples, schedules=None, workspace=None, stream=None):
        arr, dt = _problems(triples)
        ws_ptr = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
        ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
        h = ctypes.c_void_p()
        st = _lib.lib().mm_batched_graph_create(len(triples), arr, dt, _sched_array(schedules, len(triples)),
                                                 ws_ptr, ws_bytes, _stream_handle(stream), ctypes.byref(h))
        if st != MM_OK:
            raise StarmmError(st, "mm_batched_graph_create")
        self._h = h
        self._keep = (triples, workspace)

    def launch(self, stream=None) -> None:
        st = _lib.lib().mm_batched_graph_launch(self._h, _stream_handle(stream))
        if st != MM_OK:
            raise StarmmError(st, "mm_batched_graph_launch")

    def close(self) -> None:
        if self._h:
            _lib.lib().mm_batched_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan(semiring: int, dtype: int, m: int, n: int, k: int, workspace_bytes: int,
         schedule: Schedule | None = None):
    """Resolve a schedule on the host (mm_plan).  Returns (status, PlanInfo dict or None)."""
    info = PlanInfo()
    st = _lib.lib().mm_plan(semiring, dtype, m, n, k, workspace_bytes, _lib._sched_ptr(schedule),
                            ctypes.byref(info))
    return st, (info.as_dict() if st == MM_OK else None)


def workspace_bytes(semiring: int, dtype: int, m: int, n: int, k: int,
                    schedule: Schedule | None = None) -> int:
    return int(_lib.lib().mm_workspace_bytes(semiring, dtype, m, n, k, _lib._sched_ptr(schedule)))


def domain_violations(X, semiring: int, flags: int = 0, stream=None) -> int:
    """Entries of the int32 device matrix X outside the input domain of the
    semiring under the schedule flags (mm_domain_violations); synchronises."""
    torch = _torch()
    _check_matrix(X, "X")
    if X.dtype != torch.int32:
        raise TypeError("X must be int32")
    count = torch.empty(1, dtype=torch.int64, device=X.device)
    st = _lib.lib().mm_domain_violations(semiring, flags, ctypes.c_void_p(X.data_ptr()), X.shape[0], X.shape[1],
                                         _ld(X), ctypes.c_void_p(count.data_ptr()), _stream_handle(stream))
    if st != MM_OK:
        raise StarmmError(st, "mm_domain_violations")
    return int(count.item())


def cost_model_load(params) -> None:
    """Load the cost model (mm_cost_model_load) from a flat float sequence:
    t_mean, t_std, then W (out x in) and b of every layer."""
    L = _lib.lib()
    vals = [float(x) for x in params]
    buf = (ctypes.c_float * len(vals))(*vals)
    st = L.mm_cost_model_load(buf, len(vals))
    if st != MM_OK:
        raise StarmmError(st, "mm_cost_model_load")


def tuned_load(entries) -> None:
    """Load measured timings (mm_tuned_load): an iterable of
    (semiring, dtype, m, n, k, Schedule, ms)."""
    entries = list(entries)
    arr = (TunedEntry * max(len(entries), 1))()
    for i, (sr, dt, m, n, k, sched, ms) in enumerate(entries):
        arr[i] = TunedEntry(sr, dt, m, n, k, sched, ms)
    st = _lib.lib().mm_tuned_load(arr, len(entries))
    if st != MM_OK:
        raise StarmmError(st, "mm_tuned_load")


def selection_clear() -> None:
    """Back to the built-in planner for calls without a schedule."""
    _lib.lib().mm_schedule_selection_clear()


def _pick(fn, semiring, dtype, m, n, k, workspace_bytes):
    out, t = Schedule(), ctypes.c_double(0.0)
    st = fn(semiring, dtype, m, n, k, workspace_bytes, ctypes.byref(out), ctypes.byref(t))
    return st, (out if st == MM_OK else None), (t.value if st == MM_OK else None)


def propose_schedule(semiring: int, dtype: int, m: int, n: int, k: int, workspace_bytes: int):
    """The cost model's proposal (mm_propose_schedule): (status, Schedule or None, predicted ms or None)."""
    return _pick(_lib.lib().mm_propose_schedule, semiring, dtype, m, n, k, workspace_bytes)


def tuned_lookup(semiring: int, dtype: int, m: int, n: int, k: int, workspace_bytes: int):
    """The fastest loaded timing that fits (mm_tuned_lookup): (status, Schedule or None, ms or None)."""
    return _pick(_lib.lib().mm_tuned_lookup, semiring, dtype, m, n, k, workspace_bytes)


def profile_enable(on: bool = True) -> None:
    """Bracket every library kernel launch with HIP events on its stream."""
    _lib.lib().mm_profile_enable(1 if on else 0)


def profile_reset() -> None:
    _lib.lib().mm_profile_reset()


def profile_summary() -> dict:
    """{kernel family: (launches, total milliseconds)} of the recorded launches."""
    import json
    L = _lib.lib()
    need = L.mm_profile_summary(None, 0)
    buf = ctypes.create_string_buffer(int(need) + 1)
    L.mm_profile_summary(buf, len(buf))
    return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}


def measured_peaks(stream=None):
    """Achievable rates on this device from the library's microbenchmarks:
    int32 VALU lane-ops/s, bf16 and fp32 MFMA flop/s, copy bytes/s."""
    torch = _torch()
    L = _lib.lib()
    small = torch.empty(1 << 16, dtype=torch.int32, device="cuda")
    big_a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    big_b = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    out = {}
    for kind, name, iters in ((0, "valu_i32_ops", 20000), (1, "mfma_bf16_flops", 20000),
                              (2, "mfma_f32_flops", 5000), (3, "copy_bytes", 0)):
        best = 0.0
        for _ in range(3):
            work = ctypes.c_double()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            st = L.mm_microbench(kind, iters, ctypes.c_void_p((big_a if kind == 3 else small).data_ptr()),
                                 ctypes.c_void_p(big_b.data_ptr()), big_a.numel(), ctypes.byref(work),
                                 _stream_handle(stream))
            e1.record()
            e1.synchronize()
            if st != MM_OK:
                raise StarmmError(st, "mm_microbench")
            best = max(best, work.value / (e0.elapsed_time(e1) * 1e-3))
        out[name] = best
    return out


def strassen_workspace_bytes(m: int, n: int, k: int, depth: int, variant: int = WINOGRAD,
                             precision: int = PREC_BF16X3) -> int:
    return int(_lib.lib().mm_strassen_workspace_bytes(m, n, k, depth, variant, precision))
