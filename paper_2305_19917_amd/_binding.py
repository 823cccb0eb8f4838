"""ctypes binding of libredsea.so: argument marshalling only.

Every step of a solve runs in the library's HIP kernels; this module turns
PyTorch tensors into pointers, leading dimensions and a stream handle.  It
never computes a result itself and has no CPU fallback: if the library is
missing, importing a function raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libredsea.so")

# Symbols the public header declares.
EXPORTS = (
    "redsea_trsm",
    "redsea_trsm_noalloc",
    "redsea_trsm_batched",
    "redsea_batched_tune",
    "redsea_trsm_mixed",
    "redsea_trmm",
    "redsea_trsm_mixed_workspace_bytes",
    "redsea_status_string",
    "redsea_schedule",
    "redsea_version",
    "redsea_gemm_update",
    "redsea_batched_plan_create",
    "redsea_batched_plan_run",
    "redsea_batched_plan_destroy",
    "redsea_trace_begin",
    "redsea_trace_end",
    "redsea_candidate",
    "redsea_tune_shape",
    "redsea_mlp_param_count",
    "redsea_mlp_forward",
    "redsea_mlp_grad",
    "redsea_mlp_adam",
    "redsea_pick",
    "redsea_mlp_load",
    "redsea_mfma_peak",
    "redsea_potrf",
)
KERNEL_CLASSES = ("pack", "leaf", "gemm", "gemm_group", "thin", "chol_leaf", "syrk")

SIDE = {"L": 0, "R": 1, 0: 0, 1: 1}
UPLO = {"L": 0, "U": 1, 0: 0, 1: 1}
TRANS = {"N": 0, "T": 1, "C": 2, 0: 0, 1: 1, 2: 2}
DIAG = {"N": 0, "U": 1, 0: 0, 1: 1}
VARIANT = {"auto": 0, "recursive": 1, "iterative": 2, "blocked": 3, 0: 0, 1: 1, 2: 2, 3: 3}
PRECISION = {"auto": 0, "native": 1, "fp32_ir": 2, "bf16_ir": 3, 0: 0, 1: 1, 2: 2, 3: 3}

_LIB: Optional[ctypes.CDLL] = None


class RedseaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("redsea error %d: %s" % (code, msg))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("nb", ctypes.c_int), ("precision", ctypes.c_int),
                ("kappa", ctypes.c_double), ("tile", ctypes.c_int)]


class MixedStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("eta", ctypes.c_double), ("fell_back", ctypes.c_int)]


def lib() -> ctypes.CDLL:
    """Load libredsea.so (built by paper_2305_19917_amd.build); raises if absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libredsea.so is not built: run paper_2305_19917_amd/build.py "
                           "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    i64, dbl, ptr, cint, sz = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    L.redsea_mfma_peak.restype = i64
    L.redsea_mfma_peak.argtypes = [cint, i64, ptr, i64, ptr]
    L.redsea_trsm.restype = cint
    L.redsea_trsm.argtypes = [cint, cint, cint, cint, cint, i64, i64, dbl, ptr, i64, ptr, i64,
                              ctypes.POINTER(Opts), ptr]
    L.redsea_trsm_noalloc.restype = cint
    L.redsea_trsm_noalloc.argtypes = L.redsea_trsm.argtypes
    L.redsea_trsm_batched.restype = cint
    L.redsea_trsm_batched.argtypes = [cint, cint, cint, cint, cint, i64, ctypes.POINTER(i64),
                                      ctypes.POINTER(i64), dbl, ctypes.POINTER(ptr),
                                      ctypes.POINTER(i64), ctypes.POINTER(ptr),
                                      ctypes.POINTER(i64), ptr, ctypes.POINTER(Opts), ptr]
    L.redsea_trsm_mixed.restype = cint
    L.redsea_trsm_mixed.argtypes = [cint, cint, cint, cint, i64, i64, dbl, ptr, i64, ptr, i64,
                                    cint, dbl, cint, ptr, sz, ctypes.POINTER(MixedStats), ptr]
    L.redsea_trmm.restype = cint
    L.redsea_trmm.argtypes = [cint, cint, cint, cint, cint, i64, i64, dbl, ptr, i64, ptr, i64, dbl,
                              ptr, i64, cint, ptr]
    L.redsea_potrf.restype = cint
    L.redsea_potrf.argtypes = [cint, cint, i64, ptr, i64, cint, ptr, ptr]
    L.redsea_trsm_mixed_workspace_bytes.restype = sz
    L.redsea_trsm_mixed_workspace_bytes.argtypes = [cint, i64, i64, cint]
    L.redsea_status_string.restype = ctypes.c_char_p
    L.redsea_status_string.argtypes = [cint]
    L.redsea_schedule.restype = i64
    L.redsea_schedule.argtypes = [cint, i64, cint, ptr, i64]
    L.redsea_version.restype = ctypes.c_char_p
    L.redsea_version.argtypes = []
    L.redsea_gemm_update.restype = cint
    L.redsea_gemm_update.argtypes = [cint, cint, cint, i64, i64, i64, ptr, i64, ptr, i64, ptr, i64,
                                     cint, ptr]
    L.redsea_batched_tune.restype = cint
    L.redsea_batched_tune.argtypes = [cint, cint, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), cint,
                                      ctypes.POINTER(dbl), ctypes.POINTER(cint)]
    L.redsea_batched_plan_create.restype = cint
    L.redsea_batched_plan_create.argtypes = [cint, cint, cint, cint, cint, i64, ctypes.POINTER(i64),
                                             ctypes.POINTER(i64), dbl, ctypes.POINTER(ptr),
                                             ctypes.POINTER(i64), ctypes.POINTER(ptr),
                                             ctypes.POINTER(i64), ctypes.POINTER(Opts),
                                             ctypes.POINTER(ptr)]
    L.redsea_batched_plan_run.restype = cint
    L.redsea_batched_plan_run.argtypes = [ptr, ptr, ptr]
    L.redsea_batched_plan_destroy.restype = None
    L.redsea_batched_plan_destroy.argtypes = [ptr]
    L.redsea_candidate.restype = cint
    L.redsea_candidate.argtypes = [cint, ctypes.POINTER(cint), ctypes.POINTER(cint), ctypes.POINTER(cint)]
    L.redsea_tune_shape.restype = cint
    L.redsea_tune_shape.argtypes = [cint, i64, i64, dbl, ctypes.c_uint64, cint, ctypes.POINTER(cint),
                                    cint, ctypes.POINTER(dbl), ptr]
    L.redsea_mlp_param_count.restype = cint
    L.redsea_mlp_param_count.argtypes = []
    L.redsea_mlp_forward.restype = cint
    L.redsea_mlp_forward.argtypes = [ptr, ptr, i64, ptr, ptr]
    L.redsea_mlp_grad.restype = cint
    L.redsea_mlp_grad.argtypes = [ptr, ptr, ptr, ptr, i64, ptr, ptr, ptr]
    L.redsea_mlp_adam.restype = cint
    L.redsea_mlp_adam.argtypes = [ptr, ptr, ptr, ptr, i64, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, ptr]
    L.redsea_pick.restype = cint
    L.redsea_pick.argtypes = [cint, i64, i64, dbl, ctypes.POINTER(cint)]
    L.redsea_mlp_load.restype = cint
    L.redsea_mlp_load.argtypes = [ctypes.c_char_p]
    L.redsea_trace_begin.restype = None
    L.redsea_trace_begin.argtypes = []
    L.redsea_trace_end.restype = cint
    L.redsea_trace_end.argtypes = [ptr, ptr, ptr, cint]
    _LIB = L
    return L


def status_string(code: int) -> str:
    return lib().redsea_status_string(code).decode()


def _check(code: int):
    if code != 0:
        raise RedseaError(code, status_string(code))


def _ld(t) -> int:
    """Leading dimension of a column-major 2-D tensor view (stride(0) == 1)."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.shape[0] > 1 and t.shape[1] > 1 and t.stride(0) != 1:
        raise ValueError("tensor must be column-major (stride(0) == 1); use fortran_tensor()")
    if t.shape[1] <= 1:
        return max(1, t.shape[0])
    return max(1, t.stride(1))


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return 0
    if t.dtype == torch.float32:
        return 1
    raise TypeError("only float64 and float32 tensors are supported")


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def fortran_tensor(arr, device="cuda"):
    """Copy a 2-D numpy array to `device` as a column-major tensor (ld = rows)."""
    import numpy as np
    import torch
    a = np.asarray(arr)
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to(device)
    return t.t()


def trsm(A, B, side="L", uplo="L", trans="N", diag="N", alpha: float = 1.0,
         variant="auto", nb: int = 0, precision="auto", stream=None):
    """In place: B := alpha op(A)^{-1} B (side L) or alpha B op(A)^{-1} (side R).

    A and B are column-major device tensors of the same dtype.  Returns B."""
    m, n = B.shape
    opts = Opts(VARIANT[variant], int(nb), PRECISION[precision])
    rc = lib().redsea_trsm(_dtype_code(B), SIDE[side], UPLO[uplo], TRANS[trans], DIAG[diag],
                           m, n, float(alpha), A.data_ptr(), _ld(A), B.data_ptr(), _ld(B),
                           ctypes.byref(opts), _stream(stream))
    _check(rc)
    return B


def trsm_noalloc(A, B, side="L", uplo="L", trans="N", diag="N", alpha: float = 1.0,
                 variant="auto", nb: int = 0, stream=None):
    """As trsm(), through redsea_trsm_noalloc: native precision, scratch in the
    library's fixed device array, no allocation (graph-capturable)."""
    m, n = B.shape
    opts = Opts(VARIANT[variant], int(nb), PRECISION["native"])
    rc = lib().redsea_trsm_noalloc(_dtype_code(B), SIDE[side], UPLO[uplo], TRANS[trans],
                                   DIAG[diag], m, n, float(alpha), A.data_ptr(), _ld(A),
                                   B.data_ptr(), _ld(B), ctypes.byref(opts), _stream(stream))
    _check(rc)
    return B


def batched_tune(orders, nrhs, dtype: str = "f64", diag="N", reps: int = 2):
    """Time every batched task shape on generated systems of these shapes;
    returns (best candidate 1..12, milliseconds per candidate)."""
    count = len(orders)
    i64 = ctypes.c_int64
    ks = (i64 * max(1, count))(*[int(x) for x in orders])
    rs = (i64 * max(1, count))(*[int(x) for x in nrhs])
    ms = (ctypes.c_double * 12)()
    best = ctypes.c_int()
    _check(lib().redsea_batched_tune(0 if dtype == "f64" else 1, DIAG[diag], count, ks, rs,
                                     int(reps), ms, ctypes.byref(best)))
    return best.value, [float(x) for x in ms]


def trsm_batched(As: Sequence, Bs: Sequence, info, side="L", uplo="L", trans="N", diag="N",
                 alpha: float = 1.0, variant="auto", nb: int = 0, tile: int = 0, stream=None):
    """Batch of independent in-place solves; info is an int32 device tensor."""
    count = len(Bs)
    i64 = ctypes.c_int64
    ms = (i64 * count)(*[b.shape[0] for b in Bs])
    ns = (i64 * count)(*[b.shape[1] for b in Bs])
    ldas = (i64 * count)(*[_ld(a) for a in As])
    ldbs = (i64 * count)(*[_ld(b) for b in Bs])
    aps = (ctypes.c_void_p * count)(*[a.data_ptr() for a in As])
    bps = (ctypes.c_void_p * count)(*[b.data_ptr() for b in Bs])
    opts = Opts(VARIANT[variant], int(nb), 0, 0.0, int(tile))
    dt = _dtype_code(Bs[0]) if count else 0
    rc = lib().redsea_trsm_batched(dt, SIDE[side], UPLO[uplo], TRANS[trans], DIAG[diag], count,
                                   ms, ns, float(alpha), aps, ldas, bps, ldbs, info.data_ptr(),
                                   ctypes.byref(opts), _stream(stream))
    _check(rc)


def _batch_arrays(As, Bs):
    count = len(Bs)
    i64 = ctypes.c_int64
    return (count, (i64 * count)(*[b.shape[0] for b in Bs]), (i64 * count)(*[b.shape[1] for b in Bs]),
            (ctypes.c_void_p * count)(*[a.data_ptr() for a in As]),
            (i64 * count)(*[_ld(a) for a in As]),
            (ctypes.c_void_p * count)(*[b.data_ptr() for b in Bs]),
            (i64 * count)(*[_ld(b) for b in Bs]))


class BatchPlan:
    """A prepared batch (redsea_batched_plan_*): run() only launches kernels,
    so it can be captured in a graph.  The tensors must stay alive."""

    def __init__(self, As, Bs, side="L", uplo="L", trans="N", diag="N", alpha: float = 1.0,
                 variant="auto", nb: int = 0, tile: int = 0):
        self._keep = (list(As), list(Bs))
        count, ms, ns, aps, ldas, bps, ldbs = _batch_arrays(As, Bs)
        self.count = count
        opts = Opts(VARIANT[variant], int(nb), 0, 0.0, int(tile))
        h = ctypes.c_void_p()
        dt = _dtype_code(Bs[0]) if count else 0
        _check(lib().redsea_batched_plan_create(dt, SIDE[side], UPLO[uplo], TRANS[trans],
                                                DIAG[diag], count, ms, ns, float(alpha), aps,
                                                ldas, bps, ldbs, ctypes.byref(opts),
                                                ctypes.byref(h)))
        self._h = h

    def run(self, info, stream=None):
        _check(lib().redsea_batched_plan_run(self._h, info.data_ptr() if info is not None else None,
                                             _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().redsea_batched_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trsm_mixed(A, B, side="L", uplo="L", trans="N", diag="N", alpha: float = 1.0, inner: int = 0,
               tol: float = 0.0, max_iter: int = 0, work=None, stream=None) -> MixedStats:
    """FP64 solve by low-precision solves and FP64 iterative refinement."""
    m, n = B.shape
    st = MixedStats()
    wp = work.data_ptr() if work is not None else None
    wb = work.numel() * work.element_size() if work is not None else 0
    rc = lib().redsea_trsm_mixed(SIDE[side], UPLO[uplo], TRANS[trans], DIAG[diag], m, n,
                                 float(alpha), A.data_ptr(), _ld(A), B.data_ptr(), _ld(B),
                                 int(inner), float(tol), int(max_iter), wp, wb,
                                 ctypes.byref(st), _stream(stream))
    _check(rc)
    return st


TRMM_METHOD = {"mfma": 0, "int8": 1, 0: 0, 1: 1}
RESIDUAL_INT8 = 16


def trmm(A, B, C, side="L", uplo="L", trans="N", diag="N", alpha: float = 1.0,
         beta: float = 0.0, method="mfma", stream=None):
    """C := beta C + alpha op(A) B (side L) or beta C + alpha B op(A) (side R),
    A triangular; method "int8" is the exact integer emulation (FP64 only).
    Returns C."""
    m, n = C.shape
    rc = lib().redsea_trmm(_dtype_code(C), SIDE[side], UPLO[uplo], TRANS[trans], DIAG[diag], m, n,
                           float(alpha), A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), float(beta),
                           C.data_ptr(), _ld(C), TRMM_METHOD[method], _stream(stream))
    _check(rc)
    return C


def potrf(A, uplo="L", nb: int = 0, info=None, stream=None):
    """In place Cholesky factorisation of the square column-major device tensor
    A: A = L L^T (uplo "L") or U^T U (uplo "U"), only that triangle read and
    written.  info: a one-element device int32 tensor (allocated when None)
    that receives 0 or the order of the first leading minor found not
    positive definite; it is returned, to be read once the stream is done."""
    import torch
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    elif not info.is_cuda or info.dtype != torch.int32 or info.numel() < 1:
        raise ValueError("info must be a device int32 tensor of at least one element")
    rc = lib().redsea_potrf(_dtype_code(A), UPLO[uplo], n, A.data_ptr(), _ld(A), int(nb),
                            info.data_ptr(), _stream(stream))
    _check(rc)
    return info


def gemm_update(A, X, C, transa=False, transx=False, tile: int = -1, stream=None):
    """In place C := C - op(A) op(X) on the library's MFMA kernels.

    A bfloat16 A selects the BF16 product (X and C float32, X rounded to
    BF16, FP32 accumulation).

    With transx, X and C are passed as their transposes (row-major storage):
    shapes are then X^T (N x K) and C^T (N x M)."""
    if transx:
        N, M = C.shape
    else:
        M, N = C.shape
    K = A.shape[0] if transa else A.shape[1]
    import torch
    code = 2 if A.dtype == torch.bfloat16 else _dtype_code(C)
    rc = lib().redsea_gemm_update(code, int(bool(transa)), int(bool(transx)), M, N, K,
                                  A.data_ptr(), _ld(A), X.data_ptr(), _ld(X), C.data_ptr(), _ld(C),
                                  int(tile), _stream(stream))
    _check(rc)
    return C


def mixed_workspace_bytes(side, m: int, n: int, inner: int) -> int:
    return int(lib().redsea_trsm_mixed_workspace_bytes(SIDE[side], m, n, inner))


def schedule(variant, m: int, nb: int):
    """Task list of the planner as a list of (kind, row0, rows, col0, cols, round)."""
    L = lib()
    cnt = L.redsea_schedule(VARIANT[variant], m, nb, None, 0)
    if cnt < 0:
        raise RedseaError(int(cnt), "invalid argument")
    buf = (ctypes.c_int64 * (6 * max(1, cnt)))()
    L.redsea_schedule(VARIANT[variant], m, nb, ctypes.cast(buf, ctypes.c_void_p), cnt)
    return [tuple(buf[6 * i:6 * i + 6]) for i in range(cnt)]


def version() -> str:
    return lib().redsea_version().decode()


def trace_begin():
    """Start timing every kernel launch of the solver with HIP events."""
    lib().redsea_trace_begin()


def trace_end():
    """Stop tracing; returns {class: (launches, total_ms, total_flops)}."""
    n = len(KERNEL_CLASSES)
    la = (ctypes.c_int64 * n)()
    ms = (ctypes.c_double * n)()
    fl = (ctypes.c_double * n)()
    _check(lib().redsea_trace_end(ctypes.cast(la, ctypes.c_void_p), ctypes.cast(ms, ctypes.c_void_p),
                                  ctypes.cast(fl, ctypes.c_void_p), n))
    return {k: (int(la[i]), float(ms[i]), float(fl[i])) for i, k in enumerate(KERNEL_CLASSES)}


def mfma_peak(dtype: str = "f64", iters: int = 4000, reps: int = 5, stream=None) -> float:
    """Achievable matrix-core rate in TFLOP/s (median of `reps` timed launches
    of the library's MFMA-only probe kernel)."""
    import torch
    code = 0 if dtype == "f64" else 1
    out = torch.empty(4096 * 256, dtype=torch.float64 if code == 0 else torch.float32, device="cuda")
    s = _stream(stream)
    st = torch.cuda.current_stream() if stream is None else stream
    L = lib()
    flops = L.redsea_mfma_peak(code, iters, out.data_ptr(), out.numel(), s)
    if flops <= 0:
        raise RedseaError(int(flops), "mfma peak probe failed")
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        L.redsea_mfma_peak(code, iters, out.data_ptr(), out.numel(), s)
        e1.record(st)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    times.sort()
    return flops / times[len(times) // 2] / 1e12
