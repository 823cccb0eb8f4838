"""redsea: dense triangular solve with many right-hand sides on MI355X.

Thin Python face of the C library libredsea.so (include/redsea.h).  The
functions here only marshal arguments; the solves (and the Cholesky
factorisation built on them) run in the library's HIP kernels for gfx950.
"""
from ._binding import (BatchPlan, EXPORTS, KERNEL_CLASSES, LIB_PATH, trace_begin, trace_end, MixedStats, Opts, RedseaError, fortran_tensor, gemm_update, lib,
                       mfma_peak, mixed_workspace_bytes, schedule, status_string, trsm, trsm_batched,
                       trsm_mixed, trsm_noalloc, trmm, RESIDUAL_INT8, batched_tune, version, potrf)

__all__ = ["BatchPlan", "EXPORTS", "KERNEL_CLASSES", "LIB_PATH", "trace_begin", "trace_end", "MixedStats", "Opts", "RedseaError", "fortran_tensor", "gemm_update", "lib",
           "mfma_peak", "mixed_workspace_bytes", "schedule", "status_string", "trsm", "trsm_batched",
           "trsm_mixed", "trsm_noalloc", "trmm", "RESIDUAL_INT8", "batched_tune", "version", "potrf"]
