"""CPU oracle for the triangular solve op(A) X = alpha B (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The GPU library never does, and it shares no code with it.

The arithmetic lives in ``trsm_oracle.c`` (plain substitution, compensated
Dot2 substitution, compensated residual, operator norms); this module loads
it with ctypes and adds the error metrics computed from a residual:

* normwise backward error per right-hand side (Rigal and Gaches; Higham,
  "Accuracy and Stability of Numerical Algorithms", 2nd ed., Thm 7.1):
  ``eta_j = ||r_j||_inf / (||T||_inf ||x_j||_inf + ||alpha b_j||_inf)`` with T
  the matrix of that right-hand side's system (op(A) for the left side,
  op(A)^T for the right side), reported as the maximum over j;
* componentwise backward error (Oettli and Prager; Higham Thm 7.3):
  ``omega = max_i |r_i| / (|T| |x| + |alpha b|)_i``;
* forward error against a reference solution, per right-hand side, maximum.

The problem itself is the one the paper sets up in Sec. IV (L x = b with
dense lower-triangular L, extended to many right-hand sides), generalised to
BLAS xTRSM flags.

The Cholesky factorisation (the application the paper names next, Sec. VIII)
lives in ``chol_oracle.c``: ``potrf`` is its definition written out column by
column, and ``chol_backward_error`` the componentwise backward error
``max |A - F F^T|_ij / (|F||F|^T)_ij`` over entries of the stored triangle
(Higham Thm 10.3 bounds it by gamma_{n+1}), with the residual by Dot2.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import build as _build

_LIB: Optional[ctypes.CDLL] = None

LEFT, RIGHT = 0, 1
LOWER, UPPER = 0, 1
NOTRANS, TRANS = 0, 1
NONUNIT, UNIT = 0, 1


def _lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        i64, dbl, ptr, cint = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        for name in ("oracle_trsm_plain", "oracle_trsm_comp"):
            f = getattr(lib, name)
            f.restype = cint
            f.argtypes = [cint, cint, cint, cint, i64, i64, dbl, ptr, i64, ptr, i64, cint]
        lib.oracle_residual_comp.restype = cint
        lib.oracle_residual_comp.argtypes = [cint, cint, cint, cint, i64, i64, dbl, ptr, i64,
                                             ptr, i64, ptr, i64, ptr, i64, cint]
        lib.oracle_opnorm.restype = dbl
        lib.oracle_opnorm.argtypes = [cint, cint, cint, i64, ptr, i64, cint]
        lib.oracle_potrf.restype = cint
        lib.oracle_potrf.argtypes = [cint, i64, ptr, i64]
        lib.oracle_chol_residual.restype = None
        lib.oracle_chol_residual.argtypes = [cint, i64, ptr, i64, ptr, i64, i64, ptr, ptr, ptr,
                                             ptr]
        _LIB = lib
    return _LIB


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 64))


def _f64_fortran(x: np.ndarray) -> np.ndarray:
    return np.asfortranarray(np.asarray(x, dtype=np.float64))


def _order(side: int, B: np.ndarray) -> int:
    return B.shape[0] if side == LEFT else B.shape[1]


def _check(side, A, B):
    k = _order(side, B)
    if A.shape[0] < k or A.shape[1] < k:
        raise ValueError("A is %s, needs at least %d x %d" % (A.shape, k, k))


def trsm_plain(side: int, uplo: int, trans: int, diag: int, alpha: float, A: np.ndarray,
               B: np.ndarray, nthreads: Optional[int] = None) -> np.ndarray:
    """Return X with op(A) X = alpha B (left) or X op(A) = alpha B (right).

    Plain FP64 substitution in axpy form.  A is read in its stored triangle
    only; B is not modified.
    """
    A = _f64_fortran(A)
    X = np.array(B, dtype=np.float64, order="F", copy=True)
    _check(side, A, X)
    m, n = X.shape
    rc = _lib().oracle_trsm_plain(side, uplo, trans, diag, m, n, float(alpha),
                                  A.ctypes.data, max(1, A.shape[0]), X.ctypes.data, max(1, m),
                                  nthreads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle_trsm_plain failed")
    return X


def trsm_comp(side: int, uplo: int, trans: int, diag: int, alpha: float, A: np.ndarray,
              B: np.ndarray, nthreads: Optional[int] = None) -> np.ndarray:
    """Compensated (Dot2) substitution; same contract as :func:`trsm_plain`."""
    A = _f64_fortran(A)
    X = np.array(B, dtype=np.float64, order="F", copy=True)
    _check(side, A, X)
    m, n = X.shape
    rc = _lib().oracle_trsm_comp(side, uplo, trans, diag, m, n, float(alpha),
                                 A.ctypes.data, max(1, A.shape[0]), X.ctypes.data, max(1, m),
                                 nthreads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle_trsm_comp failed")
    return X


def residual_comp(side: int, uplo: int, trans: int, diag: int, alpha: float, A: np.ndarray,
                  B: np.ndarray, X: np.ndarray, nthreads: Optional[int] = None) -> np.ndarray:
    """R = alpha B - op(A) X (left) or alpha B - X op(A) (right), each entry
    accurate to about one rounding (Dot2)."""
    A = _f64_fortran(A)
    B = _f64_fortran(B)
    X = _f64_fortran(X)
    _check(side, A, B)
    if X.shape != B.shape:
        raise ValueError("X and B shapes differ")
    m, n = B.shape
    R = np.zeros((m, n), dtype=np.float64, order="F")
    rc = _lib().oracle_residual_comp(side, uplo, trans, diag, m, n, float(alpha),
                                     A.ctypes.data, max(1, A.shape[0]), B.ctypes.data,
                                     max(1, m), X.ctypes.data, max(1, m), R.ctypes.data,
                                     max(1, m), nthreads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle_residual_comp failed")
    return R


def opnorm(uplo: int, trans: int, diag: int, A: np.ndarray, k: int, which: str = "inf") -> float:
    """Infinity norm (``which='inf'``) or one norm (``'one'``) of op(A)
    restricted to its triangle, with a unit diagonal when ``diag`` is UNIT."""
    A = _f64_fortran(A)
    return float(_lib().oracle_opnorm(uplo, trans, diag, k, A.ctypes.data, max(1, A.shape[0]),
                                      0 if which == "inf" else 1))


def backward_error(side: int, uplo: int, trans: int, diag: int, alpha: float, A: np.ndarray,
                   B: np.ndarray, X: np.ndarray, R: Optional[np.ndarray] = None,
                   per_rhs: bool = False):
    """Normwise relative backward error of X as a solution of the system.

    Left side: per column j of X, ``||r_j|| / (||op(A)||_inf ||x_j|| + ||alpha b_j||)``.
    Right side: per row i, the same with ``op(A)^T`` (whose infinity norm is
    the one norm of op(A)).  All vector norms are infinity norms.  Returns the
    maximum, or the per-right-hand-side vector when ``per_rhs``.
    """
    X = np.asarray(X, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if R is None:
        R = residual_comp(side, uplo, trans, diag, alpha, A, B, X)
    k = _order(side, B)
    axis = 0 if side == LEFT else 1
    anorm = opnorm(uplo, trans, diag, A, k, "inf" if side == LEFT else "one")
    rn = np.max(np.abs(R), axis=axis, initial=0.0)
    xn = np.max(np.abs(X), axis=axis, initial=0.0)
    bn = np.max(np.abs(alpha * B), axis=axis, initial=0.0)
    den = anorm * xn + bn
    with np.errstate(invalid="ignore", divide="ignore"):
        eta = np.where(den > 0, rn / np.where(den > 0, den, 1.0), np.where(rn > 0, np.inf, 0.0))
    eta = np.where(np.isfinite(rn) & np.isfinite(xn), eta, np.inf)
    if per_rhs:
        return eta
    return float(np.max(eta, initial=0.0))


def op_dense(uplo: int, trans: int, diag: int, A: np.ndarray, k: int) -> np.ndarray:
    """op(A) as a dense k x k array (triangle only, unit diagonal applied)."""
    A = np.asarray(A, dtype=np.float64)[:k, :k]
    T = np.tril(A) if uplo == LOWER else np.triu(A)
    if diag == UNIT:
        T = T.copy()
        np.fill_diagonal(T, 1.0)
    return T.T.copy() if trans else T


def componentwise_error(side: int, uplo: int, trans: int, diag: int, alpha: float,
                        A: np.ndarray, B: np.ndarray, X: np.ndarray,
                        R: Optional[np.ndarray] = None) -> float:
    """Oettli-Prager componentwise backward error max_i |r_i| / (|T||x| + |alpha b|)_i,
    maximum over all right-hand sides.  The denominators use an FP64
    library product of absolute values (nonnegative terms, relative error
    below k*u, immaterial for a reported metric)."""
    X = np.asarray(X, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if R is None:
        R = residual_comp(side, uplo, trans, diag, alpha, A, B, X)
    k = _order(side, B)
    T = np.abs(op_dense(uplo, trans, diag, A, k))
    den = (T @ np.abs(X) if side == LEFT else np.abs(X) @ T) + np.abs(alpha * B)
    num = np.abs(R)
    with np.errstate(invalid="ignore", divide="ignore"):
        w = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return float(np.max(w, initial=0.0))


def forward_error(X: np.ndarray, Xref: np.ndarray, side: int = LEFT) -> float:
    """max over right-hand sides of ||x - x_ref||_inf / ||x_ref||_inf."""
    X = np.asarray(X, dtype=np.float64)
    Xref = np.asarray(Xref, dtype=np.float64)
    axis = 0 if side == LEFT else 1
    num = np.max(np.abs(X - Xref), axis=axis, initial=0.0)
    den = np.max(np.abs(Xref), axis=axis, initial=0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        e = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return float(np.max(e, initial=0.0))


def potrf(uplo: int, A: np.ndarray):
    """Cholesky factor of the symmetric positive definite A (lower: A = L L^T,
    upper: A = U^T U), in a copy of A; returns (F, info) with info 0 or the
    order of the first leading minor found not positive definite.  Only the
    uplo triangle of A is read; the other strict triangle of F is A's."""
    F = _f64_fortran(A).copy(order="F")
    n = F.shape[0]
    if F.shape[1] != n:
        raise ValueError("A must be square")
    info = _lib().oracle_potrf(uplo, n, F.ctypes.data, max(1, n))
    return F, int(info)


def chol_residual(uplo: int, A: np.ndarray, F: np.ndarray, pairs: np.ndarray):
    """(r, d) at the entries (i, j), i >= j, of the factor's lower storage
    (for uplo 1 the entry (j, i) of U): r = A - F F^T by Dot2, d = |F||F|^T."""
    A = _f64_fortran(A)
    F = _f64_fortran(F)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    if np.any(pairs[:, 0] < pairs[:, 1]):
        raise ValueError("pairs must have i >= j")
    pi = np.ascontiguousarray(pairs[:, 0])
    pj = np.ascontiguousarray(pairs[:, 1])
    r = np.zeros(len(pairs))
    d = np.zeros(len(pairs))
    _lib().oracle_chol_residual(uplo, A.shape[0], A.ctypes.data, max(1, A.shape[0]),
                                F.ctypes.data, max(1, F.shape[0]), len(pairs), pi.ctypes.data,
                                pj.ctypes.data, r.ctypes.data, d.ctypes.data)
    return r, d


def lower_pairs(n: int) -> np.ndarray:
    """Every (i, j) with n > i >= j >= 0."""
    i, j = np.tril_indices(n)
    return np.stack([i, j], axis=1)


def chol_backward_error(uplo: int, A: np.ndarray, F: np.ndarray, pairs=None) -> float:
    """max |A - F F^T|_ij / (|F||F|^T)_ij over the given entries of the stored
    triangle (all of them when pairs is None); an entry with a zero
    denominator counts 0 if its residual is 0, else infinity."""
    if pairs is None:
        pairs = lower_pairs(np.asarray(A).shape[0])
    r, d = chol_residual(uplo, A, F, pairs)
    num = np.abs(r)
    with np.errstate(invalid="ignore", divide="ignore"):
        w = np.where(d > 0, num / np.where(d > 0, d, 1.0), np.where(num > 0, np.inf, 0.0))
    return float(np.max(w, initial=0.0))
