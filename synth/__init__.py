"""Seeded synthetic inputs for the triangular solve (shared by tests and bench).

This module only draws and arranges numbers: it performs no part of the
solve.  Both the GPU path and the CPU oracle read the arrays it returns, so
any summation order used while building an input is irrelevant to parity.

Every generator takes a key ``(config, system, stream)`` fed to numpy's
PCG64 (``np.random.default_rng(list(key))``); stream 0 draws the matrix and
stream 1 the right-hand sides.  Arrays come back in Fortran (column-major)
order with leading dimension equal to the row count.

The paper (Sec. IV, VI) states no matrix distribution or size, so the
workload recipe is this project's own:

* ``dominant_lower``: strict lower part i.i.d. U(-1, 1); diagonal
  ``1 + sum_{j<i} |L_ij|`` (row diagonally dominant, well conditioned).
* ``rhs_normal``: i.i.d. N(0, 1).
* ``unit_lower``: rows of the dominant matrix divided by their diagonal,
  diagonal stored as NaN (a unit-diagonal solve must never read it).
* ``kappa_lower``: the same strict lower part with the constant diagonal
  ``c * (1 + max_k sum_{j<k} |L_kj|)``; smaller c gives larger condition
  numbers (the constant c for a target condition number is found with the
  oracle and stored under tests/golden).
* ``integer_exact``: small-integer L and X_true with B = op(L) X_true formed
  exactly in int64, so every partial sum of a substitution is an integer
  far below 2**24 and any correct solver returns X_true exactly.
* ``batch_shapes``: log-uniform orders and right-hand-side counts.
* ``spd_dominant`` (Cholesky inputs): symmetric, off-diagonal U(-1, 1),
  diagonal ``1 + sum_{j != i} |A_ij|`` (strictly diagonally dominant with a
  positive diagonal, so positive definite and well conditioned).
* ``integer_spd``: ``A = L0 L0^T`` formed in int64 from a small-integer lower
  L0 with diagonal in {1, 2}, so every partial sum of a Cholesky
  factorisation is an integer and any correct one returns L0 exactly.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np

Key = Sequence[int]


def rng(key: Key) -> np.random.Generator:
    return np.random.default_rng([int(k) for k in key])


def _strict_lower_uniform(n: int, key: Key) -> np.ndarray:
    draw = rng(key).uniform(-1.0, 1.0, size=(n, n))  # C order: L[i, j] = draw[i*n + j]
    return np.tril(draw, -1)


def dominant_lower(n: int, key: Key, upper_fill: float = 0.0) -> np.ndarray:
    """Lower-triangular n x n, off-diagonal U(-1,1), L_ii = 1 + sum_{j<i}|L_ij|."""
    L = _strict_lower_uniform(n, key)
    d = 1.0 + np.abs(L).sum(axis=1)
    L[np.diag_indices(n)] = d
    if upper_fill != 0.0:
        L[np.triu_indices(n, 1)] = upper_fill
    return np.asfortranarray(L)


def rhs_normal(m: int, nrhs: int, key: Key) -> np.ndarray:
    """m x nrhs, i.i.d. standard normal."""
    return np.asfortranarray(rng(key).standard_normal(size=(m, nrhs)))


def unit_lower(n: int, key: Key) -> np.ndarray:
    """Dominant lower matrix with each row divided by its diagonal; the
    diagonal itself is stored as NaN and the strict upper part as NaN."""
    L = np.array(dominant_lower(n, key), order="C")
    d = np.diag(L).copy()
    L = L / d[:, None]
    L = np.tril(L, -1)
    L[np.diag_indices(n)] = np.nan
    L[np.triu_indices(n, 1)] = np.nan
    return np.asfortranarray(L)


def upper_of(L: np.ndarray) -> np.ndarray:
    """U = L^T stored column-major, so op(U) = U^T equals L."""
    return np.asfortranarray(np.array(L).T)


def kappa_lower(n: int, c: float, key: Key) -> np.ndarray:
    """Strict lower part as in dominant_lower, constant diagonal
    c * (1 + max_k sum_{j<k} |L_kj|)."""
    L = _strict_lower_uniform(n, key)
    rows = np.abs(L).sum(axis=1)
    d = c * (1.0 + float(rows.max(initial=0.0)))
    L[np.diag_indices(n)] = d
    return np.asfortranarray(L)


def diagonal(n: int, key: Key) -> np.ndarray:
    """Diagonal matrix with entries of both signs and magnitudes in [0.5, 8)."""
    r = rng(key)
    d = r.uniform(0.5, 8.0, size=n) * r.choice([-1.0, 1.0], size=n)
    return np.asfortranarray(np.diag(d))


def integer_exact(m: int, nrhs: int, key: Key, side: int = 0, uplo: int = 0, trans: int = 0,
                  diag: int = 0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(A, B, X_true) with op(A) X_true = B (left) or X_true op(A) = B (right),
    all entries small integers.

    A's stored triangle holds integers in [-3, 3] off the diagonal and
    {+-1, +-2, +-4} on it (NaN when ``diag`` is unit); the other triangle is
    NaN.  X_true is in [-4, 4].  B is formed in int64, so it is exact.
    """
    r = rng(key)
    k = m if side == 0 else nrhs
    off = r.integers(-3, 4, size=(k, k)).astype(np.int64)
    dvals = r.choice(np.array([-4, -2, -1, 1, 2, 4], dtype=np.int64), size=k)
    Lint = np.tril(off, -1)
    Lint[np.diag_indices(k)] = 1 if diag else dvals
    Aint = Lint if uplo == 0 else Lint.T  # stored triangle of A
    # op(A) as an integer matrix
    op = Aint.T if trans else Aint
    X = r.integers(-4, 5, size=(m, nrhs)).astype(np.int64)
    B = op @ X if side == 0 else X @ op
    A = Aint.astype(np.float64)
    mask_other = np.triu(np.ones((k, k), bool), 1) if uplo == 0 else np.tril(np.ones((k, k), bool), -1)
    A[mask_other] = np.nan
    if diag:
        A[np.diag_indices(k)] = np.nan
    return np.asfortranarray(A), np.asfortranarray(B.astype(np.float64)), \
        np.asfortranarray(X.astype(np.float64))


def spd_dominant(n: int, key: Key) -> np.ndarray:
    """Symmetric positive definite n x n: off-diagonal U(-1, 1) mirrored,
    diagonal 1 + sum of the row's off-diagonal magnitudes."""
    S = _strict_lower_uniform(n, key)
    A = S + S.T
    A[np.diag_indices(n)] = 1.0 + np.abs(A).sum(axis=1)
    return np.asfortranarray(A)


def integer_spd(n: int, key: Key) -> Tuple[np.ndarray, np.ndarray]:
    """(A, L0): L0 lower with integers in [-2, 2] below the diagonal and
    {1, 2} on it, A = L0 L0^T (full symmetric) formed exactly in int64."""
    r = rng(key)
    L0 = np.tril(r.integers(-2, 3, size=(n, n)).astype(np.int64), -1)
    L0[np.diag_indices(n)] = r.choice(np.array([1, 2], dtype=np.int64), size=n)
    A = L0 @ L0.T
    return np.asfortranarray(A.astype(np.float64)), np.asfortranarray(L0.astype(np.float64))


def batch_shapes(count: int, key: Key, n_range=(32, 1024), nrhs_range=(1, 256)):
    """Orders n = round(exp(U[ln lo, ln hi])) and right-hand-side counts
    likewise; returns two int64 arrays."""
    r = rng(key)
    n = np.rint(np.exp(r.uniform(np.log(n_range[0]), np.log(n_range[1]), size=count)))
    k = np.rint(np.exp(r.uniform(np.log(nrhs_range[0]), np.log(nrhs_range[1]), size=count)))
    return n.astype(np.int64), k.astype(np.int64)
