"""Exact rational reference for tiny triangular systems (TEST INFRASTRUCTURE).

Every FP64 number is a rational, so ``fractions.Fraction`` gives the exact
solution of op(A) x = alpha b (the system of Sec. IV of the paper, under BLAS
flags) and the exact residual of any computed x.  Pure Python loops, only for
orders up to about a dozen.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence

import numpy as np

LEFT, RIGHT = 0, 1
LOWER, UPPER = 0, 1


def op_matrix(uplo: int, trans: int, diag: int, A: np.ndarray, k: int) -> List[List[Fraction]]:
    """op(A) as exact rationals: the stored triangle, one on the diagonal when
    unit, zero elsewhere; transposed when ``trans``."""
    T = [[Fraction(0)] * k for _ in range(k)]
    for r in range(k):
        for c in range(k):
            if r == c:
                v = Fraction(1) if diag else Fraction(float(A[r, c]))
            elif (uplo == LOWER and r > c) or (uplo == UPPER and r < c):
                v = Fraction(float(A[r, c]))
            else:
                v = Fraction(0)
            if trans:
                T[c][r] = v
            else:
                T[r][c] = v
    return T


def solve_exact(T: List[List[Fraction]], c: Sequence[Fraction]) -> List[Fraction]:
    """Exact solution of T y = c for triangular T (either triangle)."""
    k = len(c)
    lower = all(T[i][j] == 0 for i in range(k) for j in range(i + 1, k))
    y = [Fraction(0)] * k
    order = range(k) if lower else range(k - 1, -1, -1)
    for i in order:
        s = Fraction(c[i])
        for j in range(k):
            if j != i and T[i][j] != 0:
                s -= T[i][j] * y[j]
        y[i] = s / T[i][i]
    return y


def trsm_exact(side: int, uplo: int, trans: int, diag: int, alpha: float, A: np.ndarray,
               B: np.ndarray) -> List[List[Fraction]]:
    """Exact X (list of rows) with op(A) X = alpha B or X op(A) = alpha B."""
    m, n = B.shape
    k = m if side == LEFT else n
    T = op_matrix(uplo, trans, diag, A, k)
    a = Fraction(float(alpha))
    X = [[Fraction(0)] * n for _ in range(m)]
    if side == LEFT:
        for j in range(n):
            y = solve_exact(T, [a * Fraction(float(B[i, j])) for i in range(m)])
            for i in range(m):
                X[i][j] = y[i]
    else:
        TT = [[T[j][i] for j in range(k)] for i in range(k)]
        for i in range(m):
            y = solve_exact(TT, [a * Fraction(float(B[i, j])) for j in range(n)])
            for j in range(n):
                X[i][j] = y[j]
    return X


def residual_exact(side: int, uplo: int, trans: int, diag: int, alpha: float, A: np.ndarray,
                   B: np.ndarray, X: np.ndarray) -> List[List[Fraction]]:
    """Exact R = alpha B - op(A) X (left) or alpha B - X op(A) (right) for a
    floating-point X."""
    m, n = B.shape
    k = m if side == LEFT else n
    T = op_matrix(uplo, trans, diag, A, k)
    a = Fraction(float(alpha))
    Xf = [[Fraction(float(X[i, j])) for j in range(n)] for i in range(m)]
    R = [[Fraction(0)] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            s = a * Fraction(float(B[i, j]))
            if side == LEFT:
                for p in range(k):
                    s -= T[i][p] * Xf[p][j]
            else:
                for p in range(k):
                    s -= Xf[i][p] * T[p][j]
            R[i][j] = s
    return R


def componentwise_exact(side: int, uplo: int, trans: int, diag: int, alpha: float,
                        A: np.ndarray, B: np.ndarray, X: np.ndarray) -> Fraction:
    """Exact Oettli-Prager componentwise backward error of X:
    max_ij |r_ij| / (|T||X| + |alpha B|)_ij (0/0 counts as 0)."""
    m, n = B.shape
    k = m if side == LEFT else n
    T = op_matrix(uplo, trans, diag, A, k)
    R = residual_exact(side, uplo, trans, diag, alpha, A, B, X)
    a = Fraction(float(alpha))
    Xf = [[Fraction(float(X[i, j])) for j in range(n)] for i in range(m)]
    worst = Fraction(0)
    for i in range(m):
        for j in range(n):
            d = abs(a * Fraction(float(B[i, j])))
            if side == LEFT:
                d += sum(abs(T[i][p]) * abs(Xf[p][j]) for p in range(k))
            else:
                d += sum(abs(Xf[i][p]) * abs(T[p][j]) for p in range(k))
            r = abs(R[i][j])
            if d == 0:
                if r != 0:
                    return Fraction(10**30)
                continue
            worst = max(worst, r / d)
    return worst


def gamma(k: int, u: float = 2.0 ** -53) -> Fraction:
    """gamma_k = k u / (1 - k u) (Higham, Sec. 3.1), exactly."""
    uf = Fraction(u)
    return k * uf / (1 - k * uf)
