"""Condition numbers of lower-triangular matrices (TEST INFRASTRUCTURE).

kappa_1(L) = ||L||_1 ||L^{-1}||_1.  Exact for small orders (the inverse is
computed column by column with the oracle's substitution); estimated for
large orders with Hager's method as refined by Higham (N. J. Higham, "FORTRAN
codes for estimating the one-norm of a real or complex matrix", ACM TOMS
14(4), 1988; "Accuracy and Stability of Numerical Algorithms", 2nd ed.,
Sec. 15.3), written here from that description: it needs only solves with L
and L^T, which the oracle provides.
"""
from __future__ import annotations

import numpy as np

from . import trsm_plain


def norm1_lower(L: np.ndarray) -> float:
    """One norm (max column sum) of the lower triangle of L."""
    return float(np.abs(np.tril(L)).sum(axis=0).max(initial=0.0))


def inv_norm1_exact(L: np.ndarray) -> float:
    n = L.shape[0]
    inv = trsm_plain(0, 0, 0, 0, 1.0, L, np.asfortranarray(np.eye(n)))
    return float(np.abs(inv).sum(axis=0).max(initial=0.0))


def kappa1_exact(L: np.ndarray) -> float:
    return norm1_lower(L) * inv_norm1_exact(L)


def inv_norm1_estimate(L: np.ndarray, maxiter: int = 5) -> float:
    """Lower bound on ||L^{-1}||_1 (usually equal to it)."""
    n = L.shape[0]

    def solve(v, trans):
        return trsm_plain(0, 0, trans, 0, 1.0, L, np.asfortranarray(v.reshape(n, 1)))[:, 0]

    x = np.full(n, 1.0 / n)
    est = 0.0
    for it in range(maxiter):
        y = solve(x, 0)
        new = float(np.abs(y).sum())
        if it > 0 and new <= est:
            break
        est = new
        xi = np.where(y >= 0, 1.0, -1.0)
        z = solve(xi, 1)
        j = int(np.argmax(np.abs(z)))
        if it > 0 and abs(z[j]) <= float(z @ x):
            break
        x = np.zeros(n)
        x[j] = 1.0
    # alternating-sign safeguard vector
    b = np.array([(-1.0) ** i * (1.0 + i / max(n - 1, 1)) for i in range(n)])
    est2 = 2.0 * float(np.abs(solve(b, 0)).sum()) / (3.0 * n)
    return max(est, est2)


def kappa1_estimate(L: np.ndarray) -> float:
    return norm1_lower(L) * inv_norm1_estimate(L)
