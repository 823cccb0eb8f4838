"""Pins for the CPU oracle: values fixed by mathematics, not by the oracle.

* identity and diagonal systems have closed-form, bitwise-known answers;
* integer systems (B = op(A) X_true in int64) have exact answers that every
  correct substitution returns bitwise;
* exhaustive and random tiny systems are checked against exact rational
  arithmetic: the componentwise backward error must obey the rigorous bound
  gamma_k of triangular substitution (Higham, Thm 8.5);
* the compensated residual must be within the Dot2 error bound of the exact
  residual (Ogita, Rump, Oishi 2005, Prop. 5.5 form);
* a test plants mistakes in a copy of the oracle source and checks that the
  pins catch every one of them.
"""
import ctypes
import itertools
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import rational
import synth

U = 2.0 ** -53
FLAGS = list(itertools.product([0, 1], [0, 1], [0, 1], [0, 1]))  # side, uplo, trans, diag


def _shape(side, k, nrhs):
    return (k, nrhs) if side == 0 else (nrhs, k)


# ---------------------------------------------------------------- identity
@pytest.mark.parametrize("side,uplo,trans,diag", FLAGS)
@pytest.mark.parametrize("alpha", [1.0, -0.5, 3.0 / 7.0])
def test_identity_is_alpha_b(side, uplo, trans, diag, alpha):
    k, nrhs = 23, 7
    A = np.full((k, k), np.nan, order="F")
    stored = np.tril(np.ones((k, k), bool), -1) if uplo == 0 else np.triu(np.ones((k, k), bool), 1)
    A[stored] = 0.0
    A[np.diag_indices(k)] = np.nan if diag else 1.0
    B = synth.rhs_normal(*_shape(side, k, nrhs), key=(90, 0, 1))
    for fn in (oracle.trsm_plain, oracle.trsm_comp):
        X = fn(side, uplo, trans, diag, alpha, A, B)
        expect = B if alpha == 1.0 else alpha * B
        assert np.array_equal(X, expect), fn.__name__


def test_alpha_zero_gives_zero_without_reading_a():
    A = np.full((5, 5), np.nan, order="F")
    B = synth.rhs_normal(5, 3, (91, 0, 1))
    assert np.array_equal(oracle.trsm_plain(0, 0, 0, 0, 0.0, A, B), np.zeros((5, 3)))


# ---------------------------------------------------------------- diagonal
@pytest.mark.parametrize("side,uplo,trans", list(itertools.product([0, 1], [0, 1], [0, 1])))
@pytest.mark.parametrize("alpha", [1.0, -1.25])
def test_diagonal_is_one_division(side, uplo, trans, alpha):
    k, nrhs = 31, 9
    A = synth.diagonal(k, (92, 0, 0))
    d = np.diag(A).copy()
    B = synth.rhs_normal(*_shape(side, k, nrhs), key=(92, 0, 1))
    ab = B if alpha == 1.0 else alpha * B
    expect = ab / d[:, None] if side == 0 else ab / d[None, :]
    for fn in (oracle.trsm_plain, oracle.trsm_comp):
        X = fn(side, uplo, trans, 0, alpha, A, B)
        assert np.array_equal(X, expect), fn.__name__
    # a reciprocal multiply is not bitwise equal for these data
    recip = ab * (1.0 / d)[:, None] if side == 0 else ab * (1.0 / d)[None, :]
    assert not np.array_equal(recip, expect)


# ---------------------------------------------------------------- integer-exact
@pytest.mark.parametrize("side,uplo,trans,diag", FLAGS)
@pytest.mark.parametrize("k,nrhs", [(1, 1), (7, 3), (64, 5), (129, 17)])
def test_integer_exact(side, uplo, trans, diag, k, nrhs):
    m, n = _shape(side, k, nrhs)
    A, B, X = synth.integer_exact(m, n, (93, k, nrhs), side, uplo, trans, diag)
    for fn in (oracle.trsm_plain, oracle.trsm_comp):
        got = fn(side, uplo, trans, diag, 1.0, A, B)
        assert np.array_equal(got, X), fn.__name__
    R = oracle.residual_comp(side, uplo, trans, diag, 1.0, A, B, X)
    assert np.array_equal(R, np.zeros_like(R))
    assert oracle.backward_error(side, uplo, trans, diag, 1.0, A, B, X) == 0.0


def test_right_side_is_transposed_left_side():
    k, nrhs = 40, 11
    A = synth.dominant_lower(k, (94, 0, 0))
    B = synth.rhs_normal(nrhs, k, (94, 0, 1))
    for trans in (0, 1):
        xr = oracle.trsm_plain(1, 0, trans, 0, 0.75, A, B)
        xl = oracle.trsm_plain(0, 0, 1 - trans, 0, 0.75, A, np.asfortranarray(B.T))
        assert np.array_equal(xr, xl.T)


def test_thread_count_does_not_change_bits():
    k, nrhs = 150, 37
    A = synth.dominant_lower(k, (95, 0, 0))
    B = synth.rhs_normal(k, nrhs, (95, 0, 1))
    for fn in (oracle.trsm_plain, oracle.trsm_comp):
        x1 = fn(0, 0, 0, 0, 1.0, A, B, nthreads=1)
        x7 = fn(0, 0, 0, 0, 1.0, A, B, nthreads=7)
        assert np.array_equal(x1, x7)
    r1 = oracle.residual_comp(0, 0, 0, 0, 1.0, A, B, x1, nthreads=1)
    r5 = oracle.residual_comp(0, 0, 0, 0, 1.0, A, B, x1, nthreads=5)
    assert np.array_equal(r1, r5)


# ---------------------------------------------------------------- brute force
def _values(k, key):
    r = synth.rng(key)
    return r.standard_normal(k) * 10.0 ** r.integers(-3, 4, size=k)


def test_exhaustive_2x2_all_flags():
    gam = rational.gamma(2)
    offs = [-2.0, -1.0, 0.0, 1.0, 2.0]
    diags = [-2.0, -1.0, 1.0, 2.0, 3.0]
    worst = Fraction(0)
    for side, uplo, trans, diag in FLAGS:
        for a10, d0, d1 in itertools.product(offs, diags, diags):
            A = np.full((2, 2), np.nan, order="F")
            if uplo == 0:
                A[1, 0] = a10
            else:
                A[0, 1] = a10
            A[0, 0], A[1, 1] = (np.nan, np.nan) if diag else (d0, d1)
            B = np.asfortranarray(np.array([[0.1, -1.0 / 3.0], [2.0 / 7.0, 1e-3]]))
            X = oracle.trsm_plain(side, uplo, trans, diag, 1.0, A, B, nthreads=1)
            w = rational.componentwise_exact(side, uplo, trans, diag, 1.0, A, B, X)
            worst = max(worst, w)
            assert w <= gam, (side, uplo, trans, diag, a10, d0, d1)
    assert worst > 0  # the cases do exercise rounding


def test_exhaustive_3x3_lower():
    gam = rational.gamma(3)
    offs = [-2.0, -1.0, 0.0, 1.0, 2.0]
    diags = [-2.0, -1.0, 1.0, 2.0, 3.0, -3.0]
    B = np.asfortranarray(np.array([[0.1], [-1.0 / 3.0], [2.0 / 7.0]]))
    Af = np.zeros((3, 3), order="F")
    count = 0
    for a10, a20, a21 in itertools.product(offs, offs, offs):
        for d in itertools.product(diags, repeat=3):
            Af[1, 0], Af[2, 0], Af[2, 1] = a10, a20, a21
            Af[0, 0], Af[1, 1], Af[2, 2] = d
            X = oracle.trsm_plain(0, 0, 0, 0, 1.0, Af, B, nthreads=1)
            w = rational.componentwise_exact(0, 0, 0, 0, 1.0, Af, B, X)
            assert w <= gam, (a10, a20, a21, d)
            count += 1
    assert count == 125 * 216


@pytest.mark.parametrize("k", [4, 5, 6, 7, 8])
def test_random_tiny_against_rationals(k):
    gam = rational.gamma(k)
    for trial in range(6):
        side, uplo, trans, diag = FLAGS[(trial * 5 + k) % 16]
        r = synth.rng((96, k, trial))
        A = np.asfortranarray(r.uniform(-1, 1, (k, k)) * 10.0 ** r.integers(-2, 3, (k, k)))
        A[np.diag_indices(k)] = r.uniform(0.5, 2.0, k) * r.choice([-1, 1], k)
        nrhs = 3
        B = np.asfortranarray(_values(k * nrhs, (96, k, trial + 100)).reshape(_shape(side, k, nrhs)))
        alpha = [1.0, -0.3][trial % 2]
        X = oracle.trsm_plain(side, uplo, trans, diag, alpha, A, B, nthreads=1)
        w = rational.componentwise_exact(side, uplo, trans, diag, alpha, A, B, X)
        # alpha*B is rounded once before the solve: that is a relative
        # perturbation of u in b, within gamma_k as well.
        assert w <= gam, (k, trial, float(w))


# ---------------------------------------------------------------- compensated
@pytest.mark.parametrize("k", [3, 5, 8, 12, 20])
def test_compensated_close_to_exact(k):
    """On well-conditioned tiny systems the compensated solution is within
    3u ||x||_inf of the exact one, per right-hand side (an empirical pin:
    the largest value seen over these seeds is about 1.6u)."""
    for trial in range(8):
        A = synth.dominant_lower(k, (97, k, trial))
        B = synth.rhs_normal(k, 2, (97, k, trial + 50))
        X = oracle.trsm_comp(0, 0, 0, 0, 1.0, A, B, nthreads=1)
        Xe = rational.trsm_exact(0, 0, 0, 0, 1.0, A, B)
        for j in range(2):
            xn = max(abs(Xe[i][j]) for i in range(k))
            err = max(abs(Fraction(float(X[i, j])) - Xe[i][j]) for i in range(k))
            assert err <= 3 * Fraction(U) * xn, (k, trial, j)


def test_compensated_residual_within_dot2_bound():
    for k in (4, 9, 16):
        for trial in range(4):
            side, uplo, trans, diag = FLAGS[(trial * 3 + k) % 16]
            A = np.asfortranarray(synth.rng((98, k, trial)).uniform(-1, 1, (k, k)))
            A[np.diag_indices(k)] += 2.0
            B = synth.rhs_normal(*_shape(side, k, 3), key=(98, k, trial + 9))
            X = oracle.trsm_plain(side, uplo, trans, diag, 0.7, A, B)
            X = X * (1 + 1e-9 * synth.rng((98, 1, trial)).standard_normal(X.shape))
            R = oracle.residual_comp(side, uplo, trans, diag, 0.7, A, B, X)
            Re = rational.residual_exact(side, uplo, trans, diag, 0.7, A, B, X)
            T = rational.op_matrix(uplo, trans, diag, A, k)
            g2 = rational.gamma(k + 1) ** 2
            m, n = B.shape
            for i in range(m):
                for j in range(n):
                    terms = abs(Fraction(0.7) * Fraction(float(B[i, j])))
                    if side == 0:
                        terms += sum(abs(T[i][p] * Fraction(float(X[p, j]))) for p in range(k))
                    else:
                        terms += sum(abs(Fraction(float(X[i, p])) * T[p][j]) for p in range(k))
                    err = abs(Fraction(float(R[i, j])) - Re[i][j])
                    assert err <= Fraction(U) * abs(Re[i][j]) + g2 * terms


# ---------------------------------------------------------------- metrics
def test_backward_error_closed_form():
    """T = I and x = b + delta e_1: r = -delta e_1, so
    eta = |delta| / (||x||_inf + ||b||_inf)."""
    k = 6
    A = np.asfortranarray(np.eye(k))
    b = np.array([[0.5], [-2.0], [1.0], [0.25], [0.0], [1.5]])
    delta = 0.125
    x = b.copy()
    x[0, 0] += delta
    eta = oracle.backward_error(0, 0, 0, 0, 1.0, A, b, x)
    assert eta == delta / (2.0 + 2.0)
    omega = oracle.componentwise_error(0, 0, 0, 0, 1.0, A, b, x)
    assert omega == delta / (0.625 + 0.5)


def test_opnorm_matches_library_norm():
    A = synth.dominant_lower(33, (99, 0, 0), upper_fill=np.nan)
    for uplo, trans, diag in itertools.product([0], [0, 1], [0, 1]):
        T = oracle.op_dense(uplo, trans, diag, np.nan_to_num(A, nan=0.0), 33)
        assert oracle.opnorm(uplo, trans, diag, A, 33, "inf") == pytest.approx(
            np.linalg.norm(T, np.inf), rel=1e-15)
        assert oracle.opnorm(uplo, trans, diag, A, 33, "one") == pytest.approx(
            np.linalg.norm(T, 1), rel=1e-15)


def test_plain_oracle_backward_stable_on_dominant():
    for n in (200, 513):
        A = synth.dominant_lower(n, (100, n, 0))
        B = synth.rhs_normal(n, 16, (100, n, 1))
        X = oracle.trsm_plain(0, 0, 0, 0, 1.0, A, B)
        assert oracle.backward_error(0, 0, 0, 0, 1.0, A, B, X) <= n * U
        Xc = oracle.trsm_comp(0, 0, 0, 0, 1.0, A, B)
        assert oracle.forward_error(X, Xc) <= 1e-12


# ---------------------------------------------------------------- planted mistakes
MUTANTS = [
    ("sign of the update", "y[i * inc] = y[i * inc] - prod;", "y[i * inc] = y[i * inc] + prod;"),
    ("dropped term", "for (int64_t i = k + 1; i < m; ++i) {", "for (int64_t i = k + 2; i < m; ++i) {"),
    ("transposed operand", "int64_t r = M->trans ? j : i;", "int64_t r = M->trans ? i : j;"),
    ("reciprocal multiply", "if (!T->M.unit) xk = xk / t_at(T, k, k);",
     "if (!T->M.unit) xk = xk * (1.0 / t_at(T, k, k));"),
    ("dot2 error term dropped", "d->s = d->s + (q + r);", "d->s = d->s + q;"),
    ("unit diagonal read", "if (r == c) return M->unit ? 1.0 : M->a[r + c * M->lda];",
     "if (r == c) return M->a[r + c * M->lda];"),
]


def _pins_pass(lib_path):
    """Re-run a compact version of the pins against the library at lib_path;
    return False as soon as one fails."""
    lib = ctypes.CDLL(lib_path)
    i64, dbl, ptr, cint = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
    for name in ("oracle_trsm_plain", "oracle_trsm_comp"):
        getattr(lib, name).argtypes = [cint, cint, cint, cint, i64, i64, dbl, ptr, i64, ptr, i64, cint]
    lib.oracle_residual_comp.argtypes = [cint, cint, cint, cint, i64, i64, dbl, ptr, i64,
                                         ptr, i64, ptr, i64, ptr, i64, cint]

    def solve(name, side, uplo, trans, diag, alpha, A, B):
        X = np.array(B, dtype=np.float64, order="F", copy=True)
        A = np.asfortranarray(A, dtype=np.float64)
        getattr(lib, name)(side, uplo, trans, diag, X.shape[0], X.shape[1], alpha,
                           A.ctypes.data, A.shape[0], X.ctypes.data, X.shape[0], 2)
        return X

    # diagonal, bitwise
    A = synth.diagonal(9, (92, 0, 0))
    B = synth.rhs_normal(9, 4, (92, 0, 1))
    if not np.array_equal(solve("oracle_trsm_plain", 0, 0, 0, 0, 1.0, A, B), B / np.diag(A)[:, None]):
        return False
    # integer-exact, all flags, both solvers
    for side, uplo, trans, diag in FLAGS:
        m, n = _shape(side, 12, 5)
        A, B, X = synth.integer_exact(m, n, (93, 1, 2), side, uplo, trans, diag)
        for name in ("oracle_trsm_plain", "oracle_trsm_comp"):
            if not np.array_equal(solve(name, side, uplo, trans, diag, 1.0, A, B), X):
                return False
        R = np.zeros_like(B, order="F")
        lib.oracle_residual_comp(side, uplo, trans, diag, m, n, 1.0, A.ctypes.data, A.shape[0],
                                 B.ctypes.data, m, X.ctypes.data, m, R.ctypes.data, m, 1)
        if not np.array_equal(R, np.zeros_like(R)):
            return False
    # compensated residual against the exact residual
    k = 6
    A = np.asfortranarray(synth.rng((98, 0, 0)).uniform(-1, 1, (k, k)))
    A[np.diag_indices(k)] += 2.0
    B = synth.rhs_normal(k, 2, (98, 0, 1))
    X = solve("oracle_trsm_plain", 0, 0, 0, 0, 1.0, A, B)
    X = X * (1 + 1e-9 * synth.rng((98, 0, 2)).standard_normal(X.shape))
    X = np.asfortranarray(X)
    R = np.zeros_like(X, order="F")
    lib.oracle_residual_comp(0, 0, 0, 0, k, 2, 1.0, A.ctypes.data, k, B.ctypes.data, k,
                             X.ctypes.data, k, R.ctypes.data, k, 1)
    Re = rational.residual_exact(0, 0, 0, 0, 1.0, A, B, X)
    for i in range(k):
        for j in range(2):
            if abs(Fraction(float(R[i, j])) - Re[i][j]) > Fraction(U) * abs(Re[i][j]) * 2:
                return False
    return True


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_planted_mistakes_are_caught(tmp_path):
    from oracle import build
    src = open(build.SRC).read()
    # the pristine source passes the compact pins
    good = tmp_path / "good.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                    build.SRC, "-o", str(good), "-lm"], check=True)
    assert _pins_pass(str(good))
    for label, old, new in MUTANTS:
        assert src.count(old) >= 1, label
        mutated = src.replace(old, new)
        c = tmp_path / ("m%d.c" % MUTANTS.index((label, old, new)))
        c.write_text(mutated)
        so = str(c) + ".so"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                        str(c), "-o", so, "-lm"], check=True)
        assert not _pins_pass(so), "pins missed planted mistake: " + label
