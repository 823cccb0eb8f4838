"""Pins for the Cholesky oracle: values fixed by mathematics, not by the oracle.

* integer factors: A = L0 L0^T formed exactly, so every correct factorisation
  returns L0 bitwise (both storage triangles);
* a 2 x 2 closed form with exact square roots;
* agreement with numpy's Cholesky (LAPACK) on random positive definite
  matrices, and the componentwise backward-error bound gamma_{n+1} of
  Higham, Thm 10.3;
* the Dot2 residual against exactly known residuals of a perturbed integer
  factor;
* info: the order of the first leading minor that is not positive definite;
* the other strict triangle is neither read nor written;
* scaling by powers of two commutes with the factorisation bitwise;
* a test plants mistakes in a copy of the oracle source and checks that the
  pins catch every one of them.
"""
import ctypes
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

U = 2.0 ** -53


def _tri(F, uplo):
    return np.tril(F) if uplo == 0 else np.triu(F)


@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 7, 33, 100])
def test_integer_factor_is_exact(uplo, n):
    A, L0 = synth.integer_spd(n, (110, n, 0))
    F, info = oracle.potrf(uplo, A)
    assert info == 0
    assert np.array_equal(_tri(F, uplo), L0 if uplo == 0 else L0.T)


def test_two_by_two_closed_form():
    # [[4, 6], [6, 25]] = L L^T with L = [[2, 0], [3, 4]]
    A = np.array([[4.0, 6.0], [6.0, 25.0]])
    F, info = oracle.potrf(0, A)
    assert info == 0 and F[0, 0] == 2.0 and F[1, 0] == 3.0 and F[1, 1] == 4.0
    assert F[0, 1] == 6.0  # other triangle untouched


@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("n", [5, 64, 257])
def test_agrees_with_lapack_and_backward_bound(uplo, n):
    A = synth.spd_dominant(n, (111, n, 0))
    F, info = oracle.potrf(uplo, A)
    assert info == 0
    L = np.linalg.cholesky(A)
    got = _tri(F, uplo) if uplo == 0 else _tri(F, uplo).T
    assert np.max(np.abs(got - L)) <= 1e-13 * np.max(np.abs(L))
    gamma = (n + 1) * U / (1 - (n + 1) * U)
    assert oracle.chol_backward_error(uplo, A, F) <= gamma


def test_residual_of_perturbed_integer_factor():
    n = 9
    A, L0 = synth.integer_spd(n, (112, 0, 0))
    F = L0.copy(order="F")
    i, j = 6, 2
    F[i, j] += 0.5
    pairs = np.array([(i, jj) for jj in range(i + 1)] + [(3, 1), (8, 7), (5, 1)])
    r, d = oracle.chol_residual(0, A, F, pairs)
    # row i of F F^T changes by 0.5 L0[jj, j] at jj in [j, i) and by
    # L0[i, j] + 0.25 at (i, i); every other entry is exact
    want = []
    for ii, jj in pairs:
        if ii == i and j <= jj < i:
            want.append(-0.5 * L0[jj, j])
        elif ii == i and jj == i:
            want.append(-(L0[i, j] + 0.25))
        else:
            want.append(0.0)
    assert np.array_equal(r, np.array(want))
    absF = np.abs(F)
    dwant = [float(np.dot(absF[ii, :jj + 1], absF[jj, :jj + 1])) for ii, jj in pairs]
    assert np.array_equal(d, np.array(dwant))


@pytest.mark.parametrize("uplo", [0, 1])
def test_info_reports_first_indefinite_minor(uplo):
    A = np.diag([1.0, 2.0, -1.0, 3.0])
    F, info = oracle.potrf(uplo, A)
    assert info == 3
    assert F[0, 0] == 1.0 and F[1, 1] == np.sqrt(2.0) and F[2, 2] == -1.0  # stops at column 2
    _, info = oracle.potrf(uplo, np.ones((2, 2)))  # singular: second pivot is 0
    assert info == 2
    B = np.eye(6)
    B[4, 4] = np.nan
    _, info = oracle.potrf(uplo, B)
    assert info == 5
    # an integer matrix made indefinite at column k: columns before k are L0's
    n, k = 20, 13
    A, L0 = synth.integer_spd(n, (113, 0, 0))
    A[k, k] -= L0[k, k] ** 2 + 1.0
    F, info = oracle.potrf(uplo, A)
    assert info == k + 1
    got = _tri(F, uplo) if uplo == 0 else _tri(F, uplo).T
    assert np.array_equal(got[:, :k], L0[:, :k])


@pytest.mark.parametrize("uplo", [0, 1])
def test_other_triangle_neither_read_nor_written(uplo):
    n = 40
    A = synth.spd_dominant(n, (114, 0, 0))
    clean, _ = oracle.potrf(uplo, A)
    other = np.triu_indices(n, 1) if uplo == 0 else np.tril_indices(n, -1)
    An = A.copy(order="F")
    An[other] = np.nan
    F, info = oracle.potrf(uplo, An)
    assert info == 0
    assert np.all(np.isnan(F[other]))
    mine = np.tril_indices(n) if uplo == 0 else np.triu_indices(n)
    assert np.array_equal(F[mine], clean[mine])


def test_power_of_two_scaling_commutes():
    n = 50
    A = synth.spd_dominant(n, (115, 0, 0))
    e = synth.rng((115, 0, 1)).integers(-20, 21, size=n)
    D = np.ldexp(1.0, e)
    F, _ = oracle.potrf(0, A)
    Fs, _ = oracle.potrf(0, A * D[:, None] * D[None, :])
    assert np.array_equal(np.tril(Fs), np.tril(F) * D[:, None])


# ---------------------------------------------------------------- planted mistakes
MUTANTS = [
    ("sign of the pivot update", "piv = piv - l * l;", "piv = piv + l * l;"),
    ("dropped term", "for (int64_t k = 0; k < j; ++k) s = s -", "for (int64_t k = 1; k < j; ++k) s = s -"),
    ("transposed operand", "s = s - a[at(uplo, i, k, lda)] * a[at(uplo, j, k, lda)];",
     "s = s - a[at(uplo, k, i, lda)] * a[at(uplo, j, k, lda)];"),
    ("division by the pivot", "a[at(uplo, i, j, lda)] = s / ljj;", "a[at(uplo, i, j, lda)] = s / piv;"),
    ("upper storage ignored", "return uplo == 0 ? i + j * lda : j + i * lda;", "return i + j * lda;"),
    ("info off by one", "if (!(piv > 0.0)) return (int)(j + 1);", "if (!(piv > 0.0)) return (int)j;"),
    ("dot2 error term dropped", "c = c + (q + l);", "c = c + q;"),
]


def _pins_pass(lib_path):
    lib = ctypes.CDLL(lib_path)
    i64, ptr, cint = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    lib.oracle_potrf.restype = cint
    lib.oracle_potrf.argtypes = [cint, i64, ptr, i64]
    lib.oracle_chol_residual.restype = None
    lib.oracle_chol_residual.argtypes = [cint, i64, ptr, i64, ptr, i64, i64, ptr, ptr, ptr, ptr]

    def potrf(uplo, A):
        F = np.array(A, dtype=np.float64, order="F", copy=True)
        return F, lib.oracle_potrf(uplo, F.shape[0], F.ctypes.data, F.shape[0])

    for uplo in (0, 1):
        A, L0 = synth.integer_spd(12, (116, uplo, 0))
        F, info = potrf(uplo, A)
        if info != 0 or not np.array_equal(_tri(F, uplo), L0 if uplo == 0 else L0.T):
            return False
        _, info = potrf(uplo, np.diag([1.0, 2.0, -1.0, 3.0]))
        if info != 3:
            return False
    # Dot2 residual of a factor with an error far below its terms: the exact
    # residual at (j, j) is -e (2 L0[j, j] + e) with e = 2^-40, representable,
    # while the plainly rounded sum loses the e^2 term
    A, L0 = synth.integer_spd(8, (117, 0, 0))
    F = L0.copy(order="F")
    j = 5
    F[j, j] += 2.0 ** -40
    pi = np.array([j], dtype=np.int64)
    pj = np.array([j], dtype=np.int64)
    r = np.zeros(1)
    d = np.zeros(1)
    lib.oracle_chol_residual(0, 8, A.ctypes.data, 8, F.ctypes.data, 8, 1, pi.ctypes.data,
                             pj.ctypes.data, r.ctypes.data, d.ctypes.data)
    want = -(2.0 ** -40) * (2.0 * L0[j, j] + 2.0 ** -40)
    return r[0] == want


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_planted_mistakes_are_caught(tmp_path):
    from oracle import build
    src = open(build.CHOL_SRC).read()
    flags = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared"]
    good = tmp_path / "good.so"
    subprocess.run(flags + [build.CHOL_SRC, "-o", str(good), "-lm"], check=True)
    assert _pins_pass(str(good))
    for idx, (label, old, new) in enumerate(MUTANTS):
        assert src.count(old) == 1, label
        c = tmp_path / ("m%d.c" % idx)
        c.write_text(src.replace(old, new))
        so = str(c) + ".so"
        subprocess.run(flags + [str(c), "-o", so, "-lm"], check=True)
        assert not _pins_pass(so), "pins missed planted mistake: " + label
