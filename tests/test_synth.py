"""Input generators: reproducible, and with the structure they promise."""
import numpy as np

import synth


def test_seeds_reproduce_and_differ():
    a = synth.dominant_lower(64, (0, 0, 0))
    b = synth.dominant_lower(64, (0, 0, 0))
    c = synth.dominant_lower(64, (0, 1, 0))
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert np.array_equal(synth.rhs_normal(10, 3, (0, 0, 1)), synth.rhs_normal(10, 3, (0, 0, 1)))


def test_dominant_lower_structure():
    n = 100
    L = synth.dominant_lower(n, (1, 0, 0))
    assert L.flags.f_contiguous
    assert np.all(np.triu(L, 1) == 0)
    off = np.tril(L, -1)
    assert np.all(np.abs(off) < 1)
    assert np.allclose(np.diag(L), 1 + np.abs(off).sum(axis=1), rtol=0, atol=1e-12)
    # the draw is taken in C order: L[i, j] = draw[i*n + j]
    draw = np.random.default_rng([1, 0, 0]).uniform(-1, 1, (n, n))
    assert L[5, 2] == draw[5, 2]


def test_unit_lower_diag_is_nan_and_rows_scaled():
    L = synth.dominant_lower(40, (2, 0, 0))
    U = synth.unit_lower(40, (2, 0, 0))
    assert np.all(np.isnan(np.diag(U)))
    assert np.all(np.isnan(U[np.triu_indices(40, 1)]))
    i, j = 17, 3
    assert U[i, j] == L[i, j] / L[i, i]


def test_kappa_lower_constant_diagonal():
    L = synth.kappa_lower(50, 0.1, (3, 0, 0))
    d = np.diag(L)
    assert np.all(d == d[0])
    off = np.tril(L, -1)
    assert d[0] == 0.1 * (1 + np.abs(off).sum(axis=1).max())


def test_integer_exact_is_exact():
    for side in (0, 1):
        for uplo in (0, 1):
            for trans in (0, 1):
                A, B, X = synth.integer_exact(9, 6, (4, side, uplo), side, uplo, trans, 0)
                k = 9 if side == 0 else 6
                T = np.tril(A) if uplo == 0 else np.triu(A)
                T = np.nan_to_num(T, nan=0.0)
                op = T.T if trans else T
                assert np.array_equal(op @ X if side == 0 else X @ op, B)
                assert np.all(np.abs(X) <= 4)


def test_batch_shapes_ranges():
    n, k = synth.batch_shapes(2000, (3, 0, 2))
    assert n.min() >= 32 and n.max() <= 1024
    assert k.min() >= 1 and k.max() <= 256
    assert 120 < np.median(n) < 260
