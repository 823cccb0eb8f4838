"""Pins for the oracle's error metrics (oracle/__init__.py), both sides.

Every expected value below is worked out by hand from the definitions
(normwise backward error, Rigal and Gaches / Higham Thm 7.1; componentwise
backward error, Oettli and Prager / Higham Thm 7.3; forward error per
right-hand side) on small exact inputs, so it does not come from the oracle.
The right side solves X op(A) = alpha B: a right-hand side is a ROW of B and
X, its matrix is op(A)^T, whose infinity norm is the one norm of op(A).

A final test plants plausible mistakes in a copy of the metric code and
checks that these pins catch each one.
"""
import types

import numpy as np
import pytest

import oracle

# op(A) = [[1, 0], [3, 2]] stored lower: ||op(A)||_inf = 5 (rows), ||op(A)||_1 = 4 (columns)
A2 = np.asfortranarray([[1.0, 0.0], [3.0, 2.0]])
# right side: rows x of X with x op(A) = [4, 2] and [-1, -2]; b leaves r = [0, 0.5], [-0.25, 0]
X_R = np.asfortranarray([[1.0, 1.0], [2.0, -1.0]])
B_R = np.asfortranarray([[4.0, 2.5], [-1.25, -2.0]])


def _check_metrics(mod):
    """The pins as one predicate, so the planted-mistake test can reuse them."""
    ok = True
    # right side, normwise: row 0: 0.5 / (4 * 1 + 4) = 1/16; row 1: 0.25 / (4 * 2 + 2) = 1/40
    eta = mod.backward_error(1, 0, 0, 0, 1.0, A2, B_R, X_R, per_rhs=True)
    ok &= np.array_equal(eta, np.array([0.5 / 8.0, 0.25 / 10.0]))
    ok &= mod.backward_error(1, 0, 0, 0, 1.0, A2, B_R, X_R) == 0.5 / 8.0
    # right side, componentwise: (|X||A| + |B|) = [[8, 4.5], [6.25, 4]], |r| = [[0, .5], [.25, 0]]
    ok &= mod.componentwise_error(1, 0, 0, 0, 1.0, A2, B_R, X_R) == 0.5 / 4.5
    # left side with the same matrix: op(A) x = b per column; x = [1, 2]: A x = [1, 7]
    x = np.asfortranarray([[1.0], [2.0]])
    b = np.asfortranarray([[1.0], [7.5]])  # r = [0, 0.5]
    ok &= mod.backward_error(0, 0, 0, 0, 1.0, A2, b, x) == 0.5 / (5.0 * 2.0 + 7.5)
    # (|A||x| + |b|) = [2, 14.5]
    ok &= mod.componentwise_error(0, 0, 0, 0, 1.0, A2, b, x) == 0.5 / 14.5
    # alpha enters the denominator as |alpha b|: alpha = 2, b halved gives the same system
    ok &= mod.backward_error(0, 0, 0, 0, 2.0, A2, b / 2.0, x) == 0.5 / (5.0 * 2.0 + 7.5)
    # forward error, per column (left) and per row (right)
    Xref = np.array([[1.0, -4.0], [2.0, 2.0]])
    Xh = Xref + np.array([[0.5, 0.0], [0.0, 0.75]])
    ok &= mod.forward_error(Xh, Xref) == 0.25          # columns: .5/2, .75/4
    ok &= mod.forward_error(Xh, Xref, side=1) == 0.375  # rows: .5/4, .75/2
    # zero reference with a nonzero error is infinite; equal zero vectors are exact
    ok &= mod.forward_error(np.array([[1.0]]), np.array([[0.0]])) == np.inf
    ok &= mod.forward_error(np.zeros((3, 2)), np.zeros((3, 2))) == 0.0
    return bool(ok)


def test_metric_pins():
    assert _check_metrics(oracle)


def test_backward_error_right_side_uses_one_norm():
    # spelled out: the right-side denominator takes ||op(A)||_1 = 4, not ||op(A)||_inf = 5
    assert oracle.opnorm(0, 0, 0, A2, 2, "one") == 4.0
    assert oracle.opnorm(0, 0, 0, A2, 2, "inf") == 5.0
    assert oracle.backward_error(1, 0, 0, 0, 1.0, A2, B_R, X_R) == 0.0625


def test_backward_error_transposed_right_side():
    # trans: op(A) = A^T = [[1, 3], [0, 2]]; ||op(A)||_1 = 5.  x = [1, 1]: x op(A) = [1, 5]
    x = np.asfortranarray([[1.0, 1.0]])
    b = np.asfortranarray([[1.0, 5.25]])  # r = [0, 0.25]
    assert oracle.backward_error(1, 0, 1, 0, 1.0, A2, b, x) == 0.25 / (5.0 + 5.25)
    # |x||op(A)| + |b| = [2, 10.25]
    assert oracle.componentwise_error(1, 0, 1, 0, 1.0, A2, b, x) == 0.25 / 10.25


METRIC_MUTANTS = [
    ("right side takes the infinity norm",
     '"inf" if side == LEFT else "one"', '"inf"'),
    ("right side reduced over columns",
     "    axis = 0 if side == LEFT else 1\n    anorm", "    axis = 0\n    anorm"),
    ("alpha b term dropped", "den = anorm * xn + bn", "den = anorm * xn"),
    ("componentwise right side with the left product",
     "np.abs(X) @ T)", "T @ np.abs(X))"),
    ("componentwise right side with the transposed matrix",
     "np.abs(X) @ T)", "np.abs(X) @ T.T)"),
    ("forward error numerator halved",
     "num = np.max(np.abs(X - Xref)", "num = 0.5 * np.max(np.abs(X - Xref)"),
    ("forward error right side reduced over columns",
     "    axis = 0 if side == LEFT else 1\n    num", "    axis = 0\n    num"),
]


def _load_mutant(src, tag):
    mod = types.ModuleType("oracle._mutant_%s" % tag)
    mod.__package__ = "oracle"
    mod.__file__ = oracle.__file__
    exec(compile(src, "<oracle mutant %s>" % tag, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("label,old,new", METRIC_MUTANTS, ids=[m[0] for m in METRIC_MUTANTS])
def test_planted_metric_mistakes_are_caught(label, old, new):
    src = open(oracle.__file__).read()
    assert src.count(old) == 1, label
    assert _check_metrics(_load_mutant(src, "ok"))
    assert not _check_metrics(_load_mutant(src.replace(old, new), "bad")), label
