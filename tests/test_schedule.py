"""Planner tests on the host (no GPU): the task lists the library builds for
the recursive, iterative and blocked models of Sec. V.

* every schedule covers the triangle exactly once: the leaf and product flop
  counts add up to exactly m^2 per right-hand side;
* the counts the paper states hold: r leaves and r-1 panels (Sec. V-B), r-1
  rounds of r/2 blocks, (r-1) r / 2 blocks in all, 28 for r = 8 (Sec. V-C);
* dependencies hold: a product only reads solved rows and only writes rows
  not yet solved; no two products of one launch write the same rows;
* a CPU interpreter that runs the task list (oracle leaves, library
  products) reproduces the oracle's solution.
"""
import numpy as np
import pytest

import oracle
import paper_2305_19917_amd as rs
import synth

LEAF, GEMM = 0, 1


def _tasks(variant, m, nb):
    return rs.schedule(variant, m, nb)


@pytest.mark.parametrize("variant", ["recursive", "iterative", "blocked"])
@pytest.mark.parametrize("m,nb", [(1, 16), (16, 16), (17, 16), (100, 16), (512, 64), (1000, 64),
                                  (8192, 128), (4096, 256), (777, 32)])
def test_flop_identity(variant, m, nb):
    flops = 0
    for kind, r0, rows, c0, cols, rnd in _tasks(variant, m, nb):
        flops += rows * rows if kind == LEAF else 2 * rows * cols
    assert flops == m * m


@pytest.mark.parametrize("variant", ["recursive", "iterative", "blocked"])
@pytest.mark.parametrize("m,nb", [(64, 16), (100, 16), (1000, 64), (2048, 128), (333, 32)])
def test_dependencies(variant, m, nb):
    solved = np.zeros(m, bool)
    pending_rounds = {}
    for kind, r0, rows, c0, cols, rnd in _tasks(variant, m, nb):
        if kind == LEAF:
            assert not solved[r0:r0 + rows].any()
            # every product into these rows must have been issued before
            solved[r0:r0 + rows] = True
        else:
            assert solved[c0:c0 + cols].all(), "product reads unsolved rows"
            assert not solved[r0:r0 + rows].any(), "product writes solved rows"
            w = pending_rounds.setdefault(rnd, np.zeros(m, bool))
            assert not w[r0:r0 + rows].any(), "two writers in one launch"
            w[r0:r0 + rows] = True
    assert solved.all()


@pytest.mark.parametrize("variant", ["recursive", "iterative", "blocked"])
@pytest.mark.parametrize("m,nb", [(64, 16), (1000, 64), (2048, 128), (4096, 32), (8192, 256),
                                  (333, 32)])
def test_lookahead_splits_are_safe(variant, m, nb):
    """The executor's look-ahead runs, beside the leaf that follows a
    launch, every product of that launch that does not write the leaf's rows
    (for a single product: the rows past the leaf).  That is only race-free
    if such a leaf exists right after the launch, a product either writes
    all of the leaf's rows or none of them (blocked rounds; a single product
    starts at the leaf's first row), and nothing of the launch reads the rows
    the leaf writes."""
    t = _tasks(variant, m, nb)
    for k in range(len(t) - 1):
        kind, r0, rows, c0, cols, rnd = t[k]
        nxt = t[k + 1]
        if kind != GEMM or nxt[0] != LEAF:
            continue
        leaf_r0, leaf_rows = nxt[1], nxt[2]
        launch = [x for x in t if x[0] == GEMM and x[5] == rnd]
        for _, b_r0, b_rows, b_c0, b_cols, _ in launch:
            overlap = b_r0 < leaf_r0 + leaf_rows and leaf_r0 < b_r0 + b_rows
            if len(launch) > 1:
                assert not overlap or (b_r0 == leaf_r0 and b_rows == leaf_rows)
            else:
                assert b_r0 == leaf_r0 and b_rows >= leaf_rows
            # reads only rows solved before the leaf
            assert b_c0 + b_cols <= leaf_r0
    kinds = [x[0] for x in t]
    assert not any(a == LEAF and b == LEAF for a, b in zip(kinds, kinds[1:]))


def test_each_product_pair_applied_once():
    """Every (row, column) pair of the strict lower triangle is subtracted
    exactly once, at leaf granularity."""
    for variant in ("recursive", "iterative", "blocked"):
        m, nb = 640, 32
        hits = np.zeros((m, m), np.int64)
        for kind, r0, rows, c0, cols, _ in _tasks(variant, m, nb):
            if kind == GEMM:
                hits[r0:r0 + rows, c0:c0 + cols] += 1
            else:
                hits[r0:r0 + rows, r0:r0 + rows] += np.tril(np.ones((rows, rows), np.int64), -1)
        assert np.array_equal(hits, np.tril(np.ones((m, m), np.int64), -1)), variant


def test_recursive_levels():
    """Sec. V-A with r(i) = 2^i: at level j there are 2^j products of
    (m/2^(j+1))^2 each, and r leaves of order m / r."""
    m, nb = 1024, 64
    t = _tasks("recursive", m, nb)
    leaves = [x for x in t if x[0] == LEAF]
    prods = [x for x in t if x[0] == GEMM]
    assert len(leaves) == m // nb and all(x[2] == nb for x in leaves)
    for j in range(4):
        size = m // 2 ** (j + 1)
        assert sum(1 for x in prods if x[2] == size and x[4] == size) == 2 ** j


def test_iterative_counts():
    m, nb = 2048, 128
    t = _tasks("iterative", m, nb)
    r = m // nb
    assert sum(1 for x in t if x[0] == LEAF) == r
    prods = [x for x in t if x[0] == GEMM]
    assert len(prods) == r - 1
    # right-looking: panel p updates every row below leaf p with K = nb
    for p, x in enumerate(prods):
        assert x[1] == (p + 1) * nb and x[2] == m - (p + 1) * nb and x[3] == p * nb and x[4] == nb


@pytest.mark.parametrize("r", [2, 4, 8, 16, 32, 64, 128, 256])
def test_blocked_rounds_paper_counts(r):
    nb = 16
    t = _tasks("blocked", r * nb, nb)
    rounds = {}
    blocks = 0
    for kind, r0, rows, c0, cols, rnd in t:
        if kind == GEMM:
            rounds.setdefault(rnd, 0)
            nblk = cols // nb  # K-merged products count their blocks
            rounds[rnd] += nblk
            blocks += nblk
    assert len(rounds) == r - 1
    assert all(v == r // 2 for v in rounds.values())
    assert blocks == (r - 1) * r // 2


def test_blocked_example_r8():
    """Fig. 5 / Sec. V-C: refinement 8 gives 7 rounds of 4 blocks, 28 blocks."""
    t = _tasks("blocked", 8 * 32, 32)
    rounds = {}
    for kind, r0, rows, c0, cols, rnd in t:
        if kind == GEMM:
            p = r0 // 32
            rounds.setdefault(rnd, []).extend((p, c0 // 32 + q) for q in range(cols // 32))
    got = [sorted(v) for _, v in sorted(rounds.items())]
    assert sum(len(v) for v in got) == 28
    assert got[0] == [(1, 0), (2, 0), (3, 0), (4, 0)]
    assert got[1] == [(2, 1), (3, 1), (4, 1), (5, 0)]
    assert got[2] == [(3, 2), (4, 2), (5, 1), (5, 2)]


def test_blocked_odd_counts_valid():
    for r in (3, 5, 7, 9, 13):
        m, nb = r * 16 - 5, 16
        test_dependencies("blocked", m, nb)


def _interpret(variant, A, B, nb):
    """Run the task list on the CPU: leaves by the oracle, products by numpy."""
    X = np.array(B, dtype=np.float64, order="F", copy=True)
    m = A.shape[0]
    for kind, r0, rows, c0, cols, _ in _tasks(variant, m, nb):
        if kind == LEAF:
            X[r0:r0 + rows] = oracle.trsm_plain(0, 0, 0, 0, 1.0, A[r0:r0 + rows, r0:r0 + rows],
                                                X[r0:r0 + rows])
        else:
            X[r0:r0 + rows] -= A[r0:r0 + rows, c0:c0 + cols] @ X[c0:c0 + cols]
    return X


@pytest.mark.parametrize("variant", ["recursive", "iterative", "blocked"])
@pytest.mark.parametrize("m,nb", [(300, 32), (512, 64), (200, 128)])
def test_cpu_interpreter_matches_oracle(variant, m, nb):
    A = synth.dominant_lower(m, (20, m, 0))
    B = synth.rhs_normal(m, 9, (20, m, 1))
    X = _interpret(variant, A, B, nb)
    assert oracle.backward_error(0, 0, 0, 0, 1.0, A, B, X) <= 1e-14 * m
    Xo = oracle.trsm_plain(0, 0, 0, 0, 1.0, A, B)
    assert oracle.forward_error(X, Xo) <= 1e-12


@pytest.mark.parametrize("nb", [128, 256])
def test_bench_algorithmic_bytes_follow_the_schedule(nb):
    """bench.py's algorithmic bytes per product launch (the roofline's
    denominator) are computed from the same recursive split as the planner's
    products: same count, same M x K shapes."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "bench", os.path.join(os.path.dirname(__file__), os.pardir, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    n = nrhs = 8192
    prods = [(rows, cols) for kind, _, rows, _, cols, _ in _tasks("recursive", n, nb) if kind == GEMM]
    want = sum(8.0 * (m * k + k * nrhs + 2 * m * nrhs) for m, k in prods) / len(prods)
    assert bench.algorithmic_bytes(n, nrhs, nb) == pytest.approx(want, rel=1e-12)
    assert len(prods) == n // nb - 1
