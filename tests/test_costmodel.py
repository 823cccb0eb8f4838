"""The paper's analytic latency model (Sec. V-A/B/C) as written in
costmodel.py: its task counts and terms against the formulas, on synthetic
primitive tables whose values make each term visible."""
import math

import pytest

from paper_2305_19917_amd import costmodel


def _tables(ts=1.0, gemm=lambda mk, n: 0.0, launch=0.0, nbs=costmodel.NB_CHOICES):
    leaf = {c: {nb: ts for nb in nbs} for c in (1, 16, 256, 4096)}
    g = {(mk, n): max(gemm(mk, n), 1e-300) for mk in (16, 32, 64, 128, 256, 512, 1024, 2048, 4096,
                                                       8192, 16384)
         for n in (1, 16, 256, 4096)}
    return costmodel.Tables(leaf, g, launch)


@pytest.mark.parametrize("r", [1, 2, 4, 8, 64])
def test_task_counts(r):
    # recursive: r leaves and r - 1 products (2^j products at depth j)
    assert costmodel.task_counts("recursive", r) == (r, r - 1)
    assert costmodel.task_counts("iterative", r) == (r, r - 1)
    assert costmodel.task_counts("blocked", r) == (r, (r - 1) * (r // 2))


def test_blocked_count_of_the_paper_example():
    # Fig. 5: refinement 8, 7 rounds of 4 blocks, 28 blocks
    assert costmodel.task_counts("blocked", 8)[1] == 28


def test_leaf_term_and_launch_term():
    tab = _tables(ts=0.5, launch=0.01)
    n, nb = 4096, 256  # r = 16
    for v in costmodel.VARIANTS:
        leaves, prods = costmodel.task_counts(v, 16)
        # products cost ~0 here: Comp = r TS, Comm = tasks x launch
        got = costmodel.latency(v, n, 16, nb, tab)
        assert got == pytest.approx(16 * 0.5 + (leaves + prods) * 0.01, rel=1e-9, abs=1e-12)


def test_gemm_terms_follow_the_formulas():
    # products priced by flops (time = mk^2 n): the recursive sum is
    # sum_j 2^j (n/2^(j+1))^2 N, the blocked one (r-1) r/2 nb^2 N and the
    # iterative one sum_j (n - (j+1) nb) nb N
    tab = _tables(ts=1e-300, gemm=lambda mk, n: float(mk) ** 2 * n)
    n, nb, N = 4096, 512, 16
    r = n // nb
    rec = sum(2 ** j * (n / 2 ** (j + 1)) ** 2 * N for j in range(int(math.log2(r))))
    blk = (r - 1) * (r // 2) * nb ** 2 * N
    itr = sum((n - (j + 1) * nb) * nb * N for j in range(r - 1))
    assert costmodel.latency("recursive", n, N, nb, tab) == pytest.approx(rec, rel=1e-6)
    assert costmodel.latency("blocked", n, N, nb, tab) == pytest.approx(blk, rel=1e-6)
    assert costmodel.latency("iterative", n, N, nb, tab) == pytest.approx(itr, rel=1e-6)
    # flop identity of the three partitions (products add to n^2 - r nb^2 halves)
    assert rec == pytest.approx(itr, rel=1e-12) and itr == pytest.approx(blk, rel=1e-12)


def test_pick_prefers_cheaper_leaves_when_products_are_free():
    # leaves cost nb^2: the smallest leaf wins, recursive first on ties
    leaf = {c: {nb: float(nb) ** 2 for nb in costmodel.NB_CHOICES} for c in (1, 4096)}
    g = {(mk, n): 1e-300 for mk in (16, 16384) for n in (1, 4096)}
    tab = costmodel.Tables(leaf, g, 0.0)
    assert costmodel.pick(4096, 64, tab) == 0  # recursive, nb 32, native
