"""Condition-number tools of the oracle, pinned to a library routine, and the
stored kappa-family table (written by tests/golden/make_kappa_table.py)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import kappa

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kappa_family.json")


@pytest.mark.parametrize("n,c", [(20, 0.5), (64, 0.05), (150, 0.02), (300, 0.01)])
def test_exact_kappa_matches_library(n, c):
    L = synth.kappa_lower(n, c, (40, n, 0))
    ref = np.linalg.cond(np.tril(L), 1)
    assert kappa.kappa1_exact(L) == pytest.approx(ref, rel=1e-6)


@pytest.mark.parametrize("n,c", [(50, 0.1), (200, 0.02), (400, 0.015)])
def test_estimate_is_a_tight_lower_bound(n, c):
    L = synth.kappa_lower(n, c, (41, n, 0))
    ex = kappa.kappa1_exact(L)
    est = kappa.kappa1_estimate(L)
    assert est <= ex * (1 + 1e-9)
    assert est >= ex / 3


def test_smaller_c_is_worse_conditioned():
    ks = [kappa.kappa1_exact(synth.kappa_lower(256, c, (42, 0, 0))) for c in (0.2, 0.05, 0.02)]
    assert ks[0] < ks[1] < ks[2]


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="table not generated")
def test_golden_table_entries():
    tab = json.load(open(GOLDEN))
    assert tab["family"] == "synth.kappa_lower"
    entries = tab["entries"]
    assert {e["target"] for e in entries} == {1e2, 1e4, 1e6}
    for e in entries:
        assert e["accepted"], e
        assert abs(e["kappa1"] / e["target"] - 1) <= 0.25
    # recompute the small entries exactly
    for e in entries:
        if e["n"] == 512:
            L = synth.kappa_lower(512, e["c"], tuple(tab["key"]))
            assert kappa.kappa1_exact(L) == pytest.approx(e["kappa1"], rel=1e-9)
