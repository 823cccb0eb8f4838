"""Write kappa_family.json: the diagonal constant c of the matrix family
synth.kappa_lower(n, c, key) that gives a target one-norm condition number.

Uses only the CPU oracle (exact kappa for n <= 2048, the Hager-Higham
estimate above) and the input generator.  Bisection on log c; a result is
accepted within +-25 % of the target.  Run from the repository root:
    python tests/golden/make_kappa_table.py
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import kappa  # noqa: E402

KEY = (2, 0, 0)
TARGETS = [1e2, 1e4, 1e6]
ORDERS = [512, 2048, 8192, 16384]


def kappa_of(n, L):
    return kappa.kappa1_exact(L) if n <= 2048 else kappa.kappa1_estimate(L)


def main():
    out = {"key": list(KEY), "family": "synth.kappa_lower", "entries": []}
    for n in ORDERS:
        base = synth.kappa_lower(n, 1.0, KEY)
        d1 = base[0, 0]  # = 1.0 * (1 + max row sum)
        for target in TARGETS:
            lo, hi = math.log(1e-4), math.log(1.0)
            best = None
            for _ in range(40):
                mid = 0.5 * (lo + hi)
                c = math.exp(mid)
                L = base.copy(order="F")
                L[np.diag_indices(n)] = c * d1
                k = kappa_of(n, L)
                if best is None or abs(math.log(k / target)) < abs(math.log(best[1] / target)):
                    best = (c, k)
                if abs(math.log(k / target)) < math.log(1.05):
                    break
                if k > target:
                    lo = mid
                else:
                    hi = mid
            c, k = best
            ok = abs(k / target - 1.0) <= 0.25
            print("n=%d target=%.0e c=%.6g kappa=%.4g %s" % (n, target, c, k, "ok" if ok else "MISS"),
                  flush=True)
            out["entries"].append({"n": n, "target": target, "c": c, "kappa1": k,
                                   "method": "exact" if n <= 2048 else "hager-higham",
                                   "accepted": bool(ok)})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kappa_family.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
