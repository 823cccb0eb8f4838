"""The paper's analytic latency model, refitted to measured MI355X times, as
an interpretable picker baseline.

Sec. V gives, for refinement level r = n / nb (the paper's r(i) = 2^i), the
latency of each model of computation as Comp + Comm:

* recursive (Sec. V-A): r leaves plus, at split depth j = 0 .. log2(r) - 1,
  2^j products of order n / 2^(j+1):
      Comp = r TS(nb) + sum_j 2^j gemm(n/2^(j+1), n/2^(j+1));
* iterative (Sec. V-B): r leaves and r - 1 panels, panel j of
  (n - (j+1) nb) rows by nb columns (right-looking):
      Comp = r TS(nb) + sum_{j=0}^{r-2} gemm(n - (j+1) nb, nb);
* blocked (Sec. V-C): r leaves and (r - 1) rounds of r / 2 equal blocks
  (7 x 4 = 28 at r = 8):
      Comp = r TS(nb) + (r - 1) (r / 2) gemm(nb, nb);
* Comm: the paper prices the host-device transfers of each offloaded task.
  Here everything stays in HBM, so the per-task cost is a kernel launch:
      Comm = (tasks) x t_launch.

TS(nb) and gemm(M, K) (with the right-hand-side count as N) are not the
paper's LLVM estimates but measurements of this library's kernels on the
GPU: a leaf table (one solve of order nb per right-hand-side count) and a
product table on a grid of M = K and N, both interpolated in log space.  The
model picks the cheapest (model, nb) in native precision; it has no notion of
refinement precision, as the paper's has none.
"""
from __future__ import annotations

import bisect
import math
from typing import Dict, Sequence, Tuple

NB_CHOICES = (32, 64, 128, 256, 512)
VARIANTS = ("recursive", "iterative", "blocked")


def _interp(xs: Sequence[float], ys: Sequence[float], x: float) -> float:
    """Piecewise-linear interpolation of log y over log x, clamped at the ends."""
    lx = [math.log(v) for v in xs]
    t = math.log(max(x, 1e-30))
    if t <= lx[0]:
        return ys[0]
    if t >= lx[-1]:
        return ys[-1]
    i = bisect.bisect_right(lx, t) - 1
    w = (t - lx[i]) / (lx[i + 1] - lx[i])
    return math.exp((1 - w) * math.log(ys[i]) + w * math.log(ys[i + 1]))


class Tables:
    """Measured primitives: leaf[nrhs][nb] and gemm[(mk, n)] in milliseconds
    (mk: M = K of a square-panel product), plus the launch latency."""

    def __init__(self, leaf: Dict[int, Dict[int, float]], gemm: Dict[Tuple[int, int], float],
                 launch_ms: float):
        self.leaf = leaf
        self.leaf_cols = sorted(leaf)
        self.gemm = gemm
        self.mks = sorted({k[0] for k in gemm})
        self.ns = sorted({k[1] for k in gemm})
        self.launch_ms = launch_ms

    def ts(self, nb: int, nrhs: int) -> float:
        return _interp(self.leaf_cols, [self.leaf[c][nb] for c in self.leaf_cols], nrhs)

    def gemm_ms(self, M: int, K: int, N: int) -> float:
        """A product's time from the square table: the time of the square
        product of equal flop count (M K = mk^2) at this N, interpolated."""
        if M <= 0 or K <= 0 or N <= 0:
            return 0.0
        mk = math.sqrt(float(M) * float(K))
        per_n = [_interp(self.mks, [self.gemm[(m, n)] for m in self.mks], mk) for n in self.ns]
        return _interp(self.ns, per_n, N)


def task_counts(variant: str, r: int) -> Tuple[int, int]:
    """(leaves, products) of the model at refinement r (a power of two)."""
    if variant == "recursive":
        return r, sum(2 ** j for j in range(int(math.log2(r))))
    if variant == "iterative":
        return r, r - 1
    if variant == "blocked":
        return r, (r - 1) * (r // 2)
    raise ValueError(variant)


def latency(variant: str, n: int, nrhs: int, nb: int, tab: Tables) -> float:
    """Comp + Comm of the model in milliseconds (n rounded up to nb r with r a
    power of two, as the paper's refinement levels are)."""
    r = 1
    while r * nb < n:
        r *= 2
    nr = nb * r  # the order the model's partition covers
    leaves, products = task_counts(variant, r)
    comp = leaves * tab.ts(nb, nrhs)
    if variant == "recursive":
        for j in range(int(math.log2(r))):
            side = nr // 2 ** (j + 1)
            comp += 2 ** j * tab.gemm_ms(side, side, nrhs)
    elif variant == "iterative":
        for j in range(r - 1):
            comp += tab.gemm_ms(nr - (j + 1) * nb, nb, nrhs)
    else:
        comp += (r - 1) * (r // 2) * tab.gemm_ms(nb, nb, nrhs)
    comm = (leaves + products) * tab.launch_ms
    return comp + comm


def pick(n: int, nrhs: int, tab: Tables) -> int:
    """Candidate index (15 (variant - 1) + 3 nb_index, native precision) of the
    cheapest model; ties to the lower index."""
    best, best_t = 0, float("inf")
    for v, name in enumerate(VARIANTS):
        for b, nb in enumerate(NB_CHOICES):
            if nb > max(32, 1 << (max(n, 1) - 1).bit_length()):
                continue  # a leaf larger than the matrix is the same as the matrix
            t = latency(name, n, nrhs, nb, tab)
            if t < best_t:
                best, best_t = 15 * v + 3 * b, t
    return best


def load(leaf_json: dict, gemm_json: dict) -> Tables:
    leaf = {int(k): {int(nb): float(v) for nb, v in row.items()} for k, row in leaf_json.items()}
    gemm = {(int(e["mk"]), int(e["n"])): float(e["ms"]) for e in gemm_json["entries"]}
    return Tables(leaf, gemm, float(gemm_json["launch_ms"]))
