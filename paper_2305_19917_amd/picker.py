"""Learned schedule picker: timing database, training and evaluation.

The paper chooses its refinement level from an analytic cost model and stops
refining when two half-size leaves are no faster than one (Sec. V-A).  Here
the choice -- model of computation (recursive, iterative, blocked), leaf
size nb and precision (FP64, FP32 + refinement, BF16 + refinement) -- is made
by a small network trained on timings that the library's own exhaustive
tuner (redsea_tune_shape) measures.  Training and inference run on the
library's HIP kernels (redsea_mlp_grad / redsea_mlp_adam /
redsea_mlp_forward); this module only arranges data and launches them.

Features: (log2 n, log2 nrhs, dtype, log10 kappa); targets: the natural log
of the measured milliseconds of each of the 45 candidates, with a mask for
candidates that do not apply (refinement for FP32 data).  kappa is what an
AUTO solve uses: the caller's estimate when it gives one, else the ratio of
the largest to the smallest diagonal entry, which the library computes.  A
record of a constant-diagonal (conditioning) class therefore trains twice:
with its nominal kappa (a caller who knows it) and with kappa 1 (its
diagonal ratio, a caller who does not).  Records carry the device name and
the library's build id (its version string), and a database only resumes
records of the same device and build.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _binding as B

NCAND = 45
NB_CHOICES = (32, 64, 128, 256, 512)
# condition classes the tuner generates: constant-diagonal parameter c of the
# generated matrix (0 = diagonally dominant) and the one-norm condition number
# it gives (measured with the oracle for orders 512 .. 16384)
KAPPA_CLASSES = ((0.0, None), (0.105, 1e2), (0.012, 1e4), (0.004, 1e6))


def candidate(idx: int):
    v, nb, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    if B.lib().redsea_candidate(idx, ctypes.byref(v), ctypes.byref(nb), ctypes.byref(p)) != 0:
        raise IndexError(idx)
    return v.value, nb.value, p.value


def kappa_of_class(n: int, c: float, kappa: Optional[float]) -> float:
    """Feature value of a class as its caller would give it: the nominal kappa
    of a conditioning class, or the diagonal ratio of a dominant matrix."""
    return kappa if kappa else diag_ratio(n, c)


def diag_ratio(n: int, c: float) -> float:
    """max |a_ii| / min |a_ii| of the tuner's generated matrices: 1 for the
    constant diagonal of a conditioning class; for the dominant ones the
    diagonal 1 + sum |row| runs from 1 (row 0) to about 1 + (n - 1) / 2."""
    return 1.0 if c > 0 else 1.0 + (n - 1) / 2.0


def features(n, nrhs, dtype, kappa):
    return [math.log2(max(n, 1)), math.log2(max(nrhs, 1)), float(dtype),
            math.log10(max(kappa, 1.0))]


# ------------------------------------------------------------------ tuning

def tune(dtype: int, n: int, nrhs: int, c: float, seed: int, reps: int = 2, stream=None):
    """Milliseconds of every candidate for one generated shape (-1 = n/a).
    The library's default schedule is timed first, so that candidates far
    behind it are cut short from the start."""
    default = 3 * NB_CHOICES.index(256 if n > 128 else 128)
    order = [default] + [i for i in range(NCAND) if i != default]
    cand = (ctypes.c_int * NCAND)(*order)
    ms = (ctypes.c_double * NCAND)()
    rc = B.lib().redsea_tune_shape(dtype, n, nrhs, float(c), ctypes.c_uint64(seed), reps, cand,
                                   NCAND, ms, B._stream(stream) if stream is not None else None)
    if rc != 0:
        raise B.RedseaError(rc, B.status_string(rc))
    out = [0.0] * NCAND
    for pos, idx in enumerate(order):
        out[idx] = float(ms[pos])
    return out


# training range: orders and right-hand-side counts log-uniform in these
# intervals (the picker reports low confidence outside it)
N_RANGE = (64, 32768)
NRHS_RANGE = (1, 16384)


def sample_shapes(count: int, seed: int, n_range=N_RANGE, nrhs_range=NRHS_RANGE,
                  f32_share=0.25):
    """Log-uniform orders and right-hand-side counts, a dtype and a kappa class."""
    r = np.random.default_rng([4, seed])
    n = np.rint(np.exp(r.uniform(np.log(n_range[0]), np.log(n_range[1]), count))).astype(int)
    k = np.rint(np.exp(r.uniform(np.log(nrhs_range[0]), np.log(nrhs_range[1]), count))).astype(int)
    dt = (r.uniform(size=count) < f32_share).astype(int)
    cls = r.integers(0, len(KAPPA_CLASSES), count)
    cls[dt == 1] = 0
    return [dict(n=int(a), nrhs=int(b), dtype=int(d), cls=int(c)) for a, b, d, c in
            zip(n, k, dt, cls)]


def device_and_build():
    import torch
    return torch.cuda.get_device_name(0), B.version()


def build_db(path: str, shapes: Sequence[Dict], seed0: int, reps: int = 2, log=print):
    """Time every candidate of every shape, appending JSON lines to `path`;
    shapes already present for this device and library build (same n, nrhs,
    dtype, class) are skipped, so an interrupted run resumes."""
    dev, build = device_and_build()
    done = set()
    if os.path.exists(path):
        for line in open(path):
            d = json.loads(line)
            if d.get("device") == dev and d.get("build") == build:
                done.add((d["n"], d["nrhs"], d["dtype"], d["cls"]))
    with open(path, "a") as f:
        for i, s in enumerate(shapes):
            key = (s["n"], s["nrhs"], s["dtype"], s["cls"])
            if key in done:
                continue
            c, kap = KAPPA_CLASSES[s["cls"]]
            t0 = time.time()
            ms = tune(s["dtype"], s["n"], s["nrhs"], c, seed0 + i, reps)
            rec = dict(s, c=c, kappa=kappa_of_class(s["n"], c, kap),
                       kappa_diag=diag_ratio(s["n"], c), device=dev, build=build, ms=ms)
            f.write(json.dumps(rec) + "\n")
            f.flush()
            done.add(key)
            log("tuned %d/%d n=%d nrhs=%d dtype=%d cls=%d best=%.3f ms (%.1f s)" % (
                i + 1, len(shapes), s["n"], s["nrhs"], s["dtype"], s["cls"],
                min(x for x in ms if x > 0), time.time() - t0))


def load_db(path: str, training: bool = False):
    """Features, log-ms targets, masks and times of a database.  With
    `training`, a conditioning-class record appears twice (nominal kappa and
    diagonal-ratio kappa); otherwise once, with the kappa its caller gives."""
    recs = [json.loads(l) for l in open(path) if l.strip()]
    if training:
        recs = recs + [dict(r, kappa=r.get("kappa_diag", 1.0)) for r in recs if r["cls"] > 0]
    X = np.array([features(r["n"], r["nrhs"], r["dtype"], r["kappa"]) for r in recs], np.float64)
    ms = np.array([r["ms"] for r in recs], np.float64)
    mask = (ms > 0).astype(np.float64)
    T = np.where(ms > 0, np.log(np.where(ms > 0, ms, 1.0)), 0.0)
    return recs, X, T, mask, ms


# ------------------------------------------------------------------ network

class Net:
    """Parameters on the device plus the input normalisation."""

    def __init__(self, mu, sd, lo, hi, params=None, seed=0):
        import torch
        self.mu = np.asarray(mu, np.float64)
        self.sd = np.asarray(sd, np.float64)
        self.lo, self.hi = list(lo), list(hi)
        npar = B.lib().redsea_mlp_param_count()
        if params is None:
            params = init_params(seed)
        self.p = torch.tensor(np.asarray(params, np.float32), device="cuda")
        assert self.p.numel() == npar

    def norm(self, X):
        return ((np.asarray(X, np.float64) - self.mu) / self.sd).astype(np.float32)

    def predict(self, X):
        """Predicted log-ms of every candidate, from the GPU forward kernel."""
        import torch
        Xn = torch.tensor(self.norm(X), device="cuda")
        Y = torch.empty((Xn.shape[0], NCAND), dtype=torch.float32, device="cuda")
        B._check(B.lib().redsea_mlp_forward(self.p.data_ptr(), Xn.data_ptr(), Xn.shape[0],
                                            Y.data_ptr(), B._stream(None)))
        torch.cuda.synchronize()
        return Y.cpu().numpy().astype(np.float64)

    def save(self, path):
        P = self.p.cpu().numpy()
        with open(path, "w") as f:
            f.write("redsea-mlp 2\n%d 64 64 45\n" % len(self.mu))
            f.write(" ".join("%.9g" % v for v in self.mu) + "\n")
            f.write(" ".join("%.9g" % v for v in self.sd) + "\n")
            f.write("%.9g %.9g %.9g %.9g\n" % (self.lo[0], self.hi[0], self.lo[1], self.hi[1]))
            for i in range(0, P.size, 8):
                f.write(" ".join("%.9g" % v for v in P[i:i + 8]) + "\n")

    @staticmethod
    def load(path):
        tok = open(path).read().split()
        assert tok[0] == "redsea-mlp" and tok[1] == "2"
        nin = int(tok[2])
        vals = [float(t) for t in tok[6:]]
        mu, sd = vals[0:nin], vals[nin:2 * nin]
        lo = [vals[2 * nin], vals[2 * nin + 2]]
        hi = [vals[2 * nin + 1], vals[2 * nin + 3]]
        return Net(mu, sd, lo, hi, params=np.array(vals[2 * nin + 4:], np.float32))


def init_params(seed=0):
    """He-style initialisation, packed W1, b1, W2, b2, W3, b3."""
    r = np.random.default_rng([5, seed])
    sizes = (4, 64, 64, 45)
    out = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append(r.normal(0, math.sqrt(2.0 / a), (b, a)).ravel())
        out.append(np.zeros(b))
    return np.concatenate(out).astype(np.float32)


def train(X, T, mask, epochs=300, batch=256, lr=3e-3, seed=0, net: Optional[Net] = None,
          log=None):
    """Adam on the masked MSE of log-ms, all arithmetic in the library's HIP
    kernels.  Returns the network and the loss history (per epoch)."""
    import torch
    X = np.asarray(X, np.float64)
    if net is None:
        mu = X.mean(axis=0)
        sd = X.std(axis=0)
        sd[sd < 1e-6] = 1.0
        net = Net(mu, sd, [X[:, 0].min(), X[:, 1].min()], [X[:, 0].max(), X[:, 1].max()],
                  seed=seed)
    L = B.lib()
    dev = "cuda"
    Xn = torch.tensor(net.norm(X), device=dev)
    Td = torch.tensor(np.asarray(T, np.float32), device=dev)
    Md = torch.tensor(np.asarray(mask, np.float32), device=dev)
    g = torch.zeros_like(net.p)
    m = torch.zeros_like(net.p)
    v = torch.zeros_like(net.p)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    r = np.random.default_rng([6, seed])
    nS = Xn.shape[0]
    hist = []
    step = 0
    s = B._stream(None)
    for ep in range(epochs):
        perm = torch.tensor(r.permutation(nS), device=dev)
        tot = 0.0
        for b0 in range(0, nS, batch):
            idx = perm[b0:b0 + batch]
            xb, tb, mb = Xn[idx].contiguous(), Td[idx].contiguous(), Md[idx].contiguous()
            B._check(L.redsea_mlp_grad(net.p.data_ptr(), xb.data_ptr(), tb.data_ptr(),
                                       mb.data_ptr(), xb.shape[0], g.data_ptr(), loss.data_ptr(), s))
            step += 1
            B._check(L.redsea_mlp_adam(net.p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(),
                                       step, lr, 0.9, 0.999, 1e-8, s))
            tot += float(loss.item()) * xb.shape[0]
        hist.append(tot / nS)
        if log and (ep % 50 == 0 or ep == epochs - 1):
            log("epoch %d loss %.5f" % (ep, hist[-1]))
    return net, hist


# ------------------------------------------------------------------ evaluation

def regret(pred, ms, mask):
    """T(pick) / T(best) - 1 per shape, pick = argmin of the prediction over
    applicable candidates; exact ties go to the lower candidate index."""
    pred = np.where(mask > 0, pred, np.inf)
    pick = np.argmin(pred, axis=1)
    best = np.min(np.where(mask > 0, ms, np.inf), axis=1)
    got = ms[np.arange(len(ms)), pick]
    return got / best - 1.0, pick


def summary(reg):
    reg = np.asarray(reg)
    return dict(mean=float(reg.mean()), median=float(np.median(reg)),
                p90=float(np.percentile(reg, 90)), max=float(reg.max()))


def paper_rule_pick(n: int, nrhs: int, leaf_ms: Dict[int, Dict[int, float]]):
    """The refinement rule of Sec. V-A as the picker without the network:
    recursive model, native precision, and the leaf halved from the largest
    size while two half-size leaves are faster than one (2 TS(i+1) < TS(i)),
    with TS measured for this right-hand-side count (nearest measured)."""
    cols = sorted(leaf_ms)
    near = min(cols, key=lambda c: abs(math.log(c) - math.log(max(nrhs, 1))))
    t = leaf_ms[near]
    nb = NB_CHOICES[-1]
    for smaller in reversed(NB_CHOICES[:-1]):
        if 2.0 * t[smaller] < t[nb]:
            nb = smaller
        else:
            break
    nb = min(nb, max(32, 1 << (max(n, 1) - 1).bit_length()))
    return 15 * 0 + 3 * NB_CHOICES.index(nb) + 0


def leaf_table(nrhs_grid=(1, 4, 16, 64, 256, 1024, 4096, 8192), reps=5, seed=99):
    """TS(nb): measured time of one leaf-sized solve (order nb) per
    right-hand-side count, for the paper's refinement rule."""
    out = {}
    for k in nrhs_grid:
        row = {}
        for nb in NB_CHOICES:
            idx = 3 * NB_CHOICES.index(nb)  # recursive, this nb, native
            row[nb] = _tune_one(0, nb, k, idx, seed, reps)
        out[k] = row
    return out


def gemm_table(mks=(32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384),
               ns=(1, 4, 16, 64, 256, 1024, 4096, 16384), reps=5):
    """Milliseconds of the FP64 product update C -= A X (M = K = mk, N = n) on
    the library's default tiles, and the launch latency (a 16 x 16 x 16
    product, 200 back to back), for the analytic model's gemm term."""
    import torch
    entries = []
    r = np.random.default_rng(7)
    for mk in mks:
        A = torch.tensor(r.uniform(-1, 1, (mk, mk)), device="cuda").t()
        for n in ns:
            X = torch.tensor(r.uniform(-1, 1, (n, mk)), device="cuda").t()
            C = torch.zeros((mk, n), dtype=torch.float64, device="cuda").t().contiguous().t()
            B.gemm_update(A, X, C)
            times = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                B.gemm_update(A, X, C)
                e1.record()
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
            entries.append({"mk": mk, "n": n, "ms": sorted(times)[len(times) // 2]})
            del X, C
        del A
        torch.cuda.empty_cache()
    a = torch.ones((16, 16), dtype=torch.float64, device="cuda").t()
    c = torch.zeros((16, 16), dtype=torch.float64, device="cuda").t()
    B.gemm_update(a, a, c)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(200):
        B.gemm_update(a, a, c)
    e1.record()
    e1.synchronize()
    return {"entries": entries, "launch_ms": e0.elapsed_time(e1) / 200}


def _tune_one(dtype, n, nrhs, idx, seed, reps):
    cand = (ctypes.c_int * 1)(idx)
    ms = (ctypes.c_double * 1)()
    rc = B.lib().redsea_tune_shape(dtype, n, nrhs, 0.0, ctypes.c_uint64(seed), reps, cand, 1, ms,
                                   None)
    if rc != 0:
        raise B.RedseaError(rc, B.status_string(rc))
    return float(ms[0])


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(prog="python -m paper_2305_19917_amd.picker")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("build-db", help="time all candidates of sampled shapes")
    a.add_argument("--out", required=True)
    a.add_argument("--count", type=int, default=100)
    a.add_argument("--seed", type=int, default=0)
    a.add_argument("--first", type=int, default=0)
    a.add_argument("--reps", type=int, default=2)
    a.add_argument("--max-seconds", type=float, default=0.0)
    b = sub.add_parser("leaf-table", help="leaf times for the paper's refinement rule")
    b.add_argument("--out", required=True)
    g = sub.add_parser("gemm-table", help="product times for the paper's analytic model")
    g.add_argument("--out", required=True)
    c = sub.add_parser("train", help="train the network on a database")
    c.add_argument("--db", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--epochs", type=int, default=400)
    c.add_argument("--seed", type=int, default=0)
    d = sub.add_parser("evaluate", help="regret on held-out shapes")
    d.add_argument("--db", required=True)
    d.add_argument("--weights", required=True)
    d.add_argument("--leaf-table", default=None)
    d.add_argument("--gemm-table", default=None)
    d.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "build-db":
        shapes = sample_shapes(args.first + args.count, args.seed)[args.first:]
        t0 = time.time()
        for i in range(len(shapes)):
            # stop cleanly before the time budget ends; a later run resumes
            if args.max_seconds > 0 and time.time() - t0 > args.max_seconds:
                print("budget reached after %d shapes" % i, flush=True)
                break
            build_db(args.out, shapes[i:i + 1], seed0=1000 * args.seed + args.first + i,
                     reps=args.reps,
                     log=lambda m, i=i: print("[%d] %s" % (args.first + i, m), flush=True))
    elif args.cmd == "leaf-table":
        tab = leaf_table()
        json.dump({str(k): {str(nb): v for nb, v in row.items()} for k, row in tab.items()},
                  open(args.out, "w"), indent=1)
        print(json.dumps(tab))
    elif args.cmd == "gemm-table":
        tab = gemm_table()
        json.dump(tab, open(args.out, "w"), indent=1)
        print(json.dumps(tab))
    elif args.cmd == "train":
        recs, X, T, mask, ms = load_db(args.db, training=True)
        net, hist = train(X, T, mask, epochs=args.epochs, seed=args.seed, log=print)
        net.save(args.out)
        pred = net.predict(X)
        reg, _ = regret(pred, ms, mask)
        print(json.dumps({"train_shapes": len(recs), "final_loss": hist[-1],
                          "train_regret": summary(reg)}))
    elif args.cmd == "evaluate":
        recs, X, T, mask, ms = load_db(args.db)
        net = Net.load(args.weights)
        pred = net.predict(X)
        reg, pick = regret(pred, ms, mask)
        res = {"heldout_shapes": len(recs), "mlp_regret": summary(reg),
               "mlp_total_ms": float(ms[np.arange(len(ms)), pick].sum()),
               "best_total_ms": float(np.min(np.where(mask > 0, ms, np.inf), axis=1).sum())}
        fixed = 3 * NB_CHOICES.index(256)  # the library default: recursive, nb 256, native
        res["fixed_default_total_ms"] = float(ms[:, fixed].sum())
        if args.leaf_table:
            tab = {int(k): {int(nb): v for nb, v in row.items()}
                   for k, row in json.load(open(args.leaf_table)).items()}
            bp = np.array([paper_rule_pick(r["n"], r["nrhs"], tab) for r in recs])
            breg = ms[np.arange(len(ms)), bp] / np.min(np.where(mask > 0, ms, np.inf), axis=1) - 1
            res["paper_rule_regret"] = summary(breg)
            res["paper_rule_total_ms"] = float(ms[np.arange(len(ms)), bp].sum())
            res["mlp_gain_over_paper_rule"] = res["paper_rule_total_ms"] / res["mlp_total_ms"]
            if args.gemm_table:
                from . import costmodel
                cm = costmodel.load(json.load(open(args.leaf_table)), json.load(open(args.gemm_table)))
                ap = np.array([costmodel.pick(r["n"], r["nrhs"], cm) for r in recs])
                areg = ms[np.arange(len(ms)), ap] / np.min(np.where(mask > 0, ms, np.inf), axis=1) - 1
                res["analytic_model_regret"] = summary(areg)
                res["analytic_model_total_ms"] = float(ms[np.arange(len(ms)), ap].sum())
                res["mlp_gain_over_analytic_model"] = res["analytic_model_total_ms"] / res["mlp_total_ms"]
        print(json.dumps(res, indent=1))
        if args.out:
            json.dump(res, open(args.out, "w"), indent=1)


if __name__ == "__main__":
    main()
