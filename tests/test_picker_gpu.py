"""The picker network's HIP kernels against the FP64 CPU reference, a
memorisation test, and (when the committed timing data are present) the
regret of the trained picker on held-out shapes."""
import json
import os
import sys

import numpy as np
import pytest

import paper_2305_19917_amd as rs
from paper_2305_19917_amd import picker
from oracle import mlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2305_19917_amd", "data")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


def test_forward_grad_adam_match_cpu_reference():
    L = rs.lib()
    r = np.random.default_rng(60)
    p = r.normal(0, 0.3, mlp.count()).astype(np.float32)
    X = r.normal(0, 1, (300, 4)).astype(np.float32)
    T = r.normal(0, 1, (300, 45)).astype(np.float32)
    mask = (r.uniform(size=(300, 45)) < 0.7).astype(np.float32)
    dp, dX, dT, dM = _dev(p), _dev(X), _dev(T), _dev(mask)
    Y = torch.empty((300, 45), dtype=torch.float32, device="cuda")
    assert L.redsea_mlp_forward(dp.data_ptr(), dX.data_ptr(), 300, Y.data_ptr(), None) == 0
    g = torch.empty_like(dp)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    assert L.redsea_mlp_grad(dp.data_ptr(), dX.data_ptr(), dT.data_ptr(), dM.data_ptr(), 300,
                             g.data_ptr(), loss.data_ptr(), None) == 0
    torch.cuda.synchronize()
    Yr, _ = mlp.forward(p.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(Y.cpu().numpy() - Yr)) <= 1e-4 * np.max(np.abs(Yr))
    gr = mlp.grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                  mask.astype(np.float64))
    gg = g.cpu().numpy().astype(np.float64)
    # per parameter tensor relative error
    off = 0
    for size in (256, 64, 4096, 64, 2880, 45):
        a, b = gg[off:off + size], gr[off:off + size]
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b), off
        off += size
    assert abs(loss.item() - mlp.loss(p.astype(np.float64), X, T, mask)) <= 1e-5
    # Adam step
    m = torch.zeros_like(dp)
    v = torch.zeros_like(dp)
    assert L.redsea_mlp_adam(dp.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), 1, 1e-3, 0.9,
                             0.999, 1e-8, None) == 0
    torch.cuda.synchronize()
    pr, _, _ = mlp.adam(p.astype(np.float64), gg, np.zeros(p.size), np.zeros(p.size), 1, lr=1e-3)
    assert np.max(np.abs(dp.cpu().numpy() - pr)) <= 1e-6


def test_deterministic_gradient():
    L = rs.lib()
    r = np.random.default_rng(61)
    p, X = _dev(r.normal(0, 0.3, mlp.count())), _dev(r.normal(0, 1, (500, 4)))
    T, M = _dev(r.normal(0, 1, (500, 45))), _dev(np.ones((500, 45)))
    outs = []
    for _ in range(2):
        g = torch.empty_like(p)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        L.redsea_mlp_grad(p.data_ptr(), X.data_ptr(), T.data_ptr(), M.data_ptr(), 500,
                          g.data_ptr(), loss.data_ptr(), None)
        torch.cuda.synchronize()
        outs.append(g.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_memorisation_drives_regret_to_zero():
    """64 shapes with synthetic candidate times that vary smoothly with the
    shape (each candidate's relative cost is a different smooth function of
    log n and log nrhs): training on them alone must pick the fastest
    candidate of (almost) every one."""
    r = np.random.default_rng(62)
    n = np.exp(r.uniform(np.log(64), np.log(16384), 64)).astype(int)
    k = np.exp(r.uniform(0, np.log(8192), 64)).astype(int)
    X = np.array([picker.features(a, b, 0, 4.5 * a) for a, b in zip(n, k)])
    base = np.log(1e-3 * (n.astype(float) ** 2 * k) / 4e7 + 0.05)
    x1 = (np.log2(n) - 10) / 4
    x2 = (np.log2(k) - 6.5) / 6.5
    a, b, ph = r.normal(0, 1.5, 45), r.normal(0, 1.5, 45), r.uniform(0, 6.28, 45)
    rel = 0.5 * np.sin(np.outer(x1, a) + np.outer(x2, b) + ph)
    ms = np.exp(base[:, None] + rel)
    mask = np.ones_like(ms)
    net, hist = picker.train(X, np.log(ms), mask, epochs=3000, batch=64, lr=3e-3)
    reg, _ = picker.regret(net.predict(X), ms, mask)
    _say("memorisation: final loss %.4g, regret %s" % (hist[-1], picker.summary(reg)))
    assert hist[-1] < hist[0] / 50
    assert np.mean(reg) < 0.01


@pytest.mark.skipif(not os.path.exists(os.path.join(DATA, "tune_heldout.jsonl")),
                    reason="timing data not generated")
def test_heldout_regret_and_gain():
    w = os.path.join(os.path.dirname(rs.LIB_PATH), "picker_weights.txt")
    recs, X, T, mask, ms = picker.load_db(os.path.join(DATA, "tune_heldout.jsonl"))
    net = picker.Net.load(w)
    reg, pick = picker.regret(net.predict(X), ms, mask)
    s = picker.summary(reg)
    _say("held-out regret", s)
    best = np.min(np.where(mask > 0, ms, np.inf), axis=1).sum()
    assert ms[np.arange(len(ms)), pick].sum() <= 1.25 * best
    # the library's host-side picker agrees with the GPU forward on most shapes
    agree = 0
    for r_, p_ in zip(recs, pick):
        c = rs.lib().redsea_pick(r_["dtype"], r_["n"], r_["nrhs"], r_["kappa"], None)
        agree += int(c == p_)
    assert agree >= 0.95 * len(recs)
