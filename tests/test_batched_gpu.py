"""Batched persistent solve (redsea_trsm_batched and the plan API) against the
oracle, system by system; graph capture and replay of a plan."""
import sys

import numpy as np
import pytest

import oracle
import paper_2305_19917_amd as rs
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _make(count, key, n_range=(32, 1024), nrhs_range=(1, 256), side=0, uplo=0, trans=0, diag=0):
    ns, ks = synth.batch_shapes(count, key, n_range, nrhs_range)
    As, Bs = [], []
    for i, (n, k) in enumerate(zip(ns, ks)):
        L = synth.unit_lower(int(n), (3, i, 0)) if diag else synth.dominant_lower(int(n), (3, i, 0))
        A = np.asfortranarray(L if uplo == 0 else L.T)
        B = synth.rhs_normal(*((int(n), int(k)) if side == 0 else (int(k), int(n))), key=(3, i, 1))
        As.append(A)
        Bs.append(B)
    return As, Bs


def _run(As, Bs, dtype=np.float64, **kw):
    dAs = [rs.fortran_tensor(a.astype(dtype)) for a in As]
    dBs = [rs.fortran_tensor(b.astype(dtype)) for b in Bs]
    info = torch.full((len(Bs),), -7, dtype=torch.int32, device="cuda")
    rs.trsm_batched(dAs, dBs, info, **kw)
    torch.cuda.synchronize()
    return [b.cpu().numpy().astype(np.float64) for b in dBs], info.cpu().numpy()


@pytest.mark.parametrize("dtype,bound", [(np.float64, 1e-14), (np.float32, 5e-6)])
def test_config3_shapes_per_system(dtype, bound):
    As, Bs = _make(300, (3, 0, 2))
    Xs, info = _run(As, Bs, dtype)
    assert np.all(info == 0)
    worst = 0.0
    for A, B, X in zip(As, Bs, Xs):
        A2, B2 = A.astype(dtype).astype(np.float64), B.astype(dtype).astype(np.float64)
        eta = oracle.backward_error(0, 0, 0, 0, 1.0, A2, B2, X)
        worst = max(worst, eta / A.shape[0])
        assert eta <= bound * A.shape[0], (A.shape, B.shape, eta)
    _say("batched", dtype.__name__, "worst eta/n", worst)


@pytest.mark.parametrize("side,uplo,trans,diag", [(0, 0, 0, 0), (0, 1, 1, 0), (0, 1, 0, 1),
                                                  (0, 0, 1, 0), (1, 0, 0, 0), (1, 1, 1, 1)])
def test_integer_exact_flags(side, uplo, trans, diag):
    As, Bs, Xt = [], [], []
    shapes = [(1, 1), (5, 3), (16, 16), (17, 1), (100, 33), (257, 40), (1000, 7)]
    for i, (k, r) in enumerate(shapes):
        m, n = (k, r) if side == 0 else (r, k)
        A, B, X = synth.integer_exact(m, n, (21, i, side), side, uplo, trans, diag)
        As.append(A)
        Bs.append(B)
        Xt.append(X)
    for dtype in (np.float64, np.float32):
        Xs, info = _run(As, Bs, dtype, side=side, uplo=uplo, trans=trans, diag=diag)
        assert np.all(info == 0)
        for X, T in zip(Xs, Xt):
            assert np.array_equal(X, T)


def test_big_systems_and_empty_and_alpha():
    As, Bs = _make(20, (3, 1, 2), n_range=(32, 300))
    As.append(synth.dominant_lower(1500, (3, 99, 0)))    # above the panel limit
    Bs.append(synth.rhs_normal(1500, 20, (3, 99, 1)))
    As.append(synth.dominant_lower(10, (3, 98, 0)))      # no right-hand sides
    Bs.append(np.zeros((10, 0), order="F"))
    Xs, info = _run(As, Bs, alpha=-2.0)
    assert np.all(info == 0)
    for A, B, X in zip(As, Bs, Xs):
        if B.size:
            assert oracle.backward_error(0, 0, 0, 0, -2.0, A, B, X) <= 1e-14 * A.shape[0]


def test_diagonal_systems_divide_exactly():
    # Every row is one division x_i = b_i / d_i.  The batched solver divides
    # through a reciprocal and two Markstein corrections, redoing a block in
    # IEEE arithmetic when an operand leaves the fast path's range; the result
    # must be the IEEE quotient in every case: ordinary operands, divisors
    # 2^k with |k| up to 600, numerators from subnormal to 1e305, zeros.
    r = synth.rng((3, 9, 9))
    As, Bs, want = [], [], []
    for sysid in range(5):
        n, k = 70 + 13 * sysid, 5 + sysid
        if sysid in (0, 3, 4):
            d = np.diag(synth.diagonal(n, (3, 9, sysid)))
        else:
            d = np.ldexp(r.uniform(1.0, 2.0, n), r.integers(-600, 601, n)) * r.choice([-1.0, 1.0], n)
        B = r.standard_normal((n, k))
        if sysid in (2, 3):  # no quotient overflows: |b/d| < 2^1018
            top = 300 if sysid == 2 else 1015
            B = B * np.ldexp(1.0, r.integers(-1070, top, (n, k)).astype(np.int64))
        if sysid == 4:
            B[:, ::2] = 0.0
        A = np.full((n, n), np.nan)
        A[np.tril_indices(n, -1)] = 0.0
        A[np.diag_indices(n)] = d
        As.append(np.asfortranarray(A))
        Bs.append(np.asfortranarray(B))
        want.append(B / d[:, None])
    Xs, info = _run(As, Bs)
    assert np.all(info == 0)
    for i, (X, W) in enumerate(zip(Xs, want)):
        assert np.array_equal(X, W), i


def test_nonfinite_system_is_flagged():
    As, Bs = _make(6, (3, 2, 2), n_range=(40, 200), nrhs_range=(2, 20))
    Bs[3] = Bs[3].copy(order="F")
    Bs[3][5, 0] = np.inf
    _, info = _run(As, Bs)
    assert info[3] == 4 and np.all(np.delete(info, 3) == 0)


def test_run_to_run_bitwise_and_graph_replay():
    As, Bs = _make(120, (3, 3, 2))
    dAs = [rs.fortran_tensor(a) for a in As]
    dB0 = [rs.fortran_tensor(b) for b in Bs]
    dBs = [b.clone() for b in dB0]
    dBs = [b.t().contiguous().t() if b.numel() else b for b in dBs]
    info = torch.zeros(len(Bs), dtype=torch.int32, device="cuda")
    plan = rs.BatchPlan(dAs, dBs)
    plan.run(info)
    torch.cuda.synchronize()
    ref = [b.cpu().numpy() for b in dBs]
    # second eager run from restored inputs is bitwise identical
    for b, b0 in zip(dBs, dB0):
        b.copy_(b0)
    plan.run(info)
    torch.cuda.synchronize()
    assert all(np.array_equal(b.cpu().numpy(), r) for b, r in zip(dBs, ref))
    # capture once, replay several times with eager restores in between
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    for b, b0 in zip(dBs, dB0):
        b.copy_(b0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        plan.run(info, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for b, b0 in zip(dBs, dB0):
            b.copy_(b0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert all(np.array_equal(b.cpu().numpy(), r) for b, r in zip(dBs, ref)), rep
        assert int(info.abs().sum().item()) == 0
    plan.close()


def test_graph_replay_with_big_system_survives_larger_solve():
    """A captured plan holding a system above order 1024 owns the memory of
    that system's diagonal blocks: a larger redsea_trsm between replays (which
    regrows the library's stream workspace) leaves every replay bitwise equal
    to the eager run."""
    As, Bs = _make(30, (3, 4, 2), n_range=(32, 400))
    As.append(synth.dominant_lower(1500, (3, 97, 0)))
    Bs.append(synth.rhs_normal(1500, 40, (3, 97, 1)))
    dAs = [rs.fortran_tensor(a) for a in As]
    dB0 = [rs.fortran_tensor(b) for b in Bs]
    dBs = [b.clone() for b in dB0]
    info = torch.zeros(len(Bs), dtype=torch.int32, device="cuda")
    plan = rs.BatchPlan(dAs, dBs, variant="recursive", nb=256)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    plan.run(info, stream=s)
    torch.cuda.synchronize()
    ref = [b.cpu().numpy() for b in dBs]
    assert oracle.backward_error(0, 0, 0, 0, 1.0, As[-1], Bs[-1], ref[-1]) <= 1e-14 * 1500
    g = torch.cuda.CUDAGraph()
    for b, b0 in zip(dBs, dB0):
        b.copy_(b0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        plan.run(info, stream=s)
    torch.cuda.synchronize()
    big_L = rs.fortran_tensor(synth.dominant_lower(4000, (3, 96, 0)))
    for rep in range(3):
        # a larger solve on the same stream regrows its workspace
        big_B = rs.fortran_tensor(synth.rhs_normal(4000, 64 * (rep + 1), (3, 96, 1)))
        with torch.cuda.stream(s):
            rs.trsm(big_L, big_B, variant="recursive", nb=256, stream=s)
        torch.cuda.synchronize()
        for b, b0 in zip(dBs, dB0):
            b.copy_(b0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert all(np.array_equal(b.cpu().numpy(), r) for b, r in zip(dBs, ref)), rep
    plan.close()


def test_alpha_zero_overwrites_nonfinite_with_zero():
    """BLAS semantics: alpha = 0 sets B to zero without reading it, so Inf and
    NaN entries of B become 0, not NaN."""
    As, Bs = _make(8, (3, 5, 2), n_range=(20, 200), nrhs_range=(1, 30))
    for B in Bs:
        B[0, 0] = np.inf
        B[-1, -1] = np.nan
    Xs, info = _run(As, Bs, alpha=0.0)
    assert np.all(info == 0)
    for X in Xs:
        assert np.array_equal(X, np.zeros_like(X))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_every_task_shape_gives_the_same_bits(dtype):
    """The twelve task shapes the tuner chooses from (16 or 32 right-hand
    sides per wave task, operand prefetch depth 1, 2 or 4, 2 or 4 workgroups
    per CU) do the same arithmetic on
    every column, so their results agree bitwise; checked on a batch of
    uneven systems with ragged column counts, also against the oracle."""
    As, Bs = _make(150, (3, 6, 2), n_range=(16, 700), nrhs_range=(1, 100))
    outs = []
    for tile in range(1, 13):
        Xs, info = _run(As, Bs, dtype, tile=tile)
        assert np.all(info == 0), tile
        outs.append(Xs)
    for tile in range(2, 13):
        for i, (a, b) in enumerate(zip(outs[0], outs[tile - 1])):
            assert np.array_equal(a, b), (tile, i)
    bound = 1e-14 if dtype == np.float64 else 5e-6
    for A, B, X in zip(As[:20], Bs[:20], outs[3][:20]):
        A32, B32 = A.astype(dtype).astype(np.float64), B.astype(dtype).astype(np.float64)
        assert oracle.backward_error(0, 0, 0, 0, 1.0, A32, B32, X) <= bound * A.shape[0]


@pytest.mark.parametrize("side,uplo,trans,diag", [(0, 1, 1, 0), (1, 0, 0, 1), (1, 1, 1, 0)])
def test_wide_tasks_all_flags(side, uplo, trans, diag):
    As, Bs = _make(40, (3, 7, side), n_range=(20, 300), nrhs_range=(1, 70), side=side, uplo=uplo,
                   trans=trans, diag=diag)
    X16, i16 = _run(As, Bs, side=side, uplo=uplo, trans=trans, diag=diag, alpha=-0.5, tile=1)
    X32, i32 = _run(As, Bs, side=side, uplo=uplo, trans=trans, diag=diag, alpha=-0.5, tile=12)
    assert np.all(i16 == 0) and np.all(i32 == 0)
    for A, B, a, b in zip(As, Bs, X16, X32):
        assert np.array_equal(a, b)
        assert oracle.backward_error(side, uplo, trans, diag, -0.5, A, B, b) <= 1e-14 * A.shape[0]


def test_tuner_picks_its_fastest_candidate():
    ns, ks = synth.batch_shapes(300, (3, 8, 2))
    best, ms = rs.batched_tune(ns, ks, reps=2)
    _say("batched tuner: best", best, "ms", ["%.3f" % x for x in ms])
    assert 1 <= best <= 12 and all(x > 0 for x in ms)
    assert ms[best - 1] == min(ms) and ms.index(min(ms)) == best - 1
