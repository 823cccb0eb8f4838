"""GPU parity of redsea_trsm (called through the C-ABI) against the CPU oracle.

Bars (as fixed for this library):
* FP64: normwise backward error <= 1e-14 * order, measured with the oracle's
  compensated residual;
* FP32: <= 5e-6 * order, measured in FP64 on the FP32-rounded data;
* integer-exact and diagonal systems: bitwise;
* upper-transposed storage of L equals lower storage bitwise;
* run-to-run bitwise determinism.
"""
import itertools
import sys

import numpy as np
import pytest

import oracle
import paper_2305_19917_amd as rs
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FLAGS = list(itertools.product([0, 1], [0, 1], [0, 1], [0, 1]))
VARIANTS = ["recursive", "iterative", "blocked"]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_solve(A, B, side=0, uplo=0, trans=0, diag=0, alpha=1.0, variant="auto", nb=0,
              dtype=np.float64):
    dA = rs.fortran_tensor(np.asarray(A, dtype=dtype))
    dB = rs.fortran_tensor(np.asarray(B, dtype=dtype))
    rs.trsm(dA, dB, side=side, uplo=uplo, trans=trans, diag=diag, alpha=alpha, variant=variant,
            nb=nb)
    torch.cuda.synchronize()
    return dB.cpu().numpy().astype(np.float64)


def _stored(L, uplo):
    """A matrix whose stored triangle (uplo) holds L or L^T, the other NaN."""
    k = L.shape[0]
    A = np.array(L if uplo == 0 else L.T, order="F")
    mask = np.triu(np.ones((k, k), bool), 1) if uplo == 0 else np.tril(np.ones((k, k), bool), -1)
    A[mask] = np.nan
    return A


def _shape(side, k, nrhs):
    return (k, nrhs) if side == 0 else (nrhs, k)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("nb", [16, 32, 64, 128, 256, 512])
def test_config0_all_variants(variant, nb):
    n, nrhs = 512, 64
    _say("config0", variant, nb)
    L = synth.dominant_lower(n, (0, 0, 0))
    B = synth.rhs_normal(n, nrhs, (0, 0, 1))
    X = gpu_solve(L, B, variant=variant, nb=nb)
    eta = oracle.backward_error(0, 0, 0, 0, 1.0, L, B, X)
    assert eta <= 1e-14 * n, eta
    Xo = oracle.trsm_plain(0, 0, 0, 0, 1.0, L, B)
    assert oracle.forward_error(X, Xo) <= 1e-12


@pytest.mark.parametrize("side,uplo,trans,diag", FLAGS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_integer_exact_all_flags(side, uplo, trans, diag, dtype):
    for k, nrhs, nb in [(37, 5, 16), (200, 70, 64), (300, 33, 128), (300, 9, 256), (429, 20, 512)]:
        m, n = _shape(side, k, nrhs)
        _say("intexact", side, uplo, trans, diag, k, nrhs, nb, dtype.__name__)
        A, B, Xt = synth.integer_exact(m, n, (5, k, nrhs), side, uplo, trans, diag)
        for variant in VARIANTS:
            X = gpu_solve(A, B, side, uplo, trans, diag, variant=variant, nb=nb, dtype=dtype)
            assert np.array_equal(X, Xt), (variant, k, nrhs)


@pytest.mark.parametrize("nb", [256, 512])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_two_wave_leaf_ragged(nb, dtype):
    """Leaves of 256 rows run the two-wave leaf kernel (alternate 16-row
    blocks per wave); nb = 512 splits its blocks into such leaves.  The
    orders leave a leaf partly occupied (one wave's blocks only, ragged last
    block) and span several leaves; the column counts leave partial column
    groups."""
    bar = 1e-14 if dtype == np.float64 else 5e-6
    for k, nrhs in [(100, 45), (256, 16), (257, 3), (300, 17), (429, 33), (512, 64), (700, 1),
                    (1100, 70)]:
        _say("two-wave leaf", nb, dtype.__name__, k, nrhs)
        L = synth.dominant_lower(k, (15, k, 0)).astype(dtype)
        B = synth.rhs_normal(k, nrhs, (15, k, 1)).astype(dtype)
        for variant in VARIANTS:
            X = gpu_solve(L, B, variant=variant, nb=nb, dtype=dtype)
            eta = oracle.backward_error(0, 0, 0, 0, 1.0, L.astype(np.float64),
                                        B.astype(np.float64), X)
            assert eta <= bar * k, (k, nrhs, variant, eta)


@pytest.mark.parametrize("side,uplo,trans,diag", FLAGS)
def test_dominant_all_flags(side, uplo, trans, diag):
    k, nrhs = 333, 45
    L = synth.unit_lower(k, (6, k, 0)) if diag else synth.dominant_lower(k, (6, k, 0))
    A = _stored(L, uplo)
    B = synth.rhs_normal(*_shape(side, k, nrhs), key=(6, k, 1))
    for alpha, variant, nb in [(1.0, "recursive", 64), (-0.5, "iterative", 32),
                               (2.0, "blocked", 64), (1.0, "recursive", 256)]:
        _say("dominant", side, uplo, trans, diag, alpha, variant, nb)
        X = gpu_solve(A, B, side, uplo, trans, diag, alpha, variant=variant, nb=nb)
        assert np.all(np.isfinite(X))
        eta = oracle.backward_error(side, uplo, trans, diag, alpha, A, B, X)
        assert eta <= 1e-14 * k, (alpha, variant, eta)


@pytest.mark.parametrize("variant,nb", [("recursive", 64), ("iterative", 32), ("blocked", 64)])
def test_upper_transposed_equals_lower_bitwise(variant, nb):
    k, nrhs = 700, 130
    L = synth.dominant_lower(k, (7, 0, 0))
    B = synth.rhs_normal(k, nrhs, (7, 0, 1))
    X1 = gpu_solve(L, B, 0, 0, 0, 0, variant=variant, nb=nb)
    X2 = gpu_solve(synth.upper_of(L), B, 0, 1, 1, 0, variant=variant, nb=nb)
    assert np.array_equal(X1, X2)


def test_diagonal_is_one_division_bitwise():
    for side in (0, 1):
        k, nrhs = 150, 37
        A = synth.diagonal(k, (8, 0, 0))
        B = synth.rhs_normal(*_shape(side, k, nrhs), key=(8, 0, 1))
        d = np.diag(A)
        expect = B / d[:, None] if side == 0 else B / d[None, :]
        for variant in VARIANTS:
            X = gpu_solve(A, B, side, 0, 0, 0, variant=variant, nb=32)
            assert np.array_equal(X, expect)


def test_alpha_zero_and_identity():
    k, nrhs = 100, 20
    A = np.full((k, k), np.nan, order="F")
    B = synth.rhs_normal(k, nrhs, (9, 0, 1))
    assert np.array_equal(gpu_solve(A, B, alpha=0.0), np.zeros((k, nrhs)))
    I = np.asfortranarray(np.eye(k))
    assert np.array_equal(gpu_solve(I, B, alpha=-0.75), -0.75 * B)


def test_empty_inputs():
    dA = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    dB = torch.zeros((0, 5), dtype=torch.float64, device="cuda")
    assert rs.lib().redsea_trsm(0, 0, 0, 0, 0, 0, 5, 1.0, dA.data_ptr(), 1, dB.data_ptr(), 1,
                                None, None) == 0
    assert rs.lib().redsea_trsm(0, 0, 0, 0, 0, 5, 0, 1.0, dA.data_ptr(), 5, dB.data_ptr(), 5,
                                None, None) == 0


@pytest.mark.parametrize("k,nrhs", [(1, 1), (2, 1), (17, 3), (65, 129), (1000, 77), (1025, 1)])
def test_ragged_shapes(k, nrhs):
    L = synth.dominant_lower(k, (10, k, 0))
    B = synth.rhs_normal(k, nrhs, (10, k, 1))
    for variant, nb in [("recursive", 64), ("iterative", 16), ("blocked", 128)]:
        _say("ragged", k, nrhs, variant, nb)
        X = gpu_solve(L, B, variant=variant, nb=nb)
        assert oracle.backward_error(0, 0, 0, 0, 1.0, L, B, X) <= 1e-14 * max(k, 1)


def test_padded_leading_dimensions():
    k, nrhs, lda, ldb = 130, 40, 141, 137
    L = synth.dominant_lower(k, (11, 0, 0))
    B = synth.rhs_normal(k, nrhs, (11, 0, 1))
    Abig = np.full((lda, k), np.nan, order="F")
    Abig[:k, :k] = L
    Bbig = np.full((ldb, nrhs), 7.0, order="F")
    Bbig[:k] = B
    dA = rs.fortran_tensor(Abig)[:k, :]
    dB = rs.fortran_tensor(Bbig)
    rs.trsm(dA, dB[:k, :], variant="blocked", nb=32)
    torch.cuda.synchronize()
    out = dB.cpu().numpy()
    assert np.all(out[k:] == 7.0)
    assert oracle.backward_error(0, 0, 0, 0, 1.0, L, B, out[:k]) <= 1e-14 * k


@pytest.mark.parametrize("variant", VARIANTS)
def test_fp32_backward_error(variant):
    k, nrhs = 600, 50
    L = synth.dominant_lower(k, (12, 0, 0)).astype(np.float32)
    B = synth.rhs_normal(k, nrhs, (12, 0, 1)).astype(np.float32)
    X = gpu_solve(L, B, variant=variant, nb=64, dtype=np.float32)
    eta = oracle.backward_error(0, 0, 0, 0, 1.0, L.astype(np.float64), B.astype(np.float64), X)
    assert eta <= 5e-6 * k, eta


def test_run_to_run_bitwise():
    k, nrhs = 900, 200
    L = synth.dominant_lower(k, (13, 0, 0))
    B = synth.rhs_normal(k, nrhs, (13, 0, 1))
    for variant in VARIANTS:
        X1 = gpu_solve(L, B, variant=variant, nb=64)
        X2 = gpu_solve(L, B, variant=variant, nb=64)
        assert np.array_equal(X1, X2)


def _sampled_check(A, dB_solved, B_host, cols, uplo=0, trans=0, diag=0, bound=None):
    k = A.shape[0]
    Xs = dB_solved[:, cols].cpu().numpy()
    Bs = np.asfortranarray(B_host[:, cols])
    eta = oracle.backward_error(0, uplo, trans, diag, 1.0, A, Bs, Xs)
    assert eta <= (bound or 1e-14 * k), eta
    Xo = oracle.trsm_plain(0, uplo, trans, diag, 1.0, A, Bs)
    assert oracle.forward_error(Xs, Xo) <= 1e-10
    return eta


def test_full_size_n8192_sampled_columns():
    """The benchmark's workload (n = nrhs = 8192, FP64, lower, no transpose,
    non-unit) in the benchmark's launch configuration, checked on sampled
    columns, which the oracle can solve one at a time."""
    n = nrhs = 8192
    _say("full-size 8192x8192")
    L = synth.dominant_lower(n, (1, 0, 0))
    B = synth.rhs_normal(n, nrhs, (1, 0, 1))
    dA = rs.fortran_tensor(L)
    dB = rs.fortran_tensor(B)
    rs.trsm(dA, dB)
    torch.cuda.synchronize()
    cols = [0, 1, 63, 64, 4095, 4096, 8190, 8191]
    _sampled_check(L, dB, B, cols)


@pytest.mark.parametrize("kind", ["upper_trans", "unit"])
def test_thin_n8192_nrhs1024_sampled(kind):
    n, nrhs = 8192, 1024
    _say("thin", kind)
    if kind == "upper_trans":
        L = synth.dominant_lower(n, (1, 1, 0))
        A, uplo, trans, diag = synth.upper_of(L), 1, 1, 0
    else:
        A, uplo, trans, diag = synth.unit_lower(n, (1, 2, 0)), 0, 0, 1
    B = synth.rhs_normal(n, nrhs, (1, 1, 1))
    dA = rs.fortran_tensor(A)
    dB = rs.fortran_tensor(B)
    rs.trsm(dA, dB, uplo=uplo, trans=trans, diag=diag)
    torch.cuda.synchronize()
    _sampled_check(A, dB, B, [0, 5, 511, 1023], uplo, trans, diag)


@pytest.mark.parametrize("groups", ["2", "3", "4"])
def test_column_groups_on_streams_bitwise(groups, monkeypatch):
    """Solving column groups concurrently on helper streams changes no bit:
    every column's arithmetic is the same sequence of operations."""
    k, nrhs = 1000, 1500
    L = synth.dominant_lower(k, (14, 0, 0))
    B = synth.rhs_normal(k, nrhs, (14, 0, 1))
    for variant, nb in [("recursive", 64), ("blocked", 128)]:
        monkeypatch.setenv("REDSEA_STREAMS", "1")
        X1 = gpu_solve(L, B, variant=variant, nb=nb)
        monkeypatch.setenv("REDSEA_STREAMS", groups)
        X2 = gpu_solve(L, B, variant=variant, nb=nb)
        assert np.array_equal(X1, X2), (variant, groups)
    # the right side splits rows of B into groups
    Br = synth.rhs_normal(nrhs, k, (14, 0, 2))
    monkeypatch.setenv("REDSEA_STREAMS", "1")
    X1 = gpu_solve(L, Br, side=1, nb=64)
    monkeypatch.setenv("REDSEA_STREAMS", groups)
    X2 = gpu_solve(L, Br, side=1, nb=64)
    assert np.array_equal(X1, X2)


@pytest.mark.parametrize("k,nb", [(4096, 32), (6000, 32), (8192, 64)])
def test_blocked_rounds_split_over_launches(k, nb):
    """r = ceil(k / nb) >= 128 puts more blocks in a blocked round than one
    grouped launch carries (48), so each round is split over launches."""
    nrhs = 48
    _say("blocked split", k, nb)
    assert -(-k // nb) // 2 > 48
    L = synth.dominant_lower(k, (21, k, 0))
    B = synth.rhs_normal(k, nrhs, (21, k, 1))
    X = gpu_solve(L, B, variant="blocked", nb=nb)
    eta = oracle.backward_error(0, 0, 0, 0, 1.0, L, B, X)
    assert eta <= 1e-14 * k, eta
    assert oracle.forward_error(X, oracle.trsm_plain(0, 0, 0, 0, 1.0, L, B)) <= 1e-10


def test_two_streams_concurrently_match_serial_bitwise():
    """Two different solves in flight at once on two streams (each stream has
    its own workspace) give exactly the bits of the same solves run one after
    the other; the second stream's workspace grows while the first works."""
    shapes = [(3000, 700, (22, 0)), (4100, 900, (22, 1))]
    sysd = []
    for k, nrhs, key in shapes:
        L = synth.dominant_lower(k, key + (0,))
        B = synth.rhs_normal(k, nrhs, key + (1,))
        sysd.append((rs.fortran_tensor(L), rs.fortran_tensor(B)))
    serial = []
    for dL, dB0 in sysd:
        dB = dB0.clone()
        rs.trsm(dL, dB, variant="recursive", nb=256)
        torch.cuda.synchronize()
        serial.append(dB.cpu().numpy())
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        outs = [dB0.clone() for _, dB0 in sysd]
        torch.cuda.synchronize()
        for (dL, _), dB, st in zip(sysd, outs, streams):
            rs.trsm(dL, dB, variant="recursive", nb=256, stream=st)
        torch.cuda.synchronize()
        for o, ref in zip(outs, serial):
            assert np.array_equal(o.cpu().numpy(), ref), rep
        streams.reverse()


def test_graph_capture_is_refused_not_dangling():
    """redsea_trsm on a stream under graph capture returns
    REDSEA_ERR_UNSUPPORTED before launching anything; the library keeps
    working afterwards."""
    k, nrhs = 300, 20
    L = synth.dominant_lower(k, (23, 0, 0))
    B = synth.rhs_normal(k, nrhs, (23, 0, 1))
    dL, dB = rs.fortran_tensor(L), rs.fortran_tensor(B)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    code = None
    with torch.cuda.graph(g, stream=s):
        try:
            rs.trsm(dL, dB, variant="recursive", nb=128, stream=s)
        except rs.RedseaError as e:
            code = e.code
    torch.cuda.synchronize()
    assert code == 5
    X = gpu_solve(L, B, variant="recursive", nb=128)
    assert oracle.backward_error(0, 0, 0, 0, 1.0, L, B, X) <= 1e-14 * k


@pytest.mark.parametrize("k,nrhs,nb", [(8192, 64, 256), (3000, 500, 256), (2048, 333, 128),
                                       (1000, 100, 64)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_lookahead_changes_no_bit(k, nrhs, nb, dtype, monkeypatch):
    """Look-ahead (the rows of a product beyond the next leaf, or the blocks
    of a blocked round that the next leaf does not read, updated on a helper
    stream while that leaf runs) gives exactly the bits of the sequential
    order."""
    L = synth.dominant_lower(k, (24, k, 0))
    B = synth.rhs_normal(k, nrhs, (24, k, 1))
    monkeypatch.setenv("REDSEA_THIN", "0")  # the split schedules, whatever the width
    for variant in ("recursive", "iterative", "blocked"):
        monkeypatch.setenv("REDSEA_LOOKAHEAD", "0")
        X0 = gpu_solve(L, B, variant=variant, nb=nb, dtype=dtype)
        monkeypatch.setenv("REDSEA_LOOKAHEAD", "1")
        X1 = gpu_solve(L, B, variant=variant, nb=nb, dtype=dtype)
        assert np.array_equal(X0, X1), (variant, dtype)
