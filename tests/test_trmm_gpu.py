"""redsea_trmm, C := beta C + alpha op(A) B (or B op(A)), on both methods,
against the oracle's compensated residual: with alpha = -a and B = X the
oracle computes beta C - op(A) (a X) to about one rounding (Dot2), so
   C_ref = oracle.residual_comp(side, uplo, trans, diag, beta, A, C0, -alpha B)
when -alpha B is exact (alpha a power of two here).

Bars:
* matrix-core method: |C - C_ref| <= 2 (k + 2) u (|beta C0| + |alpha| |op(A)| |B|),
  the dot-product error bound with a margin (FP32: u = 2^-24);
* INT8 emulation (Ozaki scheme II): rows of op(A) and columns of B are
  rounded to 53-bit integers relative to their largest entry, the integer
  product is exact, then rounded to FP64, so
  |C - C_ref| <= |alpha| 2^-52 (rowmax_i |op(A)| ||b_j||_1 + colmax_j |B| ||op(A)_i||_1)
                 + 4 u (|C_ref| + |beta C0|),
  far below the FP64 product bound for long rows; small-integer data is exact.
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
U64 = 2.0 ** -53
FLAGS = list(itertools.product([0, 1], [0, 1], [0, 1], [0, 1]))


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _stored(L, uplo):
    k = L.shape[0]
    A = np.array(L if uplo == 0 else L.T, order="F")
    A[np.triu_indices(k, 1) if uplo == 0 else np.tril_indices(k, -1)] = np.nan
    return A


def _gpu_trmm(A, B, C0, side, uplo, trans, diag, alpha, beta, method, dtype=np.float64):
    dA = rs.fortran_tensor(A.astype(dtype))
    dB = rs.fortran_tensor(B.astype(dtype))
    dC = rs.fortran_tensor(C0.astype(dtype))
    rs.trmm(dA, dB, dC, side=side, uplo=uplo, trans=trans, diag=diag, alpha=alpha, beta=beta,
            method=method)
    torch.cuda.synchronize()
    return dC.cpu().numpy().astype(np.float64)


def _ref(A, B, C0, side, uplo, trans, diag, alpha, beta):
    C0z = np.zeros_like(C0) if beta == 0.0 else C0
    return oracle.residual_comp(side, uplo, trans, diag, beta, np.nan_to_num(A, nan=0.0), C0z,
                                -alpha * B)


def _ozaki_bound(A, B, C0, Cref, side, uplo, trans, diag, alpha, beta):
    k = A.shape[0]
    T = np.abs(oracle.op_dense(uplo, trans, diag, np.nan_to_num(A, nan=0.0), k))
    Ab = np.abs(B)
    if side == 0:   # rows of op(A) against columns of B
        rmax = T.max(axis=1)[:, None]
        cmax = Ab.max(axis=0)[None, :]
        e = rmax * Ab.sum(axis=0)[None, :] + cmax * T.sum(axis=1)[:, None]
    else:           # rows of B against columns of op(A)
        rmax = Ab.max(axis=1)[:, None]
        cmax = T.max(axis=0)[None, :]
        e = rmax * T.sum(axis=0)[None, :] + cmax * Ab.sum(axis=1)[:, None]
    return abs(alpha) * 2.0 ** -52 * e + 4 * U64 * (np.abs(Cref) + np.abs(beta * C0))


def _case(side, uplo, trans, diag, k, nrhs, key):
    L = synth.unit_lower(k, key + (0,)) if diag else synth.dominant_lower(k, key + (0,))
    A = _stored(np.nan_to_num(L, nan=0.0) + (np.eye(k) if diag else 0), uplo)
    if diag:
        A[np.diag_indices(k)] = np.nan  # a unit diagonal is never read
    shape = (k, nrhs) if side == 0 else (nrhs, k)
    B = synth.rhs_normal(*shape, key=key + (1,))
    C0 = synth.rhs_normal(*shape, key=key + (2,))
    return A, B, C0


@pytest.mark.parametrize("side,uplo,trans,diag", FLAGS)
def test_trmm_mfma_all_flags(side, uplo, trans, diag):
    for k, nrhs, alpha, beta in [(1, 3, 1.0, 0.0), (37, 20, -1.0, 1.5), (300, 130, 2.0, 0.0),
                                 (515, 64, -0.5, -1.0)]:
        A, B, C0 = _case(side, uplo, trans, diag, k, nrhs, (40, k))
        if beta == 0.0:
            C0 = np.full_like(C0, np.nan)  # beta = 0: C is not read
        got = _gpu_trmm(A, B, C0, side, uplo, trans, diag, alpha, beta, "mfma")
        ref = _ref(A, B, C0, side, uplo, trans, diag, alpha, beta)
        T = np.abs(oracle.op_dense(uplo, trans, diag, np.nan_to_num(A, nan=0.0), k))
        prod = T @ np.abs(B) if side == 0 else np.abs(B) @ T
        b0 = 0.0 if beta == 0.0 else np.abs(beta * C0)
        bound = 2 * (k + 2) * U64 * (b0 + abs(alpha) * prod)
        assert np.all(np.abs(got - ref) <= bound), (k, nrhs, alpha, beta)


def test_trmm_mfma_fp32():
    k, nrhs = 333, 77
    for side, uplo, trans, diag in [(0, 0, 0, 0), (1, 1, 1, 0), (0, 1, 0, 1)]:
        A, B, C0 = _case(side, uplo, trans, diag, k, nrhs, (41, side))
        A32 = A.astype(np.float32).astype(np.float64)
        B32 = B.astype(np.float32).astype(np.float64)
        C32 = C0.astype(np.float32).astype(np.float64)
        got = _gpu_trmm(A32, B32, C32, side, uplo, trans, diag, -1.0, 0.5, "mfma", np.float32)
        ref = _ref(A32, B32, C32, side, uplo, trans, diag, -1.0, 0.5)
        T = np.abs(oracle.op_dense(uplo, trans, diag, np.nan_to_num(A32, nan=0.0), k))
        prod = T @ np.abs(B32) if side == 0 else np.abs(B32) @ T
        bound = 2 * (k + 2) * 2.0 ** -24 * (np.abs(0.5 * C32) + prod)
        assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("side,uplo,trans,diag", FLAGS)
def test_trmm_int8_emulation_all_flags(side, uplo, trans, diag):
    for k, nrhs, alpha, beta in [(1, 3, 1.0, 0.0), (37, 20, -1.0, 1.5), (300, 130, 2.0, 0.0),
                                 (515, 64, -0.5, -1.0), (1000, 17, 1.0, 1.0)]:
        A, B, C0 = _case(side, uplo, trans, diag, k, nrhs, (42, k))
        if beta == 0.0:
            C0 = np.full_like(C0, np.nan)
        got = _gpu_trmm(A, B, C0, side, uplo, trans, diag, alpha, beta, "int8")
        ref = _ref(A, B, C0, side, uplo, trans, diag, alpha, beta)
        C0b = np.zeros_like(C0) if beta == 0.0 else C0
        bound = _ozaki_bound(A, B, C0b, ref, side, uplo, trans, diag, alpha, beta)
        err = np.abs(got - ref)
        assert np.all(err <= bound), (k, nrhs, float(np.max(err / bound)))


def test_trmm_int8_integer_data_is_exact():
    """Small integers are exact after scaling; the emulated product must equal
    the integer product bitwise (so must the matrix-core one)."""
    for side, uplo, trans, diag in [(0, 0, 0, 0), (0, 1, 1, 1), (1, 0, 1, 0), (1, 1, 0, 1)]:
        k, nrhs = 257, 45
        r = synth.rng((43, side, uplo))
        T = np.tril(r.integers(-3, 4, (k, k))).astype(np.float64)
        T[np.diag_indices(k)] = 1.0 if diag else r.choice([-4.0, -2.0, 2.0, 4.0], k)
        A = _stored(T, uplo)
        if diag:
            A[np.diag_indices(k)] = np.nan
        shape = (k, nrhs) if side == 0 else (nrhs, k)
        B = r.integers(-50, 51, shape).astype(np.float64)
        C0 = r.integers(-1000, 1001, shape).astype(np.float64)
        Top = oracle.op_dense(uplo, trans, diag, np.nan_to_num(A, nan=0.0), k)
        want = 3.0 * C0 + (Top @ B if side == 0 else B @ Top)
        for method in ("int8", "mfma"):
            got = _gpu_trmm(A, B, C0, side, uplo, trans, diag, 1.0, 3.0, method)
            assert np.array_equal(got, want), (method, side, uplo, trans, diag)


def test_trmm_int8_nonfinite_and_zero_columns():
    k, nrhs = 200, 6
    A, B, C0 = _case(0, 0, 0, 0, k, nrhs, (44, 0))
    B[:, 2] = 0.0
    B[7, 4] = np.nan
    got = _gpu_trmm(A, B, C0, 0, 0, 0, 0, 1.0, 1.0, "int8")
    assert np.all(np.isnan(got[:, 4]))
    assert np.array_equal(got[:, 2], C0[:, 2])  # zero column: C unchanged
    keep = [0, 1, 3, 5]
    ref = _ref(A, B[:, keep], C0[:, keep], 0, 0, 0, 0, 1.0, 1.0)
    assert np.all(np.abs(got[:, keep] - ref) <= _ozaki_bound(A, B[:, keep], C0[:, keep], ref,
                                                               0, 0, 0, 0, 1.0, 1.0))


def test_trmm_argument_errors():
    L = rs.lib()
    # method 1 is FP64 only; bad method; ldc too small
    assert L.redsea_trmm(1, 0, 0, 0, 0, 4, 3, 1.0, 8, 4, 8, 4, 0.0, 8, 4, 1, None) == -16
    assert L.redsea_trmm(0, 0, 0, 0, 0, 4, 3, 1.0, 8, 4, 8, 4, 0.0, 8, 4, 7, None) == -16
    assert L.redsea_trmm(0, 0, 0, 0, 0, 4, 3, 1.0, 8, 4, 8, 4, 0.0, 8, 3, 0, None) == -15
    assert L.redsea_trmm(0, 0, 0, 0, 0, 0, 3, 1.0, None, 1, None, 1, 0.0, None, 1, 1, None) == 0


def test_trmm_int8_config2_size_sampled_columns():
    """The residual of the mixed-precision workload at its full size (order
    16384, 4096 right-hand sides, kappa_1 ~ 1e4 family) by the INT8 emulation,
    against the oracle's compensated residual on sampled columns, within the
    scheme's bound; the FP64 matrix-core residual for comparison."""
    n, nrhs = 16384, 4096
    _say("config-2 size emulated residual: generating")
    L = synth.kappa_lower(n, 0.009821718891880384, (2, 0, 0))
    B = synth.rhs_normal(n, nrhs, (2, 0, 1))
    dL = rs.fortran_tensor(L)
    dB0 = rs.fortran_tensor(B)
    dX = dB0.clone()
    rs.trsm(dL, dX, variant="recursive", nb=256)  # a solution to take the residual of
    cols = [0, 1, 511, 2048, 4095]
    out = {}
    for method in ("int8", "mfma"):
        dC = dB0.clone()
        rs.trmm(dL, dX, dC, alpha=-1.0, beta=1.0, method=method)
        torch.cuda.synchronize()
        out[method] = dC[:, cols].cpu().numpy()
    Xs = np.asfortranarray(dX[:, cols].cpu().numpy())
    Bs = np.asfortranarray(B[:, cols])
    ref = oracle.residual_comp(0, 0, 0, 0, 1.0, L, Bs, Xs)
    bound = _ozaki_bound(L, Xs, Bs, ref, 0, 0, 0, 0, -1.0, 1.0)
    err = np.abs(out["int8"] - ref)
    _say("int8 residual: max err %.3e, max err/bound %.3e, max |r| %.3e; fp64 max err %.3e"
         % (err.max(), (err / bound).max(), np.abs(ref).max(), np.abs(out["mfma"] - ref).max()))
    assert np.all(err <= bound)
