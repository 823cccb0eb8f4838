"""redsea_potrf (Cholesky, built on the library's solve and matrix-core
products) against the CPU oracle.

Bars:
* integer factors (A = L0 L0^T formed exactly, L0 with diagonal in {1, 2}):
  every partial sum is an integer and every division and square root exact,
  so the factor is L0 bitwise, FP64 and FP32;
* random positive definite matrices: the componentwise backward error
  max |A - F F^T| / (|F||F|^T) over the stored triangle within 4 gamma_{n+1}
  (Higham Thm 10.3 bounds any ordering of the factorisation's sums by
  gamma_{n+1}; the factor of four covers the solve's row scaling and the
  blocked sums), and elementwise |F - F_oracle| <= 4 (n + 1) u max|F_oracle|
  on these well-conditioned matrices (u of the data type);
* info equals the oracle's, and the columns before it are the factor;
* the other strict triangle (NaN here) is neither read nor written;
* scaling by powers of two commutes with the factorisation bitwise.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2305_19917_amd as rs
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U = {np.float64: 2.0 ** -53, np.float32: 2.0 ** -24}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _other(n, uplo):
    return np.triu_indices(n, 1) if uplo == 0 else np.tril_indices(n, -1)


def _mine(F, uplo):
    return np.tril(F) if uplo == 0 else np.triu(F)


def _gpu_potrf(A, uplo, nb=0, dtype=np.float64, ld_pad=0):
    """Factor A on the GPU (other triangle set to NaN first); returns the
    whole stored matrix (float64) and info."""
    n = A.shape[0]
    An = np.array(A, dtype=np.float64, order="F")
    An[_other(n, uplo)] = np.nan
    host = np.full((n + ld_pad, n), -7.0)
    host[:n, :n] = An
    dA = rs.fortran_tensor(host.astype(dtype))
    view = dA[:n, :n]
    info = rs.potrf(view, uplo="L" if uplo == 0 else "U", nb=nb)
    torch.cuda.synchronize()
    out = dA.cpu().numpy().astype(np.float64)
    assert np.all(out[n:, :] == -7.0), "rows past n (padding) were written"
    return out[:n, :n], int(info.cpu().item())


@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("n,nb", [(1, 0), (2, 32), (33, 32), (128, 0), (129, 64), (300, 32),
                                  (300, 128), (517, 64), (1100, 0)])
def test_integer_factor_bitwise_f64(uplo, n, nb):
    _say("potrf integer f64", uplo, n, nb)
    A, L0 = synth.integer_spd(n, (120, n, uplo))
    F, info = _gpu_potrf(A, uplo, nb)
    assert info == 0
    assert np.array_equal(_mine(F, uplo), L0 if uplo == 0 else L0.T)
    assert np.all(np.isnan(F[_other(n, uplo)]))


@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("n,nb", [(65, 64), (300, 0), (600, 32)])
def test_integer_factor_bitwise_f32(uplo, n, nb):
    _say("potrf integer f32", uplo, n, nb)
    A, L0 = synth.integer_spd(n, (121, n, uplo))
    F, info = _gpu_potrf(A, uplo, nb, dtype=np.float32)
    assert info == 0
    assert np.array_equal(_mine(F, uplo), L0 if uplo == 0 else L0.T)
    assert np.all(np.isnan(F[_other(n, uplo)]))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("n", [7, 255, 1000])
def test_random_spd_against_oracle(dtype, uplo, n):
    _say("potrf random", dtype.__name__, uplo, n)
    A = synth.spd_dominant(n, (122, n, uplo)).astype(dtype).astype(np.float64)
    F, info = _gpu_potrf(A, uplo, dtype=dtype)
    assert info == 0
    Fo, info_o = oracle.potrf(uplo, A)
    assert info_o == 0
    u = U[dtype]
    mine = np.tril_indices(n) if uplo == 0 else np.triu_indices(n)
    assert np.max(np.abs(F[mine] - Fo[mine])) <= 4 * (n + 1) * u * np.max(np.abs(Fo[mine]))
    Fm = np.where(np.isnan(F), 0.0, F)
    eta = oracle.chol_backward_error(uplo, A, Fm)
    assert eta <= 4 * (n + 1) * u, eta


@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("k", [0, 5, 63, 64, 200, 299])
def test_info_and_leading_columns(uplo, k):
    _say("potrf info", uplo, k)
    n = 300
    A, L0 = synth.integer_spd(n, (123, k, uplo))
    A[k, k] -= L0[k, k] ** 2 + 1.0  # pivot of column k becomes -1
    F, info = _gpu_potrf(A, uplo, nb=64)
    Fo, info_o = oracle.potrf(uplo, A)
    assert info_o == k + 1
    assert info == info_o
    got = _mine(F, uplo) if uplo == 0 else _mine(F, uplo).T
    assert np.array_equal(got[:, :k], L0[:, :k])
    assert np.all(np.isnan(F[_other(n, uplo)]))


def test_nan_pivot_sets_info():
    n = 200
    A = synth.spd_dominant(n, (124, 0, 0))
    A[150, 150] = np.nan
    _, info = _gpu_potrf(A, 0, nb=64)
    assert info == oracle.potrf(0, A)[1] == 151


@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("n,pad", [(301, 13), (700, 1)])
def test_leading_dimension_larger_than_n(uplo, n, pad):
    _say("potrf ld", uplo, n, pad)
    A, L0 = synth.integer_spd(n, (125, n, uplo))
    F, info = _gpu_potrf(A, uplo, nb=0, ld_pad=pad)
    assert info == 0
    assert np.array_equal(_mine(F, uplo), L0 if uplo == 0 else L0.T)


def test_power_of_two_scaling_commutes():
    n = 400
    A = synth.spd_dominant(n, (126, 0, 0))
    D = np.ldexp(1.0, synth.rng((126, 0, 1)).integers(-30, 31, size=n))
    F, _ = _gpu_potrf(A, 0, nb=64)
    Fs, _ = _gpu_potrf(A * D[:, None] * D[None, :], 0, nb=64)
    assert np.array_equal(np.tril(Fs), np.tril(F) * D[:, None])


def test_empty_matrix_clears_info():
    info = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    A = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    rs.potrf(A[:0, :0], info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0


def test_trace_counts_leaves_and_updates():
    n, nb = 1000, 128  # splits 512 (4 leaves) + 488 (256 + 232 -> 128, 128, 128, 104)
    A = synth.spd_dominant(n, (127, 0, 0))
    dA = rs.fortran_tensor(A)
    rs.trace_begin()
    info = rs.potrf(dA, nb=nb)
    torch.cuda.synchronize()
    tr = rs.trace_end()
    assert int(info.item()) == 0
    leaves = tr["chol_leaf"][0]
    assert leaves == 8
    assert tr["syrk"][0] == leaves - 1
    assert tr["chol_leaf"][2] == pytest.approx(7 * 128 ** 3 / 3 + 104 ** 3 / 3)


def test_large_order_sampled():
    n = 8192
    _say("potrf large", n)
    A = synth.spd_dominant(n, (128, 0, 0))
    dA = rs.fortran_tensor(A)
    info = rs.potrf(dA)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    F = np.tril(dA.cpu().numpy())
    r = synth.rng((128, 0, 1))
    i = r.integers(0, n, size=3000)
    j = (r.random(3000) * (i + 1)).astype(np.int64)
    pairs = np.stack([i, np.minimum(j, i)], axis=1)
    pairs = np.concatenate([pairs, np.array([[n - 1, n - 1], [n - 1, 0], [4096, 4095]])])
    eta = oracle.chol_backward_error(0, A, F, pairs)
    assert eta <= 4 * (n + 1) * U[np.float64], eta
    # the last diagonal entries against the oracle's definition, one column
    # at a time: l_jj^2 = a_jj - sum_k l_jk^2 with the GPU's own row j
    for jj in (n - 1, 5000, 127):
        piv = A[jj, jj] - np.dot(F[jj, :jj], F[jj, :jj])
        assert abs(F[jj, jj] - np.sqrt(piv)) <= 4 * (n + 1) * U[np.float64] * F[jj, jj]


def test_graph_capture_is_refused_before_anything_is_enqueued():
    """Above the leaf order the panel solves need the per-stream buffer, so a
    stream under graph capture is refused (REDSEA_ERR_UNSUPPORTED) before any
    launch, info included; the library keeps working afterwards."""
    n = 300
    A, L0 = synth.integer_spd(n, (129, 0, 0))
    dA = rs.fortran_tensor(A)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    code = None
    with torch.cuda.graph(g, stream=s):
        try:
            rs.potrf(dA, info=info, stream=s)
        except rs.RedseaError as e:
            code = e.code
    torch.cuda.synchronize()
    assert code == 5
    F, inf = _gpu_potrf(A, 0)
    assert inf == 0 and np.array_equal(np.tril(F), L0)
