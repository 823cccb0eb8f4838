"""GPU product update C := C - op(A) op(X) (redsea_gemm_update) on every tile
configuration and storage layout, against an FP64 CPU product.

Bar: |C_gpu - C_ref| <= 2 K u (|C| + |A||X|) elementwise (the standard
dot-product error bound with a margin), and bitwise on integer data whose
partial sums are exact."""
import numpy as np
import pytest

import paper_2305_19917_amd as rs
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U64, U32 = 2.0 ** -53, 2.0 ** -24
TILES = list(range(18))


def _run(A, X, C, transa, transx, tile, dtype):
    # stored forms: op(A) is M x K; with transa the stored A is K x M
    dA = rs.fortran_tensor((A.T if transa else A).astype(dtype))
    dX = rs.fortran_tensor((X.T if transx else X).astype(dtype))
    dC = rs.fortran_tensor((C.T if transx else C).astype(dtype))
    rs.gemm_update(dA, dX, dC, transa=transa, transx=transx, tile=tile)
    torch.cuda.synchronize()
    out = dC.cpu().numpy().astype(np.float64)
    return out.T if transx else out


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("transa,transx", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_update_random(tile, transa, transx):
    for (M, N, K) in [(1, 1, 1), (37, 129, 5), (200, 300, 150), (64, 64, 64), (130, 70, 300)]:
        r = synth.rng((30, M, N + K))
        A = r.standard_normal((M, K))
        X = r.standard_normal((K, N))
        C = r.standard_normal((M, N))
        got = _run(A, X, C, transa, transx, tile, np.float64)
        ref = C - A @ X
        bound = 2 * K * U64 * (np.abs(C) + np.abs(A) @ np.abs(X))
        assert np.all(np.abs(got - ref) <= bound), (M, N, K)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_update_integer_exact(tile, dtype):
    M, N, K = 150, 90, 77
    r = synth.rng((31, 0, 0))
    A = r.integers(-4, 5, (M, K)).astype(np.float64)
    X = r.integers(-4, 5, (K, N)).astype(np.float64)
    C = r.integers(-100, 100, (M, N)).astype(np.float64)
    for transa, transx in [(0, 0), (1, 1)]:
        got = _run(A, X, C, transa, transx, tile, dtype)
        assert np.array_equal(got, C - A @ X)


@pytest.mark.parametrize("transa,transx", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_direct_lds_tiles_match_register_staged(transa, transx):
    # Tiles 11-17 stage operands with direct-to-LDS loads; on shapes they
    # accept they run the same MFMA sequence in the same k order as the
    # register-staged tile 5, so the results agree bit for bit.  Shapes span
    # several tiles with ragged tails in every dimension (all even, as the
    # direct path requires).
    # odd shapes take the 4-byte-load variant of the same kernels
    for (M, N, K) in [(520, 390, 266), (256, 128, 16), (2, 2, 2), (258, 130, 18), (768, 256, 1024),
                      (521, 391, 267), (37, 129, 5), (255, 131, 17), (1, 1, 1)]:
        r = synth.rng((33, M, N + K))
        A = r.standard_normal((M, K))
        X = r.standard_normal((K, N))
        C = r.standard_normal((M, N))
        want = _run(A, X, C, transa, transx, 5, np.float64)
        for fast in range(11, 18):
            got = _run(A, X, C, transa, transx, fast, np.float64)
            assert np.array_equal(got, want), (M, N, K, fast)
        ref = C - A @ X
        bound = 2 * K * U64 * (np.abs(C) + np.abs(A) @ np.abs(X))
        assert np.all(np.abs(got - ref) <= bound), (M, N, K)


@pytest.mark.parametrize("transa,transx", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_direct_lds_odd_leading_dimensions(transa, transx):
    # Operands as column blocks of larger arrays with odd leading dimensions
    # and odd offsets (8-byte aligned only): the direct path loads them with
    # 4-byte accesses and must still agree bit for bit with tile 5.
    M, N, K = 300, 200, 150
    r = synth.rng((34, transa, transx))
    A = r.standard_normal((M, K))
    X = r.standard_normal((K, N))
    C = r.standard_normal((M, N))

    def padded(mat, extra):
        big = np.full((mat.shape[0] + extra, mat.shape[1] + 1), np.nan, order="F")
        big[1:1 + mat.shape[0], 1:] = mat
        t = rs.fortran_tensor(big)
        return t[1:1 + mat.shape[0], 1:]

    outs = []
    for tile in (5, 11, 12, 13, 14, 15, 16, 17):
        dA = padded(A.T if transa else A, 3)
        dX = padded(X.T if transx else X, 5)
        dC = padded(C.T if transx else C, 7)
        rs.gemm_update(dA, dX, dC, transa=transa, transx=transx, tile=tile)
        torch.cuda.synchronize()
        out = dC.cpu().numpy()
        outs.append(out.T if transx else out)
    for tile, out in zip((11, 12, 13, 14, 15, 16, 17), outs[1:]):
        assert np.array_equal(out, outs[0]), tile
    ref = C - A @ X
    assert np.all(np.abs(outs[0] - ref) <= 2 * K * U64 * (np.abs(C) + np.abs(A) @ np.abs(X)))


def test_update_fp32_bound():
    M, N, K = 257, 190, 333
    r = synth.rng((32, 0, 0))
    A = r.standard_normal((M, K)).astype(np.float32).astype(np.float64)
    X = r.standard_normal((K, N)).astype(np.float32).astype(np.float64)
    C = r.standard_normal((M, N)).astype(np.float32).astype(np.float64)
    for tile in TILES:
        got = _run(A, X, C, 0, 0, tile, np.float32)
        ref = C - A @ X
        bound = 2 * (K + 1) * U32 * (np.abs(C) + np.abs(A) @ np.abs(X))
        assert np.all(np.abs(got - ref) <= bound), tile


def test_update_leaves_outside_untouched():
    M, N, K, ld = 50, 40, 30, 64
    r = synth.rng((33, 0, 0))
    A = r.standard_normal((M, K))
    X = r.standard_normal((K, N))
    Cbig = np.full((ld, N), 9.0, order="F")
    Cbig[:M] = r.standard_normal((M, N))
    dA, dX, dC = rs.fortran_tensor(A), rs.fortran_tensor(X), rs.fortran_tensor(Cbig)
    for tile in TILES:
        rs.gemm_update(dA, dX, dC[:M, :], tile=tile)
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    assert np.all(out[M:] == 9.0)


def test_mfma_peak_probe():
    # The diagnostic MFMA-only probe reports a positive operation count and a
    # rate in the range of the matrix cores (FP32 about twice FP64); bad
    # arguments are rejected before any launch.
    L = rs.lib()
    out = torch.empty(4096 * 256, dtype=torch.float64, device="cuda")
    assert L.redsea_mfma_peak(0, 0, out.data_ptr(), out.numel(), None) == -1
    assert L.redsea_mfma_peak(7, 16, out.data_ptr(), out.numel(), None) == -1
    assert L.redsea_mfma_peak(0, 16, out.data_ptr(), 100, None) == -3
    f64 = rs.mfma_peak("f64", iters=512, reps=3)
    f32 = rs.mfma_peak("f32", iters=512, reps=3)
    assert 10.0 < f64 < 100.0, f64
    assert f32 > 1.5 * f64, (f32, f64)


def _round_bf16(x):
    """FP32 -> BF16 by round-to-nearest-even on the bit pattern (finite
    inputs), returned as float64 values."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _run_bf16(A, X, C, transa, transx):
    """A holds BF16 values; X and C are FP32."""
    dA = rs.fortran_tensor((A.T if transa else A).astype(np.float32)).to(torch.bfloat16)
    dA = dA.t().contiguous().t()  # keep column-major storage after the cast
    dX = rs.fortran_tensor((X.T if transx else X).astype(np.float32))
    dC = rs.fortran_tensor((C.T if transx else C).astype(np.float32))
    rs.gemm_update(dA, dX, dC, transa=transa, transx=transx)
    torch.cuda.synchronize()
    out = dC.cpu().numpy().astype(np.float64)
    return out.T if transx else out


def test_bf16_rounding_helper():
    # ties go to even, and values already in BF16 are fixed points
    one = np.float32(1.0).view(np.uint32)
    half_ulp = np.array([one + 0x8000, one + 0x18000], np.uint32).view(np.float32)
    got = _round_bf16(half_ulp)
    assert got[0] == 1.0 and got[1] == 1.0 + 2.0 ** -6
    v = np.array([0.5, -3.0, 2.0 ** -20, 1.0 + 2.0 ** -7], np.float32)
    assert np.array_equal(_round_bf16(v), v.astype(np.float64))


@pytest.mark.parametrize("transa,transx", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_bf16_product_elementwise(transa, transx):
    """C := C - A RN_bf16(X) with FP32 accumulation, checked element by element
    against an FP64 product of the same BF16 operands (exact products) within
    the FP32 accumulation bound (K + 1) u32 (|C| + |A||X|)."""
    # with transa (A stored k-contiguous), transx off and K a multiple of 8 the
    # direct-to-LDS kernel runs; the other shapes and layouts take the
    # register-staged kernel
    for (M, N, K) in [(1, 1, 1), (37, 129, 5), (128, 128, 32), (200, 300, 150), (130, 70, 301),
                      (515, 260, 1030), (515, 260, 1024), (130, 70, 304), (256, 300, 64),
                      (1000, 1000, 2048), (3, 700, 8)]:
        r = synth.rng((34, M, N + K))
        A = _round_bf16(r.standard_normal((M, K)))
        X = r.standard_normal((K, N)).astype(np.float32).astype(np.float64)
        C = r.standard_normal((M, N)).astype(np.float32).astype(np.float64)
        got = _run_bf16(A, X, C, transa, transx)
        Xb = _round_bf16(X)
        ref = C - A @ Xb
        bound = (K + 1) * U32 * (np.abs(C) + np.abs(A) @ np.abs(Xb))
        err = np.abs(got - ref)
        assert np.all(err <= bound), (M, N, K, float(np.max(err / np.maximum(bound, 1e-300))))
        # rounding X matters: the unrounded product is farther away somewhere
        if K >= 32:
            assert np.max(np.abs(got - (C - A @ X))) > np.max(err)


def test_bf16_product_integer_exact():
    """Small integers are exact in BF16 and every FP32 partial sum is exact:
    the result must equal the integer product bitwise."""
    M, N, K = 300, 170, 257
    r = synth.rng((35, 0, 0))
    A = r.integers(-8, 9, (M, K)).astype(np.float64)
    X = r.integers(-8, 9, (K, N)).astype(np.float64)
    C = r.integers(-1000, 1000, (M, N)).astype(np.float64)
    for transa, transx in [(0, 0), (1, 0), (0, 1), (1, 1)]:
        assert np.array_equal(_run_bf16(A, X, C, transa, transx), C - A @ X)
