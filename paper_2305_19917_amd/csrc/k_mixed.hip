// Kernels of the mixed-precision solve with FP64 iterative refinement:
// precision conversions, per-right-hand-side norms, the FP64 correction
// update, and the BF16 product update (BF16 operands, FP32 accumulation) on
// the gfx950 v_mfma_f32_16x16x32_bf16 matrix instruction.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "mixed.h"
#include "tiles.h"

namespace redsea {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v8f __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ conversions

// dst (k x k, ld = k) := stored triangle of src (uplo) rounded to nearest
// even; the other triangle is zero and a unit diagonal is one (neither is
// read by the solver).  BF16 goes FP64 -> FP32 -> BF16, rounding to nearest
// even at each step.
template <typename TO>
__global__ __launch_bounds__(256) void convert_tri_kernel(const double* __restrict__ src,
                                                          int64_t lda, int64_t k, int uplo,
                                                          int unit, TO* __restrict__ dst) {
    const int64_t total = k * k;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx % k, j = idx / k;
        float v = 0.f;
        if (i == j) v = unit ? 1.f : (float)src[i + j * lda];
        else if ((uplo == 0 && i > j) || (uplo == 1 && i < j)) v = (float)src[i + j * lda];
        dst[idx] = (TO)v;
    }
}

// dst (k rows, row-major, ld ldd >= k) := M rounded FP64 -> FP32 -> BF16
// (nearest even at each step), where M = A (op_trans = 0) or A^T (op_trans =
// 1) restricted to the stored triangle of A (uplo), with a unit diagonal as
// one; the rest of each row, padding columns included, is zero.  A row of M
// is then contiguous, which is the k-contiguous operand layout of the BF16
// product.  64 x 64 tiles pass through LDS so that both the reads of A and
// the writes of dst are coalesced whichever way M lies in A.
__global__ __launch_bounds__(256) void convert_rows_bf16_kernel(const double* __restrict__ a,
                                                                int64_t lda, int64_t k, int uplo,
                                                                int unit, int op_trans,
                                                                __bf16* __restrict__ dst,
                                                                int64_t ldd) {
    __shared__ float t[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // (i, j) of M is element (r, c) = (i, j) or (j, i) of A; stored iff in uplo's triangle
    auto m_at = [&](int64_t i, int64_t j) -> float {
        if (i >= k || j >= k) return 0.f;
        if (i == j) return unit ? 1.f : (float)a[i + i * lda];
        const int64_t r = op_trans ? j : i, c = op_trans ? i : j;
        const bool stored = uplo == 0 ? r > c : r < c;
        return stored ? (float)a[r + c * lda] : 0.f;
    };
    for (int q = ty; q < 64; q += 4) {
        // consecutive threads along A's contiguous index
        if (!op_trans) t[tx][q] = m_at(i0 + tx, j0 + q);  // A(i, j): i contiguous
        else t[q][tx] = m_at(i0 + q, j0 + tx);            // A(j, i): j contiguous
    }
    __syncthreads();
    for (int q = ty; q < 64; q += 4) {
        const int64_t i = i0 + q, j = j0 + tx;
        if (i < k && j < ldd) dst[j + i * ldd] = (__bf16)t[q][tx];
    }
}

// B32 := RN32(scale_r * B) over an m x n matrix; scale_r is the inverse
// norm of the right-hand side the entry belongs to (its column for the left
// side, its row for the right side), or one when inv is null.
__global__ __launch_bounds__(256) void scale_to_f32_kernel(const double* __restrict__ src,
                                                           int64_t ld, int64_t m, int64_t n,
                                                           const double* __restrict__ inv,
                                                           int rhs_rows, double alpha,
                                                           float* __restrict__ dst, int64_t ldd) {
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx % m, j = idx / m;
        double v = alpha * src[i + j * ld];
        if (inv) v *= inv[rhs_rows ? i : j];
        dst[i + j * ldd] = (float)v;
    }
}

// X := (scale ? X : 0) + s_r * D with s_r the norm of the entry's right-hand
// side (one when s is null), in FP64.
__global__ __launch_bounds__(256) void update_kernel(double* __restrict__ x, int64_t ldx,
                                                     int64_t m, int64_t n,
                                                     const float* __restrict__ d, int64_t ldd,
                                                     const double* __restrict__ s, int rhs_rows,
                                                     int accumulate) {
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx % m, j = idx / m;
        double v = (double)d[i + j * ldd];
        if (s) v *= s[rhs_rows ? i : j];
        double* p = x + i + j * ldx;
        *p = accumulate ? *p + v : v;
    }
}

// dst := alpha * src (m x n, FP64).
__global__ __launch_bounds__(256) void copy_scaled_kernel(const double* __restrict__ src,
                                                          int64_t lds, int64_t m, int64_t n,
                                                          double alpha, double* __restrict__ dst,
                                                          int64_t ldd) {
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx % m, j = idx / m;
        const double v = src[i + j * lds];
        dst[i + j * ldd] = alpha == 1.0 ? v : alpha * v;
    }
}

// ------------------------------------------------------------------ norms

// out[r] = max |entry| over right-hand side r (max is order independent, so
// the result does not depend on the reduction order).  Columns (left side):
// one workgroup per column, LDS reduction.  Rows (right side): one thread per
// row, consecutive threads on consecutive rows.
__global__ __launch_bounds__(256) void colmax_kernel(const double* __restrict__ a, int64_t ld,
                                                     int64_t m, int64_t n, double scale,
                                                     double* __restrict__ out) {
    __shared__ double red[256];
    const int64_t j = blockIdx.x;
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 256) {
        const double v = fabs(scale * a[i + j * ld]);
        mx = (v > mx || v != v) ? v : mx;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}

__global__ __launch_bounds__(256) void rowmax_kernel(const double* __restrict__ a, int64_t ld,
                                                     int64_t m, int64_t n, double scale,
                                                     double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double mx = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double v = fabs(scale * a[i + j * ld]);
        mx = (v > mx || v != v) ? v : mx;
    }
    out[i] = mx;
}

// Row sums of |T| for ||T||_inf (T the canonical triangle, unit diagonal as
// 1).  Storage not transposed: a row of T runs across columns, so a
// workgroup takes 64 rows (one per lane, coalesced reads down each column)
// and its eight waves split the columns the triangle covers; the partial sums
// are added in a fixed order.  Transposed: a row is contiguous in storage and
// one wave sums it, lanes striding along it, then a fixed shuffle tree.
__global__ __launch_bounds__(512) void tri_rowsum_rows_kernel(const double* __restrict__ a,
                                                              int64_t lda, int64_t k, int lower,
                                                              int unit, double* __restrict__ out) {
    __shared__ double part[8][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64, i = r0 + lane;
    const int64_t jlo = lower ? 0 : r0, jhi = lower ? (r0 + 64 < k ? r0 + 64 : k) : k;
    const int64_t per = (jhi - jlo + 7) / 8;
    const int64_t ja = jlo + w * per, jb = ja + per < jhi ? ja + per : jhi;
    auto term = [&](int64_t j) -> double {
        const bool in = lower ? j <= i : j >= i;
        if (!in) return 0.0;
        return (unit && j == i) ? 1.0 : __builtin_fabs(a[i + j * lda]);
    };
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (i < k) {
        int64_t j = ja;
        for (; j + 4 <= jb; j += 4) {
            s0 += term(j);
            s1 += term(j + 1);
            s2 += term(j + 2);
            s3 += term(j + 3);
        }
        for (; j < jb; ++j) s0 += term(j);
    }
    part[w][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (w == 0 && i < k) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) t += part[q][lane];
        out[i] = t;
    }
}

__global__ __launch_bounds__(512) void tri_rowsum_trans_kernel(const double* __restrict__ a,
                                                               int64_t lda, int64_t k, int lower,
                                                               int unit, double* __restrict__ out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 8 + w;
    if (i >= k) return;  // uniform over the wave
    const int64_t jlo = lower ? 0 : i, jhi = lower ? i + 1 : k;
    const double* row = a + i * lda;  // element (i, j) of T at row[j]
    double s = 0.0;
    for (int64_t j = jlo + lane; j < jhi; j += 64) s += (unit && j == i) ? 1.0 : __builtin_fabs(row[j]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) out[i] = s;
}

// ------------------------------------------------------------------ BF16 product

// C (FP32) -= A (BF16) X (FP32 rounded to BF16 on load), FP32 accumulation.
// 128 x 128 tiles, four waves of 64 x 64, K in stages of 32.  Both operands
// are kept k-contiguous in LDS so each lane reads its eight k values of an
// MFMA operand with one 16-byte load.
constexpr int HB_BM = 128, HB_BN = 128, HB_BK = 32, HB_PAD = 8;

template <bool AT, bool RT>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) __bf16 As[HB_BM][HB_BK + HB_PAD];
    __shared__ __attribute__((aligned(16))) __bf16 Xs[HB_BN][HB_BK + HB_PAD];
    const int64_t tiles_m = (g.M + HB_BM - 1) / HB_BM;
    const int64_t m0 = (blockIdx.x % tiles_m) * HB_BM, n0 = (blockIdx.x / tiles_m) * HB_BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1, gq = lane >> 4, cc = lane & 15;
    const __bf16* a = (const __bf16*)g.a;
    const float* x = (const float*)g.x;
    float* c = (float*)g.c;
    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    const __bf16 zero = (__bf16)0.f;
    for (int64_t k0 = 0; k0 < g.K; k0 += HB_BK) {
        // A tile: BM x BK
#pragma unroll 4
        for (int p = 0; p < HB_BM * HB_BK / 256; ++p) {
            const int idx = p * 256 + tid;
            int mm, kk;
            if (!AT) { mm = idx % HB_BM; kk = idx / HB_BM; }
            else { kk = idx % HB_BK; mm = idx / HB_BK; }
            const int64_t gi = m0 + mm, gk = k0 + kk;
            As[mm][kk] = (gi < g.M && gk < g.K) ? (AT ? a[gk + gi * g.lda] : a[gi + gk * g.lda]) : zero;
        }
#pragma unroll 4
        for (int p = 0; p < HB_BN * HB_BK / 256; ++p) {
            const int idx = p * 256 + tid;
            int jj, kk;
            if (!RT) { kk = idx % HB_BK; jj = idx / HB_BK; }
            else { jj = idx % HB_BN; kk = idx / HB_BN; }
            const int64_t gj = n0 + jj, gk = k0 + kk;
            const float v = (gj < g.N && gk < g.K) ? (RT ? x[gj + gk * g.ldx] : x[gk + gj * g.ldx]) : 0.f;
            Xs[jj][kk] = (__bf16)v;
        }
        __syncthreads();
        v8bf fa[4], fx[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) fa[i] = *(const v8bf*)&As[wm * 64 + i * 16 + cc][8 * gq];
#pragma unroll
        for (int j = 0; j < 4; ++j) fx[j] = *(const v8bf*)&Xs[wn * 64 + j * 16 + cc][8 * gq];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fx[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = m0 + wm * 64 + i * 16 + 4 * gq + r;
                const int64_t gj = n0 + wn * 64 + j * 16 + cc;
                if (gi < g.M && gj < g.N) {
                    float* p = RT ? c + gj + gi * g.ldc : c + gi + gj * g.ldc;
                    *p = *p - acc[i][j][r];
                }
            }
}

// C (FP32) -= A (BF16) X (FP32 rounded to BF16 as it is read), FP32
// accumulation, for operands that are both contiguous along k:
//   A(i, k) = a[k + i*lda]  (row-major BF16, lda % 8 == 0),
//   X(k, j) = x[k + j*ldx]  (column-major FP32, ldx % 4 == 0),
//   C(i, j) = c[i + j*ldc],  K % 8 == 0, a and x 16-byte aligned.
// Both operands go from memory straight into LDS (buffer_load_dwordx4 ... lds:
// 16 bytes per lane, LDS address M0 + 16 lane; a chunk past the operand's
// rows, columns or K is not requested and reads zero), two stages, one
// barrier per k-stage of 32.  In a stage, A is 4 chunks of 8 k per row and X
// 8 chunks of 4 k per column; which chunk a lane fetches is XOR-swizzled
// (A: chunk q of row m at slot 4m + (q ^ (m/4 % 4)); X: chunk q of column j
// at slot 8j + (q ^ (j/2 % 8))) so that the 16 lanes of a fragment read,
// 16 rows (or columns) at one k offset, hit 16 different 16-byte bank
// groups.  Each wave holds a (BM/WM) x (BN/WN) block of 16 x 16
// v_mfma_f32_16x16x32_bf16 accumulators; an X fragment is two 16-byte LDS
// reads converted to BF16 by v_cvt_pk_bf16_f32 (nearest even).
constexpr int HB2_BK = 32;

template <int BM, int BN, int WM, int WN>
struct Bf16Cfg {
    static constexpr int NW = WM * WN, NT = 64 * NW, SM = BM / WM, SN = BN / WN;
    static constexpr int FM = SM / 16, FN = SN / 16;
    static constexpr int A_LOADS = BM * 4 / 64, X_LOADS = BN * 8 / 64;  // 1 KB loads per stage
    static constexpr int A_BYTES = BM * 64, X_BYTES = BN * 128, STAGE = A_BYTES + X_BYTES;
    static_assert(A_LOADS % NW == 0 && X_LOADS % NW == 0, "loads per wave");
    static_assert(SM % 16 == 0 && SN % 16 == 0, "wave tile");
};

typedef __attribute__((address_space(3))) void* lds_ptr_bf_t;
constexpr unsigned kBfOob = 0x7FFFFFF0u;  // byte offset at the record count: reads zero

template <typename D>
__device__ __forceinline__ void bf16_stage(const GemmArgs& g, int64_t m0, int64_t n0, int64_t k0,
                                           char* st, int wave, int lane) {
    const __bf16* pa = (const __bf16*)g.a + k0 + m0 * g.lda;
    const float* px = (const float*)g.x + k0 + n0 * g.ldx;
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc((void*)pa, 0, (int)kBfOob, 0x00020000);
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc((void*)px, 0, (int)kBfOob, 0x00020000);
    const int64_t mlim = g.M - m0, nlim = g.N - n0, klim = g.K - k0;
#pragma unroll
    for (int u = 0; u < D::A_LOADS / D::NW; ++u) {
        const int q = u * D::NW + wave;
        const int slot = 64 * q + lane, m = slot >> 2, kq = (slot & 3) ^ ((m >> 2) & 3);
        const unsigned voff = (m < mlim && 8 * kq < klim) ? (unsigned)((8 * kq + m * g.lda) * 2) : kBfOob;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr_bf_t)(st + q * 1024), 16, voff, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < D::X_LOADS / D::NW; ++u) {
        const int q = u * D::NW + wave;
        const int slot = 64 * q + lane, j = slot >> 3, kq = (slot & 7) ^ ((j >> 1) & 7);
        const unsigned voff = (j < nlim && 4 * kq < klim) ? (unsigned)((4 * kq + j * g.ldx) * 4) : kBfOob;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_ptr_bf_t)(st + D::A_BYTES + q * 1024), 16,
                                                 voff, 0, 0, 0);
    }
}

template <int BM, int BN, int WM, int WN, int MINB>
__global__ __launch_bounds__(64 * WM * WN, MINB) void gemm_bf16_dma_kernel(GemmArgs g) {
    typedef Bf16Cfg<BM, BN, WM, WN> D;
    __shared__ __attribute__((aligned(1024))) char smem[2 * D::STAGE];
    const int64_t tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
    int64_t tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int lane = threadIdx.x & 63, gq = lane >> 4, cc = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WM, wn = wave / WM;
    // LDS byte offsets of this lane's fragments (A: row, chunk gq; X: column, chunks 2gq, 2gq+1)
    int oa[D::FM], ox0[D::FN], ox1[D::FN];
#pragma unroll
    for (int i = 0; i < D::FM; ++i) {
        const int m = wm * D::SM + 16 * i + cc;
        oa[i] = (4 * m + (gq ^ ((m >> 2) & 3))) * 16;
    }
#pragma unroll
    for (int j = 0; j < D::FN; ++j) {
        const int col = wn * D::SN + 16 * j + cc;
        ox0[j] = D::A_BYTES + (8 * col + ((2 * gq) ^ ((col >> 1) & 7))) * 16;
        ox1[j] = D::A_BYTES + (8 * col + ((2 * gq + 1) ^ ((col >> 1) & 7))) * 16;
    }
    v4f acc[D::FM][D::FN];
#pragma unroll
    for (int i = 0; i < D::FM; ++i)
#pragma unroll
        for (int j = 0; j < D::FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t ke = (g.K + HB2_BK - 1) / HB2_BK;
    if (ke > 0) bf16_stage<D>(g, m0, n0, 0, smem, wave, lane);
    __syncthreads();
    for (int64_t kt = 0; kt < ke; ++kt) {
        const char* st = smem + (kt & 1) * D::STAGE;
        if (kt + 1 < ke) bf16_stage<D>(g, m0, n0, (kt + 1) * HB2_BK, smem + ((kt + 1) & 1) * D::STAGE, wave, lane);
        v8bf fa[D::FM], fx[D::FN];
#pragma unroll
        for (int i = 0; i < D::FM; ++i) fa[i] = *(const v8bf*)(st + oa[i]);
#pragma unroll
        for (int j = 0; j < D::FN; ++j) {
            const v4f lo = *(const v4f*)(st + ox0[j]), hi = *(const v4f*)(st + ox1[j]);
            const v8f f = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            fx[j] = __builtin_convertvector(f, v8bf);
        }
#pragma unroll
        for (int i = 0; i < D::FM; ++i)
#pragma unroll
            for (int j = 0; j < D::FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fx[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // C -= acc: lane holds rows 4 gq .. 4 gq + 3 of one column, contiguous in C
    float* c = (float*)g.c;
    const bool vec = ((g.ldc & 3) == 0) && (((uintptr_t)c & 15) == 0);
#pragma unroll
    for (int i = 0; i < D::FM; ++i)
#pragma unroll
        for (int j = 0; j < D::FN; ++j) {
            const int64_t gi = m0 + wm * D::SM + 16 * i + 4 * gq;
            const int64_t gj = n0 + wn * D::SN + 16 * j + cc;
            if (gj >= g.N) continue;
            float* p = c + gi + gj * g.ldc;
            if (vec && gi + 3 < g.M) {
                v4f cv = *(v4f*)p;
                cv -= acc[i][j];
                *(v4f*)p = cv;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (gi + r < g.M) p[r] = p[r] - acc[i][j][r];
            }
        }
}

template <int BM, int BN, int WM, int WN, int MINB>
bool bf16_dma_ok(const GemmArgs& g) {
    if ((g.K & 7) || (g.lda & 7) || (g.ldx & 3)) return false;
    if (((uintptr_t)g.a | (uintptr_t)g.x) & 15) return false;
    const int64_t lim = (int64_t)1 << 30;  // byte span of one stage within a buffer offset
    return (HB2_BK + (BM - 1) * g.lda) * 2 < lim && (HB2_BK + (BN - 1) * g.ldx) * 4 < lim;
}

template <int BM, int BN, int WM, int WN, int MINB>
hipError_t bf16_dma_launch(const GemmArgs& g, hipStream_t s) {
    const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_bf16_dma_kernel<BM, BN, WM, WN, MINB>), dim3((unsigned)tiles),
                       dim3(64 * WM * WN), 0, s, g);
    return hipGetLastError();
}

unsigned grid_for(int64_t total) {
    int64_t b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_convert_tri(int to_bf16, const double* a, int64_t lda, int64_t k, int uplo,
                              bool unit, void* dst, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    if (to_bf16)
        hipLaunchKernelGGL(convert_tri_kernel<__bf16>, dim3(grid_for(k * k)), dim3(256), 0, s, a,
                           lda, k, uplo, unit ? 1 : 0, (__bf16*)dst);
    else
        hipLaunchKernelGGL(convert_tri_kernel<float>, dim3(grid_for(k * k)), dim3(256), 0, s, a,
                           lda, k, uplo, unit ? 1 : 0, (float*)dst);
    return hipGetLastError();
}

hipError_t launch_scale_to_f32(const double* src, int64_t ld, int64_t m, int64_t n,
                               const double* inv, bool rhs_rows, double alpha, float* dst,
                               int64_t ldd, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_to_f32_kernel, dim3(grid_for(m * n)), dim3(256), 0, s, src, ld, m, n,
                       inv, rhs_rows ? 1 : 0, alpha, dst, ldd);
    return hipGetLastError();
}

hipError_t launch_update(double* x, int64_t ldx, int64_t m, int64_t n, const float* d, int64_t ldd,
                         const double* scale, bool rhs_rows, bool accumulate, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(update_kernel, dim3(grid_for(m * n)), dim3(256), 0, s, x, ldx, m, n, d, ldd,
                       scale, rhs_rows ? 1 : 0, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_copy_scaled(const double* src, int64_t lds, int64_t m, int64_t n, double alpha,
                              double* dst, int64_t ldd, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_scaled_kernel, dim3(grid_for(m * n)), dim3(256), 0, s, src, lds, m, n,
                       alpha, dst, ldd);
    return hipGetLastError();
}

hipError_t launch_rhs_max(const double* a, int64_t ld, int64_t m, int64_t n, bool rhs_rows,
                          double scale, double* out, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (!rhs_rows)
        hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)n), dim3(256), 0, s, a, ld, m, n, scale,
                           out);
    else
        hipLaunchKernelGGL(rowmax_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, ld,
                           m, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_tri_rowsum(const double* a, int64_t lda, int64_t k, bool a_trans, bool lower,
                             bool unit, double* out, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    if (!a_trans)
        hipLaunchKernelGGL(tri_rowsum_rows_kernel, dim3((unsigned)((k + 63) / 64)), dim3(512), 0, s,
                           a, lda, k, lower ? 1 : 0, unit ? 1 : 0, out);
    else
        hipLaunchKernelGGL(tri_rowsum_trans_kernel, dim3((unsigned)((k + 7) / 8)), dim3(512), 0, s,
                           a, lda, k, lower ? 1 : 0, unit ? 1 : 0, out);
    return hipGetLastError();
}

hipError_t launch_convert_rows_bf16(const double* a, int64_t lda, int64_t k, int uplo, bool unit,
                                   bool op_trans, void* dst, int64_t ldd, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    dim3 grid((unsigned)((ldd + 63) / 64), (unsigned)((k + 63) / 64));
    hipLaunchKernelGGL(convert_rows_bf16_kernel, grid, dim3(256), 0, s, a, lda, k, uplo,
                       unit ? 1 : 0, op_trans ? 1 : 0, (__bf16*)dst, ldd);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16(bool a_trans, bool rhs_trans, const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
    // 256 x 128 tiles on eight waves; short products (the updates near the
    // leaves, where 256-row tiles would leave most CUs idle) on 64 x 64 tiles
    // of four waves
    if (a_trans && !rhs_trans && g.M <= 512 && bf16_dma_ok<64, 64, 2, 2, 4>(g))
        return bf16_dma_launch<64, 64, 2, 2, 4>(g, s);
    if (a_trans && !rhs_trans && bf16_dma_ok<256, 128, 4, 2, 2>(g))
        return bf16_dma_launch<256, 128, 4, 2, 2>(g, s);
    const int64_t tiles = ((g.M + HB_BM - 1) / HB_BM) * ((g.N + HB_BN - 1) / HB_BN);
    if (!a_trans && !rhs_trans)
        hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), dim3((unsigned)tiles), dim3(256), 0, s, g);
    else if (a_trans && !rhs_trans)
        hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), dim3((unsigned)tiles), dim3(256), 0, s, g);
    else if (!a_trans && rhs_trans)
        hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), dim3((unsigned)tiles), dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), dim3((unsigned)tiles), dim3(256), 0, s, g);
    return hipGetLastError();
}

}  // namespace redsea
