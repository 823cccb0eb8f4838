// Trailing-update product C -= A X on MFMA matrix cores, gfx950.
//
// This is the "gemm" task the paper offloads to the accelerator (Sec. V-A:
// with many right-hand sides the update of stage 2 of Sec. IV becomes a
// matrix-matrix product; the grey rectangles of Fig. 2-4).  Each workgroup of
// four waves owns a 128 x 128 tile of C; each wave a 64 x 64 quarter held as
// 4 x 4 MFMA accumulators of 16 x 16.  K advances in steps of 16 through a
// double-buffered LDS stage: the next stage's global loads are in flight
// while the current stage feeds the matrix cores.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace redsea {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 16, PAD = 2;
constexpr int NT = 256;

// Per-type MFMA 16x16x4 operations.  For both types lane l supplies
// A[l % 16][l / 16] and X[l / 16][l % 16]; the 16 x 16 result lives in four
// registers per lane whose row index differs between the two instructions.
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row of register r for lane l (column is l % 16)
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T>
struct Smem {
    T a[2][BK][BM + PAD];
    T x[2][BK][BN + PAD];
};

template <typename T, bool AT, bool RT>
__device__ __forceinline__ void load_stage(const GemmArgs& g, int64_t m0, int64_t n0, int64_t k0,
                                           int tid, T (&ra)[BM * BK / NT],
                                           T (&rx)[BN * BK / NT]) {
    const T* a = (const T*)g.a;
    const T* x = (const T*)g.x;
#pragma unroll
    for (int p = 0; p < BM * BK / NT; ++p) {
        const int idx = p * NT + tid;
        int kk, mm;
        if (!AT) { kk = idx / BM; mm = idx % BM; }   // column of A: BM contiguous rows
        else { mm = idx / BK; kk = idx % BK; }       // row of A^T storage: BK contiguous k
        const int64_t gi = m0 + mm, gk = k0 + kk;
        T v = T(0);
        if (gi < g.M && gk < g.K) v = AT ? a[gk + gi * g.lda] : a[gi + gk * g.lda];
        ra[p] = v;
    }
#pragma unroll
    for (int p = 0; p < BN * BK / NT; ++p) {
        const int idx = p * NT + tid;
        int kk, jj;
        if (!RT) { jj = idx / BK; kk = idx % BK; }   // column of X: BK contiguous k
        else { kk = idx / BN; jj = idx % BN; }       // row of X^T storage: BN contiguous j
        const int64_t gj = n0 + jj, gk = k0 + kk;
        T v = T(0);
        if (gj < g.N && gk < g.K) v = RT ? x[gj + gk * g.ldx] : x[gk + gj * g.ldx];
        rx[p] = v;
    }
}

template <typename T, bool AT, bool RT>
__device__ __forceinline__ void store_stage(Smem<T>& sm, int buf, int tid,
                                            const T (&ra)[BM * BK / NT],
                                            const T (&rx)[BN * BK / NT]) {
#pragma unroll
    for (int p = 0; p < BM * BK / NT; ++p) {
        const int idx = p * NT + tid;
        int kk, mm;
        if (!AT) { kk = idx / BM; mm = idx % BM; }
        else { mm = idx / BK; kk = idx % BK; }
        sm.a[buf][kk][mm] = ra[p];
    }
#pragma unroll
    for (int p = 0; p < BN * BK / NT; ++p) {
        const int idx = p * NT + tid;
        int kk, jj;
        if (!RT) { jj = idx / BK; kk = idx % BK; }
        else { kk = idx / BN; jj = idx % BN; }
        sm.x[buf][kk][jj] = rx[p];
    }
}

template <typename T, bool AT, bool RT>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int64_t m0, int64_t n0,
                                          Smem<T>& sm) {
    typedef typename Mfma<T>::acc_t acc_t;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    T ra[BM * BK / NT], rx[BN * BK / NT];
    const int64_t nk = (g.K + BK - 1) / BK;
    load_stage<T, AT, RT>(g, m0, n0, 0, tid, ra, rx);
    store_stage<T, AT, RT>(sm, 0, tid, ra, rx);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int buf = (int)(kt & 1);
        const bool more = kt + 1 < nk;
        if (more) load_stage<T, AT, RT>(g, m0, n0, (kt + 1) * BK, tid, ra, rx);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            T fa[4], fx[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) fa[i] = sm.a[buf][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) fx[j] = sm.x[buf][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::mma(fa[i], fx[j], acc[i][j]);
        }
        if (more) store_stage<T, AT, RT>(sm, buf ^ 1, tid, ra, rx);
        __syncthreads();
    }

    T* c = (T*)g.c;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = m0 + wm * 64 + i * 16 + Mfma<T>::row(lane, r);
                const int64_t gj = n0 + wn * 64 + j * 16 + (lane & 15);
                if (gi < g.M && gj < g.N) {
                    T* p = RT ? c + gj + gi * g.ldc : c + gi + gj * g.ldc;
                    *p = *p - acc[i][j][r];
                }
            }
}

template <typename T, bool AT, bool RT>
__global__ __launch_bounds__(NT) void gemm_kernel(GemmArgs g) {
    __shared__ Smem<T> sm;
    const int64_t tiles_m = (g.M + BM - 1) / BM;
    const int64_t tile = blockIdx.x;
    gemm_tile<T, AT, RT>(g, (tile % tiles_m) * BM, (tile / tiles_m) * BN, sm);
}

template <typename T, bool AT, bool RT>
__global__ __launch_bounds__(NT) void gemm_group_kernel(GemmGroup grp, int64_t tiles_m_max) {
    __shared__ Smem<T> sm;
    const GemmArgs& g = grp.g[blockIdx.y];
    const int64_t tm = blockIdx.x % tiles_m_max, tn = blockIdx.x / tiles_m_max;
    if (tm * BM >= g.M || tn * BN >= g.N) return;  // uniform over the workgroup
    gemm_tile<T, AT, RT>(g, tm * BM, tn * BN, sm);
}

template <typename T, bool AT, bool RT>
hipError_t gemm_launch_t(const GemmArgs& g, hipStream_t s) {
    const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_kernel<T, AT, RT>), dim3((unsigned)tiles), dim3(NT), 0, s, g);
    return hipGetLastError();
}

template <typename T, bool AT, bool RT>
hipError_t gemm_group_launch_t(const GemmGroup& grp, hipStream_t s) {
    int64_t max_m = 0, max_n = 0;
    for (int i = 0; i < grp.count; ++i) {
        if (grp.g[i].M > max_m) max_m = grp.g[i].M;
        if (grp.g[i].N > max_n) max_n = grp.g[i].N;
    }
    if (max_m <= 0 || max_n <= 0) return hipSuccess;
    const int64_t tm = (max_m + BM - 1) / BM, tn = (max_n + BN - 1) / BN;
    hipLaunchKernelGGL((gemm_group_kernel<T, AT, RT>), dim3((unsigned)(tm * tn), (unsigned)grp.count),
                       dim3(NT), 0, s, grp, tm);
    return hipGetLastError();
}

template <typename T>
hipError_t gemm_launch_any(bool at, bool rt, const GemmArgs& g, hipStream_t s) {
    if (!at && !rt) return gemm_launch_t<T, false, false>(g, s);
    if (at && !rt) return gemm_launch_t<T, true, false>(g, s);
    if (!at && rt) return gemm_launch_t<T, false, true>(g, s);
    return gemm_launch_t<T, true, true>(g, s);
}

template <typename T>
hipError_t gemm_group_any(bool at, bool rt, const GemmGroup& grp, hipStream_t s) {
    if (!at && !rt) return gemm_group_launch_t<T, false, false>(grp, s);
    if (at && !rt) return gemm_group_launch_t<T, true, false>(grp, s);
    if (!at && rt) return gemm_group_launch_t<T, false, true>(grp, s);
    return gemm_group_launch_t<T, true, true>(grp, s);
}

}  // namespace

hipError_t launch_gemm(int dtype, bool a_trans, bool rhs_trans, const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
    return dtype == 0 ? gemm_launch_any<double>(a_trans, rhs_trans, g, s)
                      : gemm_launch_any<float>(a_trans, rhs_trans, g, s);
}

hipError_t launch_gemm_group(int dtype, bool a_trans, bool rhs_trans, const GemmGroup& grp,
                             hipStream_t s) {
    if (grp.count <= 0) return hipSuccess;
    if (grp.count > kMaxGroup) return hipErrorInvalidValue;
    return dtype == 0 ? gemm_group_any<double>(a_trans, rhs_trans, grp, s)
                      : gemm_group_any<float>(a_trans, rhs_trans, grp, s);
}

}  // namespace redsea
