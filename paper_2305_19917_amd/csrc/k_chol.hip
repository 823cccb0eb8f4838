// Cholesky factorisation of one diagonal block, gfx950: the leaf of the
// recursive factorisation (the application the paper names for its solver,
// Sec. VIII; the recursion itself mirrors the split of Sec. V-A).
//
// One workgroup of 1024 threads factors a block of order b <= B (32, 64 or
// 128) as the lower factor L (an upper factorisation reads the block through
// swapped strides, so U = L^T is factored as the same L).  The 32 x 32 thread
// grid holds the block 2-D cyclically in registers: thread (tr, tk) owns the
// entries (tr + 32 p, tk + 32 q), (B/32)^2 of them.  Step j (right-looking):
// the owners of column j publish it to LDS (double-buffered, so one barrier
// per step) and the pivot's owner publishes 1 / d_j beside it; every thread
// reads the pivot d_j = A(j, j) and updates its own entries of the trailing
// triangle, A(r, k) -= A(r, j) (A(k, j) / d_j), which is l_rj l_kj with
// l = a / sqrt(d); the update touches registers only, so its LDS reads
// issue together.  At the end every entry is divided by the square root of
// its column's pivot (the diagonal becomes that root): the same correctly
// rounded l_rk = a_rk / l_kk as column-by-column scaling.  A pivot that is
// not positive (or NaN) stops the block: info := its global column + 1, the
// columns before it are finished and the rest is written back as it stands.
// A block whose info is already set (an earlier block failed) does nothing.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace redsea {

namespace {

// G x G threads; each holds (B/G) x (B/G) entries of the block.  At B = 128
// the 32 x 32 grid (16 entries per thread) takes 86 us per block, a 16 x 16
// grid (64 entries per thread, four waves) took 142 us: a step is a chain of
// barrier, LDS round trips and one wave's share of the update, and smaller
// shares shorten it.
constexpr int kCholGrid = 32;

template <typename T, int B>
__global__ __launch_bounds__(kCholGrid * kCholGrid) void potrf_leaf_kernel(T* a, int64_t sr,
                                                                           int64_t sc, int b,
                                                                           int64_t col0,
                                                                           int* info) {
    constexpr int G = kCholGrid, NR = B / G;  // entries per thread: NR x NR
    __shared__ T col[2][B];  // column j of step j before scaling, double-buffered
    __shared__ T rcp[2];     // 1 / A(j, j), from the pivot's owner
    if (*info != 0) return;  // uniform
    const int tid = threadIdx.x;
    // the owners of a column (equal tk) are one contiguous half-wave, so one
    // wave publishes at each step, whatever the storage order (for an upper
    // factorisation the block's loads and stores are then strided; they run
    // once per block and mostly from L2)
    const int tr = tid % G;  // rows tr + G p
    const int tk = tid / G;  // columns tk + G q
    // rows that are never published (past b) read as zero, so every entry
    // the update touches stays finite
    for (int i = tid; i < 2 * B; i += G * G) col[i / B][i % B] = T(0);
    T v[NR][NR];  // v[p][q] = A(tr + G p, tk + G q), lower triangle (p >= q)
#pragma unroll
    for (int p = 0; p < NR; ++p)
#pragma unroll
        for (int q = 0; q <= p; ++q) {
            const int r = tr + G * p, k = tk + G * q;
            v[p][q] = (r < b && k <= r) ? a[r * sr + k * sc] : T(0);
        }
    T dk[NR];  // pivots of the owned columns
#pragma unroll
    for (int q = 0; q < NR; ++q) dk[q] = T(0);
    __syncthreads();
    int fail = -1;
    for (int j = 0; j < b; ++j) {
        const int par = j & 1, qj = j / G;
        const bool owner = tk == j % G;
        if (owner) {  // the owners of column j publish it (rows >= j)
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if (q != qj) continue;  // uniform
#pragma unroll
                for (int p = q; p < NR; ++p) {
                    const int r = tr + G * p;
                    if (r >= j && r < b) col[par][r] = v[p][q];
                }
                if (tr == j % G) rcp[par] = T(1) / v[q][q];  // the pivot's owner
            }
        }
        __syncthreads();
        const T d = col[par][j];
        if (!(d > T(0))) {  // uniform: every thread read the same pivot
            fail = j;
            break;
        }
        if (owner) {
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (q == qj) dk[q] = d;
        }
        const T rd = rcp[par];
        // Schur complement: A(r, k) -= A(r, j) (A(k, j) / d) for j < k <= r.
        // The multiplier of a finished column (k <= j) is zero, which leaves
        // its entries as they are; entries outside the triangle (k > r, or
        // r >= b) are updated too and never stored.  Sets of G columns that
        // lie wholly at or before j are skipped.
        T cr[NR], ck[NR];
#pragma unroll
        for (int p = 0; p < NR; ++p) cr[p] = col[par][tr + G * p];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const T c = col[par][tk + G * q];
            ck[q] = tk + G * q > j ? c * rd : T(0);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if (G * q + G - 1 <= j) continue;  // uniform
#pragma unroll
            for (int p = q; p < NR; ++p) v[p][q] = v[p][q] - cr[p] * ck[q];
        }
    }
    if (fail >= 0 && tid == 0) *info = (int)(col0 + fail + 1);
    const int done = fail >= 0 ? fail : b;  // columns whose pivot was taken
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int k = tk + G * q;
        const T l = sqrt(dk[q]);
#pragma unroll
        for (int p = q; p < NR; ++p) {
            const int r = tr + G * p;
            if (r < b && k <= r) {
                if (k < done) v[p][q] = r == k ? l : v[p][q] / l;
                a[r * sr + k * sc] = v[p][q];
            }
        }
    }
}

__global__ void info_clear_kernel(int* info) {
    if (threadIdx.x == 0) info[0] = 0;
}

template <typename T>
hipError_t leaf_t(void* a, int64_t sr, int64_t sc, int b, int64_t col0, int* info,
                  hipStream_t s) {
    T* p = (T*)a;
    const dim3 block(kCholGrid * kCholGrid);
    if (b <= 32)
        hipLaunchKernelGGL((potrf_leaf_kernel<T, 32>), dim3(1), block, 0, s, p, sr, sc, b, col0,
                           info);
    else if (b <= 64)
        hipLaunchKernelGGL((potrf_leaf_kernel<T, 64>), dim3(1), block, 0, s, p, sr, sc, b, col0,
                           info);
    else
        hipLaunchKernelGGL((potrf_leaf_kernel<T, 128>), dim3(1), block, 0, s, p, sr, sc, b, col0,
                           info);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_potrf_leaf(int dtype, void* a, int64_t sr, int64_t sc, int b, int64_t col0,
                             int* info, hipStream_t s) {
    if (b <= 0) return hipSuccess;
    if (b > kCholLeafMax) return hipErrorInvalidValue;
    return dtype == 0 ? leaf_t<double>(a, sr, sc, b, col0, info, s)
                      : leaf_t<float>(a, sr, sc, b, col0, info, s);
}

hipError_t launch_info_clear(int* info, hipStream_t s) {
    hipLaunchKernelGGL(info_clear_kernel, dim3(1), dim3(64), 0, s, info);
    return hipGetLastError();
}

}  // namespace redsea
