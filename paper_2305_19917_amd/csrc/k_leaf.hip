// Diagonal-block (leaf) solve and its helpers, gfx950.
//
// The leaf is the "TS" task that the paper's models leave at the finest
// granularity (Sec. V-A: the white triangles of the recursive model; the
// same tasks appear in Sec. V-B and V-C).  Here it runs on the GPU: each
// lane owns one right-hand-side column, keeps the column's nb entries in
// registers and performs the forward substitution of Sec. IV on them (axpy
// order: after unknown k is divided out, every later row is updated with it).
// The triangle is uniform across the wave: it is copied once into LDS from a
// packed canonical copy and read with broadcast loads.  The dependency chain
// per unknown is one IEEE division followed by fused multiply-adds.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace redsea {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void pack_diag_kernel(const T* __restrict__ A, int64_t off,
                                                        int64_t tr, int64_t tc, int64_t m,
                                                        int nb, int64_t first_blk, int64_t nblk,
                                                        int unit, T* __restrict__ P) {
    const int64_t nn = (int64_t)nb * nb;
    for (int64_t blk = blockIdx.y; blk < nblk; blk += gridDim.y) {
        const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
        if (idx >= nn) continue;
        const int r = (int)(idx % nb), c = (int)(idx / nb);
        const int64_t gi = (first_blk + blk) * nb + r, gj = (first_blk + blk) * nb + c;
        T v;
        if (r < c) v = T(0);
        else if (gi >= m) v = (r == c) ? T(1) : T(0);
        else if (r == c && unit) v = T(1);
        else v = A[off + gi * tr + gj * tc];
        P[blk * nn + idx] = v;
    }
}

// One wave per 64 columns.  rows <= NB; the packed block completes rows past
// `rows` with the identity, so they stay zero and are not stored.  The
// triangle is staged in LDS once per workgroup and read with broadcast loads
// (every lane reads the same element).
template <typename T, int NB, bool UNIT, bool FULL>
__global__ __launch_bounds__(64) void leaf_kernel(const T* __restrict__ P, int rows,
                                                  T* __restrict__ B, int64_t off, int64_t br,
                                                  int64_t bc, int64_t ncols) {
    __shared__ T Ls[NB * NB];
    for (int idx = threadIdx.x; idx < NB * NB; idx += 64) Ls[idx] = P[idx];
    __syncthreads();
    const int64_t col = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (col >= ncols) return;
    T* bp = B + off + col * bc;
    T b[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) b[i] = (FULL || i < rows) ? bp[i * br] : T(0);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        T x = b[k];
        if (!UNIT) x = x / Ls[k + k * NB];
        b[k] = x;
#pragma unroll
        for (int i = k + 1; i < NB; ++i) b[i] = __builtin_fma(-Ls[i + k * NB], x, b[i]);
        // Keep the axpy order: every update of step k is materialised here,
        // and no LDS read of a later step is hoisted above this point.
#pragma unroll
        for (int i = k; i < NB; ++i) asm volatile("" : "+v"(b[i]));
        asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
        if (FULL || i < rows) bp[i * br] = b[i];
}

template <typename T>
__global__ __launch_bounds__(256) void scale_kernel(T* __restrict__ B, int64_t m, int64_t n,
                                                    int64_t ldb, T alpha) {
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx % m, j = idx / m;
        T* p = B + i + j * ldb;
        *p = alpha == T(0) ? T(0) : alpha * *p;
    }
}

// One workgroup scans the matrix; the verdict is reduced in LDS and written by
// thread 0, so the result is a plain store (no atomics).
template <typename T>
__global__ __launch_bounds__(256) void check_finite_kernel(const T* __restrict__ B, int64_t m,
                                                           int64_t n, int64_t ldb,
                                                           int* __restrict__ info, int code) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    int mine = 0;
    const int64_t total = m * n;
    for (int64_t idx = threadIdx.x; idx < total; idx += 256) {
        const T v = B[(idx % m) + (idx / m) * ldb];
        if (!__builtin_isfinite(v)) mine = 1;
    }
    if (mine) bad = 1;  // benign race: every writer stores the same value
    __syncthreads();
    if (threadIdx.x == 0) info[0] = bad ? code : 0;
}

template <typename T, int NB>
hipError_t leaf_dispatch(const T* P, int64_t rows, T* B, int64_t off, int64_t br, int64_t bc,
                         int64_t ncols, bool unit, hipStream_t s) {
    dim3 grid((unsigned)((ncols + 63) / 64)), block(64);
    const bool full = rows == NB;
    if (unit && full)
        hipLaunchKernelGGL((leaf_kernel<T, NB, true, true>), grid, block, 0, s, P, (int)rows, B,
                           off, br, bc, ncols);
    else if (unit)
        hipLaunchKernelGGL((leaf_kernel<T, NB, true, false>), grid, block, 0, s, P, (int)rows, B,
                           off, br, bc, ncols);
    else if (full)
        hipLaunchKernelGGL((leaf_kernel<T, NB, false, true>), grid, block, 0, s, P, (int)rows, B,
                           off, br, bc, ncols);
    else
        hipLaunchKernelGGL((leaf_kernel<T, NB, false, false>), grid, block, 0, s, P, (int)rows,
                           B, off, br, bc, ncols);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pack_diag(int dtype, const TriView& T, int64_t m, int nb, int64_t first_blk,
                            int64_t nblk, bool unit, void* packed, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    const int64_t nn = (int64_t)nb * nb;
    dim3 grid((unsigned)((nn + 255) / 256), (unsigned)(nblk < 65535 ? nblk : 65535)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL(pack_diag_kernel<double>, grid, block, 0, s, (const double*)T.base,
                           T.off, T.tr, T.tc, m, nb, first_blk, nblk, unit ? 1 : 0, (double*)packed);
    else
        hipLaunchKernelGGL(pack_diag_kernel<float>, grid, block, 0, s, (const float*)T.base,
                           T.off, T.tr, T.tc, m, nb, first_blk, nblk, unit ? 1 : 0, (float*)packed);
    return hipGetLastError();
}

hipError_t launch_leaf(int dtype, int nb, const void* pblk, int64_t rows, const RhsView& B,
                       int64_t row0, int64_t ncols, bool unit, hipStream_t s) {
    if (ncols <= 0 || rows <= 0) return hipSuccess;
    const int64_t off = B.off + row0 * B.br;
    if (dtype == 0) {
        const double* P = (const double*)pblk;
        double* b = (double*)B.base;
        switch (nb) {
            case 16: return leaf_dispatch<double, 16>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 32: return leaf_dispatch<double, 32>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 64: return leaf_dispatch<double, 64>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            default: return hipErrorInvalidValue;
        }
    } else {
        const float* P = (const float*)pblk;
        float* b = (float*)B.base;
        switch (nb) {
            case 16: return leaf_dispatch<float, 16>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 32: return leaf_dispatch<float, 32>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 64: return leaf_dispatch<float, 64>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            default: return hipErrorInvalidValue;
        }
    }
}

hipError_t launch_check_finite(int dtype, const void* b, int64_t m, int64_t n, int64_t ldb,
                               int* info, int code, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(check_finite_kernel<double>, dim3(1), dim3(256), 0, s,
                           (const double*)b, m, n, ldb, info, code);
    else
        hipLaunchKernelGGL(check_finite_kernel<float>, dim3(1), dim3(256), 0, s,
                           (const float*)b, m, n, ldb, info, code);
    return hipGetLastError();
}

hipError_t launch_scale(int dtype, void* b, int64_t m, int64_t n, int64_t ldb, double alpha,
                        hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    int64_t blocks = (m * n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (dtype == 0)
        hipLaunchKernelGGL(scale_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (double*)b, m, n, ldb, alpha);
    else
        hipLaunchKernelGGL(scale_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (float*)b, m, n, ldb, (float)alpha);
    return hipGetLastError();
}

}  // namespace redsea
