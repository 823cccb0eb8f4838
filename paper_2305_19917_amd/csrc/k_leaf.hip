// Diagonal-block (leaf) solve and its helpers, gfx950.
//
// The leaf is the "TS" task that the paper's models leave at the finest
// granularity (Sec. V-A: the white triangles of the recursive model; the
// same tasks appear in Sec. V-B and V-C).  Here it runs on the GPU, by the
// forward substitution of Sec. IV in axpy order (after unknown k is divided
// out, every later row is updated with it), on a packed canonical copy of the
// diagonal block staged in LDS.  FP32 data is solved by the same kernel: it
// is widened to FP64 on load and rounded to FP32 on store, so an FP32 leaf is
// at least as accurate as one computed in FP32.
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

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Step 1-2 of a 16-row diagonal block, for one wave's 16 columns: `frag`
// holds rows g + 4r of the block (column c) in accumulator layout; the block
// is gathered through the wave's LDS buffer Xw so that every lane holds its
// column's 16 values, solved by substitution against the 16 x 16 lower
// triangle Lb (LDS, element (row j, column i) at Lb[i*16 + j], axpy order,
// one IEEE division per row unless UNIT), and each lane keeps its own four
// rows of the solution in `frag`.
template <bool UNIT>
__device__ __forceinline__ void solve_diag16(const double* Lb, double (*Xw)[17], v4d& frag, int g,
                                             int c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) Xw[g + 4 * r][c] = frag[r];
    wave_sync();
    double y[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) y[i] = Xw[i][c];
    // Column i+1 of the block is read from LDS while column i is applied, so
    // the chain of a step is one division and one fused multiply-add.
    double cur[16], nxt[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) cur[j] = Lb[j];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i + 1 < 16) {
#pragma unroll
            for (int j = i + 1; j < 16; ++j) nxt[j] = Lb[(i + 1) * 16 + j];
        }
        double x = y[i];
        if (!UNIT) x = x / cur[i];
        y[i] = x;
#pragma unroll
        for (int j = i + 1; j < 16; ++j) y[j] = __builtin_fma(-cur[j], x, y[j]);
#pragma unroll
        for (int j = i; j < 16; ++j) asm volatile("" : "+v"(y[j]));
        asm volatile("" ::: "memory");
#pragma unroll
        for (int j = i + 1; j < 16; ++j) cur[j] = nxt[j];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double v01 = g == 0 ? y[4 * r] : y[4 * r + 1];
        const double v23 = g == 2 ? y[4 * r + 2] : y[4 * r + 3];
        frag[r] = g < 2 ? v01 : v23;
    }
    wave_sync();  // every lane has read Xw before it is written again
}

// Panel leaf on matrix cores.  A workgroup of four waves covers 64
// right-hand-side columns, each wave 16 of them, and holds its NP x 16 slab of
// B in MFMA accumulator layout: fragment f, register r of lane l is row
// 16 f + l/16 + 4 r, column l % 16 (the v_mfma_f64_16x16x4f64 result
// layout).  The lower triangle of the packed diagonal block is staged in LDS
// once, as 16 x 16 blocks (all loads issued together).  Then the panel is
// solved by 16-row diagonal blocks:
//   1. the 16 x 16 block of each column is gathered into one lane (every
//      lane of the column's four lane groups gets the whole column, through
//      LDS) and solved there by substitution, one IEEE division per row;
//   2. each lane keeps its own four rows of the result;
//   3. every later 16-row fragment is updated on the matrix cores,
//      frag_p -= L_ps X_s, whose B operand for k-slice kk is exactly register
//      kk of the solved fragment, so no data moves for the update.
// After staging, the four waves run independently.
template <typename TS, int NP, bool UNIT, bool FULL>
__global__ __launch_bounds__(256) void leaf_mfma_kernel(const TS* __restrict__ P, int rows,
                                                        TS* __restrict__ B, int64_t off,
                                                        int64_t br, int64_t bc, int64_t ncols) {
    constexpr int NF = NP / 16;
    constexpr int NO = NF * (NF - 1) / 2;  // strictly lower 16 x 16 blocks
    // block (p, s), p >= s, element (row j, column i) at [i*16 + j]:
    // diagonal blocks first, then (p, s), p > s, at NF + p(p-1)/2 + s
    __shared__ double Ls[(NF + NO) * 256];
    __shared__ double Xs[4][16][17];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
    {
        TS t[NF + NO];
#pragma unroll
        for (int f = 0; f < NF; ++f) t[f] = P[(16 * f + tid / 16) * NP + 16 * f + tid % 16];
#pragma unroll
        for (int p = 1; p < NF; ++p)
#pragma unroll
            for (int q = 0; q < p; ++q)
                t[NF + p * (p - 1) / 2 + q] = P[(16 * q + tid / 16) * NP + 16 * p + tid % 16];
#pragma unroll
        for (int b = 0; b < NF + NO; ++b) Ls[b * 256 + tid] = (double)t[b];
    }
    const int64_t col = (int64_t)blockIdx.x * 64 + w * 16 + c;
    const bool colok = col < ncols;
    TS* bp = B + off + (colok ? col : 0) * bc;
    v4d fr[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * f + g + 4 * r;
            fr[f][r] = (colok && (FULL || row < rows)) ? (double)bp[row * br] : 0.0;
        }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NF; ++s) {
        // 1-2. solve the diagonal block; each lane keeps its rows
        solve_diag16<UNIT>(Ls + s * 256, Xs[w], fr[s], g, c);
        // 3. matrix-core update of the fragments below; A operand for
        // k-slice kk: element (16p + c, 16s + 4kk + g) of the triangle
#pragma unroll
        for (int p = s + 1; p < NF; ++p) {
            const double* Lo = Ls + (NF + p * (p - 1) / 2 + s) * 256;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                fr[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(-Lo[(4 * kk + g) * 16 + c], fr[s][kk],
                                                             fr[p], 0, 0, 0);
        }
    }
    if (colok) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * f + g + 4 * r;
                if (FULL || row < rows) bp[row * br] = (TS)fr[f][r];
            }
    }
}

template <typename TS, int NP>
hipError_t leaf_mfma_dispatch(const TS* P, int64_t rows, TS* B, int64_t off, int64_t br,
                              int64_t bc, int64_t ncols, bool unit, hipStream_t s) {
    dim3 grid((unsigned)((ncols + 63) / 64)), block(256);
    const bool full = rows == NP;
    if (unit && full)
        hipLaunchKernelGGL((leaf_mfma_kernel<TS, NP, true, true>), grid, block, 0, s, P,
                           (int)rows, B, off, br, bc, ncols);
    else if (unit)
        hipLaunchKernelGGL((leaf_mfma_kernel<TS, NP, true, false>), grid, block, 0, s, P,
                           (int)rows, B, off, br, bc, ncols);
    else if (full)
        hipLaunchKernelGGL((leaf_mfma_kernel<TS, NP, false, true>), grid, block, 0, s, P,
                           (int)rows, B, off, br, bc, ncols);
    else
        hipLaunchKernelGGL((leaf_mfma_kernel<TS, NP, false, false>), grid, block, 0, s, P,
                           (int)rows, B, off, br, bc, ncols);
    return hipGetLastError();
}

// Elements e = e0 + x + k*NS (k < PER) of the lower triangle of segment t of
// a packed NP2 x NP2 diagonal block, copied by thread x of NS into dst in the
// blocked LDS layout of leaf_mfma_kernel: 16 x 16 block (p, s) of the segment
// is block (8t + p, 8t + s) of the square; diagonal blocks first, then
// p > s at 8 + p(p-1)/2 + s; element (row j, column i) at [i*16 + j].
template <typename TS, int NP2, int PER, int NS>
__device__ __forceinline__ void stage_tri(const TS* __restrict__ P, int t, double* dst, int e0,
                                          int x) {
    const TS* Pt = P + (int64_t)128 * t * NP2 + 128 * t;
    double v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = e0 + x + k * NS, blk = e >> 8, i = (e >> 4) & 15, j = e & 15;
        int pp = blk, ss = blk;
        if (blk >= 8) {
            int u = blk - 8;
            pp = 1;
            while (u >= pp) {
                u -= pp;
                ++pp;
            }
            ss = u;
        }
        v[k] = (double)Pt[(16 * ss + i) * NP2 + 16 * pp + j];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) dst[e0 + x + k * NS] = v[k];
}

// Segmented leaf: a diagonal block of NQ*128 rows solved in one launch.  A
// workgroup covers CG column groups of 16 right-hand sides; each column group
// has NQ waves, wave q holding rows [128q, 128q + 128) of its 16 columns in
// accumulator layout (as in leaf_mfma_kernel).  The block is the recursive
// split of Sec. V-A carried out inside the kernel: in phase t, wave t solves
// its segment against the segment's triangle (in LDS) exactly as
// leaf_mfma_kernel does, and publishes every solved 16-row block through LDS;
// each later wave of the column group applies that block to its own rows at
// once on the matrix cores (the off-diagonal product of the split), reading
// the coupling block from the packed diagonal block in global memory, where
// all workgroups share it in L2.  When phase t ends, segment t+1 has received
// all of its updates; no product between segments goes through HBM.  The
// triangle of segment t+1 is staged into the second LDS buffer by the waves
// of segment t+1 during phase t, one slice per 16-row step, so no phase waits
// for its triangle.
template <typename TS, int NQ, int CG, bool UNIT, bool FULL>
__global__ __launch_bounds__(64 * NQ * CG) void leaf_seg_kernel(const TS* __restrict__ P, int rows,
                                                                TS* __restrict__ B, int64_t off,
                                                                int64_t br, int64_t bc,
                                                                int64_t ncols) {
    constexpr int NP2 = 128 * NQ;          // order of the packed block
    constexpr int NF = 8, NO = 28;         // 16-row blocks of a segment
    constexpr int NT = 64 * NQ * CG;       // threads
    constexpr int NE = (NF + NO) * 256;    // triangle elements of a segment
    constexpr int SL = NE / NF;            // elements staged per 16-row step
    static_assert(NE % NT == 0 && SL % (64 * CG) == 0, "staging assumes whole passes");
    __shared__ double Ls[2][NE];           // triangles of phases t (t & 1)
    __shared__ double Xs[CG][16][17];      // gather buffer of the solving wave
    __shared__ v4d Xb[2][CG][64];          // solved blocks, accumulator layout
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
    const int q = w / CG, cg = w % CG;
    const int nseg = FULL ? NQ : (rows + 127) / 128;
    const int64_t col = (int64_t)blockIdx.x * (16 * CG) + cg * 16 + c;
    const bool colok = col < ncols;
    TS* bp = B + off + (colok ? col : 0) * bc;
    v4d fr[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 128 * q + 16 * f + g + 4 * r;
            fr[f][r] = (colok && (FULL || row < rows)) ? (double)bp[row * br] : 0.0;
        }
    stage_tri<TS, NP2, NE / NT, NT>(P, 0, Ls[0], 0, tid);
    __syncthreads();
    for (int t = 0; t < nseg; ++t) {
        // Ls[t & 1] was completed before the last block barrier of phase t-1,
        // and nobody reads Ls[(t + 1) & 1] after that barrier
        const double* Lt = Ls[t & 1];
        const bool solver = q == t, later = q > t && q < nseg;
        const bool stager = q == t + 1 && q < nseg;
#pragma unroll
        for (int s = 0; s < NF; ++s) {
            const int b = NF * t + s;  // block column in the packed square
            double a[NF][4];           // coupling block (L_qb), later waves only
            if (solver) {
                solve_diag16<UNIT>(Lt + s * 256, Xs[cg], fr[s], g, c);
                Xb[b & 1][cg][lane] = fr[s];
            } else if (later) {
                // A operand of k-slice kk for fragment p: element
                // (128q + 16p + c, 16b + 4kk + g) of the square, loaded while
                // block b is being solved
                const TS* Pc = P + (int64_t)(16 * b + g) * NP2 + 128 * q + c;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                    for (int p = 0; p < NF; ++p) a[p][kk] = -(double)Pc[4 * kk * NP2 + 16 * p];
                if (stager)
                    stage_tri<TS, NP2, SL / (64 * CG), 64 * CG>(P, t + 1, Ls[(t + 1) & 1],
                                                                 s * SL, cg * 64 + lane);
            }
            __syncthreads();  // block b published
            if (solver) {
#pragma unroll
                for (int p = s + 1; p < NF; ++p) {
                    const double* Lo = Lt + (NF + p * (p - 1) / 2 + s) * 256;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
                        fr[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(-Lo[(4 * kk + g) * 16 + c],
                                                                     fr[s][kk], fr[p], 0, 0, 0);
                }
            } else if (later) {
                const v4d xb = Xb[b & 1][cg][lane];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                    for (int p = 0; p < NF; ++p)
                        fr[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p][kk], xb[kk], fr[p], 0, 0,
                                                                     0);
            }
        }
        if (solver && colok) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 128 * q + 16 * f + g + 4 * r;
                    if (FULL || row < rows) bp[row * br] = (TS)fr[f][r];
                }
        }
    }
}

template <typename TS, int NQ, int CG>
hipError_t leaf_seg_dispatch(const TS* P, int64_t rows, TS* B, int64_t off, int64_t br, int64_t bc,
                             int64_t ncols, bool unit, hipStream_t s) {
    dim3 grid((unsigned)((ncols + 16 * CG - 1) / (16 * CG))), block(64 * NQ * CG);
    const bool full = rows == 128 * NQ;
    if (unit && full)
        hipLaunchKernelGGL((leaf_seg_kernel<TS, NQ, CG, true, true>), grid, block, 0, s, P,
                           (int)rows, B, off, br, bc, ncols);
    else if (unit)
        hipLaunchKernelGGL((leaf_seg_kernel<TS, NQ, CG, true, false>), grid, block, 0, s, P,
                           (int)rows, B, off, br, bc, ncols);
    else if (full)
        hipLaunchKernelGGL((leaf_seg_kernel<TS, NQ, CG, false, true>), grid, block, 0, s, P,
                           (int)rows, B, off, br, bc, ncols);
    else
        hipLaunchKernelGGL((leaf_seg_kernel<TS, NQ, CG, false, false>), grid, block, 0, s, P,
                           (int)rows, B, off, br, bc, ncols);
    return hipGetLastError();
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
            case 16: return leaf_mfma_dispatch<double, 16>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 32: return leaf_mfma_dispatch<double, 32>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 64: return leaf_mfma_dispatch<double, 64>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 128:
                return leaf_mfma_dispatch<double, 128>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 256:
                return leaf_seg_dispatch<double, 2, 2>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            default: return hipErrorInvalidValue;
        }
    } else {
        const float* P = (const float*)pblk;
        float* b = (float*)B.base;
        switch (nb) {
            case 16: return leaf_mfma_dispatch<float, 16>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 32: return leaf_mfma_dispatch<float, 32>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 64: return leaf_mfma_dispatch<float, 64>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 128:
                return leaf_mfma_dispatch<float, 128>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
            case 256:
                return leaf_seg_dispatch<float, 2, 2>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
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
