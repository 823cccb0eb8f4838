// Diagonal-block (leaf) solve and its helpers, gfx950.
//
// The leaf is the "TS" task that the paper's models leave at the finest
// granularity (Sec. V-A: the white triangles of the recursive model; the
// same tasks appear in Sec. V-B and V-C).  Here it runs on the GPU, by the
// forward substitution of Sec. IV in axpy order (every later row is updated
// with each new unknown), on a packed canonical copy of the diagonal block
// scaled by rows: the packed block holds D^-1 L (each strictly lower entry
// divided by its row's diagonal, correctly rounded; the diagonal itself
// kept), and the leaf divides its panel by the diagonal once before the
// substitution, so no division sits on the chain of dependent steps.  This
// is substitution on the row-scaled system (componentwise backward stable;
// a diagonal system is still one correctly rounded division per entry).  Leaves of up to 128 rows keep the block's whole triangle
// in LDS (leaf_mfma_kernel); 256-row leaves keep only its 16 x 16 diagonal
// blocks there and apply the rest as matrix-core products between two waves
// (leaf_ilv_kernel).  FP32 data is solved by the same kernels: it is widened
// to FP64 on load and rounded to FP32 on store, so an FP32 leaf is at least
// as accurate as one computed in FP32.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace redsea {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void pack_diag_kernel(const T* __restrict__ A, int64_t off,
                                                        int64_t tr, int64_t tc, int64_t m,
                                                        int nb, int64_t first_blk, int64_t nblk,
                                                        int unit, int64_t stride,
                                                        T* __restrict__ P) {
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
        else if (r == c || unit) v = A[off + gi * tr + gj * tc];
        else  // row-scaled: L(r, c) / L(r, r), correctly rounded
            v = (T)((double)A[off + gi * tr + gj * tc] / (double)A[off + gi * tr + gi * tc]);
        P[blk * stride + idx] = v;
    }
}

// For 256-row leaves: the 120 strictly lower 16 x 16 blocks (p, s), p > s, of
// each packed square, negated, in the A-operand order of
// v_mfma_f64_16x16x4f64: block p(p-1)/2 + s holds, for lane l and k-slice kk,
// -L(16p + l % 16, 16s + 4kk + l / 16) at [l*4 + kk], so one lane's four
// k-slices are 32 contiguous bytes.  Reads the square written just before
// (stream order) and writes behind it.
template <typename T>
__global__ __launch_bounds__(256) void pack_frag_kernel(T* __restrict__ P, int64_t nblk,
                                                        int64_t stride) {
    constexpr int NP2 = 256;
    for (int64_t blk = blockIdx.y; blk < nblk; blk += gridDim.y) {
        const int e = blockIdx.x * 256 + threadIdx.x;  // < 120 * 256 by the grid
        const int bidx = e >> 8, l = (e >> 2) & 63, kk = e & 3;
        int p = 1, u = bidx;
        while (u >= p) {
            u -= p;
            ++p;
        }
        const int s = u;
        T* sq = P + blk * stride;
        sq[NP2 * NP2 + e] = -sq[(16 * s + 4 * kk + (l >> 4)) * NP2 + 16 * p + (l & 15)];
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
// column's 16 values, solved by substitution against the unit lower 16 x 16
// triangle Lb (LDS, element (row j, column i) at Lb[i*16 + j], axpy order;
// the diagonal entries are not read), and each lane keeps its own four rows
// of the solution in `frag`.
__device__ __forceinline__ void solve_diag16(const double* Lb, double (*Xw)[17], v4d& frag, int g,
                                             int c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) Xw[g + 4 * r][c] = frag[r];
    wave_sync();
    double y[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) y[i] = Xw[i][c];
    // Column i+1 of the block is read from LDS while column i is applied, so
    // the chain of a step is one fused multiply-add.
    double cur[16], nxt[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) cur[j] = Lb[j];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i + 1 < 16) {
#pragma unroll
            for (int j = i + 1; j < 16; ++j) nxt[j] = Lb[(i + 1) * 16 + j];
        }
        const double x = y[i];
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
//      LDS) and solved there by unit-diagonal substitution (the panel was
//      divided by the diagonal beforehand);
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
    if (!UNIT) {
        // the panel divided by the diagonal (correctly rounded) once: the
        // packed block holds D^-1 L, so every step below is unit-diagonal
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) fr[f][r] = fr[f][r] / Ls[f * 256 + (g + 4 * r) * 17];
    }
#pragma unroll
    for (int s = 0; s < NF; ++s) {
        // 1-2. solve the (unit) diagonal block; each lane keeps its rows
        solve_diag16(Ls + s * 256, Xs[w], fr[s], g, c);
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

// Interleaved 256-row leaf.  Each column group of 16 right-hand sides has two
// waves; wave v holds the 16-row blocks s = v, v + 2, ..., 14 + v of the leaf
// (fragment j is block 2j + v, accumulator layout as in leaf_mfma_kernel).
// Block s is solved by its owner wave, which publishes the solution x_s
// through LDS.  After the block barrier the other wave, owner of block
// s + 1, applies x_s to that block only (four MFMAs on the critical path)
// and goes on to solve it; x_s reaches its later blocks one step after, in
// the same order.  The owner of block s meanwhile applies x_{s-1} and x_s to
// its own later blocks.  Every update is the Sec. IV product of a solved
// block into the rows below, applied block by block in increasing s (the
// same MFMA sequence per block as solving 128-row halves one after the
// other).  The coupling blocks come from the packed diagonal block in global
// memory (L2-resident, shared by all workgroups), each loaded by the wave
// that applies it one or two steps before it is needed.  Only the 16
// diagonal 16 x 16 blocks live in LDS.
template <typename TS, int CG, bool UNIT, bool FULL>
__global__ __launch_bounds__(128 * CG) void leaf_ilv_kernel(const TS* __restrict__ P, int rows,
                                                            TS* __restrict__ B, int64_t off,
                                                            int64_t br, int64_t bc,
                                                            int64_t ncols) {
    constexpr int NP2 = 256, NBK = 16, NJ = 8, NT = 128 * CG;
    static_assert((NBK * 256) % NT == 0, "staging assumes whole passes");
    __shared__ double Ds[NBK * 256];       // diagonal block s at s*256, [i*16 + j]
    __shared__ double Xs[CG][16][17];      // gather buffer of the solving wave
    __shared__ v4d Xb[2][CG][64];          // solved blocks, accumulator layout
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, c = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar branches
    const int v = w / CG, cg = w % CG;
    const int64_t col = (int64_t)blockIdx.x * (16 * CG) + cg * 16 + c;
    const bool colok = col < ncols;
    TS* bp = B + off + (colok ? col : 0) * bc;
    v4d fr[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * (2 * j + v) + g + 4 * r;
            fr[j][r] = (colok && (FULL || row < rows)) ? (double)bp[row * br] : 0.0;
        }
    {
        double t[NBK * 256 / NT];
#pragma unroll
        for (int k = 0; k < NBK * 256 / NT; ++k) {
            const int e = tid + k * NT, b = e >> 8, i = (e >> 4) & 15, jj = e & 15;
            t[k] = (double)P[(16 * b + i) * NP2 + 16 * b + jj];
        }
#pragma unroll
        for (int k = 0; k < NBK * 256 / NT; ++k) Ds[tid + k * NT] = t[k];
    }
    __syncthreads();
    if (!UNIT) {
        // the panel divided by the diagonal (correctly rounded) once: the
        // packed block holds D^-1 L, so every step below is unit-diagonal
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) fr[j][r] = fr[j][r] / Ds[(2 * j + v) * 256 + (g + 4 * r) * 17];
    }
    // A operands of block (p, s), k-slices 0..3, from the fragment-ordered
    // copy behind the square (one 32- or 16-byte load per lane)
    const TS* F = P + NP2 * NP2;
    auto lop4 = [&](int p, int s, double* out) {
        const TS* q = F + (p * (p - 1) / 2 + s) * 256 + lane * 4;
        if constexpr (sizeof(TS) == 8) {
            const v4d v = *(const v4d*)q;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) out[kk] = v[kk];
        } else {
            typedef float v4f __attribute__((ext_vector_type(4)));
            const v4f v = *(const v4f*)q;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) out[kk] = (double)v[kk];
        }
    };
    // Coupling blocks the owner of block s applies right after solving it:
    // (p, s - 1) and (p, s) for its blocks p = 2j + (s & 1) > s.  Loaded two
    // steps ahead into the other half of a double buffer (the owner's steps
    // alternate halves), right after the previous barrier.
    double adq[2][NJ][2][4];
    auto load_deferred = [&](int s) {
#pragma unroll
        for (int j = (s >> 1) + 1; j < NJ; ++j) {
            if (s > 0) lop4(2 * j + (s & 1), s - 1, adq[(s >> 1) & 1][j][0]);
            lop4(2 * j + (s & 1), s, adq[(s >> 1) & 1][j][1]);
        }
    };
    double ac[4];  // block (s + 1, s), applied by the owner of block s + 1
    auto load_critical = [&](int s) { lop4(s + 1, s, ac); };
    if (v == 0) {
        load_deferred(0);
    } else {
        load_critical(0);
        load_deferred(1);
    }
    v4d xp = {0.0, 0.0, 0.0, 0.0};  // x_{s-1}, not yet applied to the later own blocks
#pragma clang loop unroll(full)
    for (int s = 0; s < NBK; ++s) {
        const int par = s & 1, jo = s >> 1;  // owner parity, owner's fragment
        const bool own = v == par;
        if (own) {
            solve_diag16(Ds + s * 256, Xs[cg], fr[jo], g, c);
            Xb[par][cg][lane] = fr[jo];
        }
        __syncthreads();  // x_s published
        if (own) {
            // operands of this wave's next two steps: the critical update of
            // step s + 1 and the deferred updates of step s + 2
            if (s + 2 < NBK) {
                load_critical(s + 1);
                load_deferred(s + 2);
            }
            double (&ad)[NJ][2][4] = adq[(s >> 1) & 1];
            if (s > 0) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                    for (int j = jo + 1; j < NJ; ++j)
                        fr[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[j][0][kk], xp[kk], fr[j],
                                                                     0, 0, 0);
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int j = jo + 1; j < NJ; ++j)
                    fr[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[j][1][kk], fr[jo][kk], fr[j],
                                                                 0, 0, 0);
        } else if (s + 1 < NBK) {
            const v4d xb = Xb[par][cg][lane];
            const int jn = (s + 1) >> 1;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                fr[jn] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[kk], xb[kk], fr[jn], 0, 0, 0);
            xp = xb;
        }
    }
    if (colok) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * (2 * j + v) + g + 4 * r;
                if (FULL || row < rows) bp[row * br] = (TS)fr[j][r];
            }
    }
}

template <typename TS, int CG>
hipError_t leaf_ilv_dispatch(const TS* P, int64_t rows, TS* B, int64_t off, int64_t br, int64_t bc,
                             int64_t ncols, bool unit, hipStream_t s) {
    dim3 grid((unsigned)((ncols + 16 * CG - 1) / (16 * CG))), block(128 * CG);
    const bool full = rows == 256;
    if (unit && full)
        hipLaunchKernelGGL((leaf_ilv_kernel<TS, CG, true, true>), grid, block, 0, s, P, (int)rows,
                           B, off, br, bc, ncols);
    else if (unit)
        hipLaunchKernelGGL((leaf_ilv_kernel<TS, CG, true, false>), grid, block, 0, s, P, (int)rows,
                           B, off, br, bc, ncols);
    else if (full)
        hipLaunchKernelGGL((leaf_ilv_kernel<TS, CG, false, true>), grid, block, 0, s, P, (int)rows,
                           B, off, br, bc, ncols);
    else
        hipLaunchKernelGGL((leaf_ilv_kernel<TS, CG, false, false>), grid, block, 0, s, P,
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

// out[0] = max |T(i, i)|, out[1] = min |T(i, i)| over the k diagonal entries
// (a NaN entry makes both NaN).  One workgroup; max and min do not depend on
// the reduction order.
template <typename T>
__global__ __launch_bounds__(256) void diag_extremes_kernel(const T* __restrict__ a, int64_t off,
                                                            int64_t step, int64_t k,
                                                            double* __restrict__ out) {
    __shared__ double mx[256], mn[256];
    double hi = 0.0, lo = __builtin_inf();
    for (int64_t i = threadIdx.x; i < k; i += 256) {
        const double v = __builtin_fabs((double)a[off + i * step]);
        hi = (v > hi || v != v) ? v : hi;
        lo = (v < lo || v != v) ? v : lo;
    }
    mx[threadIdx.x] = hi;
    mn[threadIdx.x] = lo;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double h = mx[threadIdx.x + w], l = mn[threadIdx.x + w];
            if (h > mx[threadIdx.x] || h != h) mx[threadIdx.x] = h;
            if (l < mn[threadIdx.x] || l != l) mn[threadIdx.x] = l;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = mx[0];
        out[1] = mn[0];
    }
}

}  // namespace

hipError_t launch_diag_extremes(int dtype, const TriView& T, int64_t k, double* out,
                                hipStream_t s) {
    if (k <= 0) return hipSuccess;
    const int64_t step = T.tr + T.tc;  // (i, i) -> (i + 1, i + 1)
    if (dtype == 0)
        hipLaunchKernelGGL(diag_extremes_kernel<double>, dim3(1), dim3(256), 0, s,
                           (const double*)T.base, T.off, step, k, out);
    else
        hipLaunchKernelGGL(diag_extremes_kernel<float>, dim3(1), dim3(256), 0, s,
                           (const float*)T.base, T.off, step, k, out);
    return hipGetLastError();
}

hipError_t launch_pack_diag(int dtype, const TriView& T, int64_t m, int nb, int64_t first_blk,
                            int64_t nblk, bool unit, void* packed, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    const int64_t nn = (int64_t)nb * nb, stride = leaf_block_elems(nb);
    const unsigned gy = (unsigned)(nblk < 65535 ? nblk : 65535);
    dim3 grid((unsigned)((nn + 255) / 256), gy), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL(pack_diag_kernel<double>, grid, block, 0, s, (const double*)T.base,
                           T.off, T.tr, T.tc, m, nb, first_blk, nblk, unit ? 1 : 0, stride,
                           (double*)packed);
    else
        hipLaunchKernelGGL(pack_diag_kernel<float>, grid, block, 0, s, (const float*)T.base,
                           T.off, T.tr, T.tc, m, nb, first_blk, nblk, unit ? 1 : 0, stride,
                           (float*)packed);
    if (nb == 256) {
        dim3 fgrid(120, gy);
        if (dtype == 0)
            hipLaunchKernelGGL(pack_frag_kernel<double>, fgrid, block, 0, s, (double*)packed, nblk,
                               stride);
        else
            hipLaunchKernelGGL(pack_frag_kernel<float>, fgrid, block, 0, s, (float*)packed, nblk,
                               stride);
    }
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
                return leaf_ilv_dispatch<double, 2>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
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
                return leaf_ilv_dispatch<float, 2>(P, rows, b, off, B.br, B.bc, ncols, unit, s);
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
