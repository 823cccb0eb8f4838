// Persistent batched solver: many independent triangular systems of uneven
// order and right-hand-side count in one launch (the solve of Sec. IV per
// system).
//
// Work is a list of tasks (system, tile of up to 16 right-hand sides) in one
// queue per XCD (a system's tiles in one queue, each queue longest-first).
// Every wave repeatedly claims the next task, from its own XCD's queue first
// (the tiles of a system then share its triangle in that XCD's L2), and
// solves it alone, left-looking over 16-row blocks with its
// 16 x 16 block of the right-hand sides held in the v_mfma_f64_16x16x4f64
// accumulator layout (lane l, register r = row l/16 + 4r, column l % 16):
//   acc = alpha B_p;  acc -= L_pq X_q for every solved block q < p on the
//   matrix cores (operands for q+1 are requested while q is multiplied);
//   then the 16 x 16 diagonal block is solved by substitution in every lane
//   (one correctly rounded division per row, from a reciprocal of the
//   diagonal prepared while the matrix cores run) and X_p is stored.
// A task never depends on another, so the result does not depend on which
// wave ran it.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "batched.h"
#include "fdiv.h"

namespace redsea {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void batch_reset_kernel(int* counters, int* info, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        info[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < kBatchCounterInts) counters[threadIdx.x] = 0;
}

template <typename TS, bool UNIT, int W, int D>
__global__ __launch_bounds__(256) void batched_kernel(const BatchSys* __restrict__ sys,
                                                      const BatchTask* __restrict__ tasks,
                                                      BatchQueues queues, int* __restrict__ counters,
                                                      int* __restrict__ info, double alpha) {
    // The first QL solved blocks of a wave's task stay in LDS, in B-operand
    // order (k-slice kk of block q: XL[w][q][G][kk][lane] = X_q(4 kk + g, c),
    // which is register kk of the solved accumulator fragment), so the
    // left-looking products read them on chip instead of from memory (56 or
    // 48 KB per workgroup: two workgroups still fit per CU).
    constexpr int QL = 7 / W;
    __shared__ double XL[4][QL][W][4][64];
    __shared__ double Xs[4][W][16][17];  // per-wave gather buffer, one per column group
    __shared__ double Ls[4][16 * 16];    // per-wave diagonal block, (j, i) at [i*16 + j]
    __shared__ double Rs[4][16];         // per-wave 1 / diagonal
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    // the group whose column c this lane solves in the substitution (the four
    // row slices g of a column split evenly over the W groups)
    const int sg = W == 1 ? 0 : (g >> 1);
    const int home = (int)(blockIdx.x % kBatchQueues);  // this workgroup's XCD
    int visited = 0;                                     // queues found empty
    for (;;) {
        const int q = (home + visited) % kBatchQueues;
        int t = 0;
        if (lane == 0) t = atomicAdd(counters + 32 * q, 1);
        t = __shfl(t, 0);
        if (t >= queues.count[q]) {  // uniform over the wave
            if (++visited == kBatchQueues) break;
            continue;
        }
        const BatchTask task = tasks[queues.start[q] + t];
        const BatchSys S = sys[task.sys];
        const int64_t k = S.k, c0 = task.c0;
        bool colok[W];
        int64_t bcol[W];
#pragma unroll
        for (int G = 0; G < W; ++G) {
            colok[G] = c0 + 16 * G + c < S.nrhs;
            bcol[G] = S.b_off + (colok[G] ? c0 + 16 * G + c : c0) * S.bc;
        }
        const int nblk = (int)((k + 15) / 16);
        // Operand reads are unconditional, through global-address-space
        // pointers, with clamped indices: a read past the order or past the
        // task's columns fetches a valid element (row k - 1, the task's first
        // column) that only feeds accumulator rows or columns that are never
        // stored.  Every value stays untouched until its use (the sign of L
        // is the MFMA's A negation, alpha is applied after the products), so
        // a step's loads are in flight together and the ring of D operand
        // sets is D deep.  (A predicated or post-processed load makes the
        // compiler wait for it right where it is issued.)
        typedef const __attribute__((address_space(1))) TS* GConst;
        typedef __attribute__((address_space(1))) TS* GMut;
        const GConst Ag = (GConst)S.a;
        const GConst Bg = (GConst)S.b;
        const GMut Bw = (GMut)S.b;
        auto bidx = [&](int G, int64_t row) -> int64_t { return bcol[G] + (row < k ? row : k - 1) * S.br; };
        auto aidx = [&](int64_t row, int64_t col) -> int64_t {
            return S.a_off + (row < k ? row : k - 1) * S.tr + (col < k ? col : k - 1) * S.tc;
        };
        int bad = 0;
        for (int p = 0; p < nblk; ++p) {
            v4d acc[W];
            TS bv[W][4];  // alpha B_p, applied after the products
            TS dv[4];     // this lane's entries of the diagonal block: rows g + 4r, column c
#pragma unroll
            for (int G = 0; G < W; ++G) {
                acc[G] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int r = 0; r < 4; ++r) bv[G][r] = Bg[bidx(G, 16 * p + g + 4 * r)];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) dv[r] = Ag[aidx(16 * p + g + 4 * r, 16 * p + c)];
            if (alpha != 0.0) {  // BLAS: alpha = 0 gives B := 0
                // acc -= L_pq X_q, q < p, on the matrix cores; operand set d of
                // the ring holds step q = q0 + d and is reloaded for step
                // q + D right after its MFMAs (past the last step it reloads
                // step p - 1, unused); each block of L feeds the W groups
                TS xa[D][W][4], aa[D][4];
                auto load_set = [&](int d, int q) {
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
#pragma unroll
                        for (int G = 0; G < W; ++G) xa[d][G][kk] = Bg[bidx(G, 16 * q + 4 * kk + g)];
                        aa[d][kk] = Ag[aidx(16 * p + c, 16 * q + 4 * kk + g)];
                    }
                };
                if (p > 0) {
                    // (a) the solved blocks kept in LDS: only L is loaded
                    const int pl = p < QL ? p : QL;
                    {
                        TS al[D][4];
                        auto load_l = [&](int d, int q) {
#pragma unroll
                            for (int kk = 0; kk < 4; ++kk) al[d][kk] = Ag[aidx(16 * p + c, 16 * q + 4 * kk + g)];
                        };
#pragma unroll
                        for (int d = 0; d < D; ++d) load_l(d, d < pl ? d : pl - 1);
                        for (int q0 = 0; q0 < pl; q0 += D) {
#pragma unroll
                            for (int d = 0; d < D; ++d) {
                                const int q = q0 + d;
                                if (q < pl) {  // uniform over the wave
                                    double xl[4][W];
#pragma unroll
                                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                                        for (int G = 0; G < W; ++G) xl[kk][G] = XL[w][q][G][kk][lane];
#pragma unroll
                                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                                        for (int G = 0; G < W; ++G)
                                            acc[G] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                                (double)al[d][kk], xl[kk][G], acc[G], 0, 0,
                                                1 /* negate A */);
                                }
                                load_l(d, q + D < pl ? q + D : pl - 1);
                            }
                        }
                    }
                    // (b) the rest, X from memory through the ring
                    if (p > pl) {
#pragma unroll
                        for (int d = 0; d < D; ++d) load_set(d, pl + d < p ? pl + d : p - 1);
                        for (int q0 = pl; q0 < p; q0 += D) {
#pragma unroll
                            for (int d = 0; d < D; ++d) {
                                const int q = q0 + d;
                                if (q < p) {  // uniform over the wave
#pragma unroll
                                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                                        for (int G = 0; G < W; ++G)
                                            acc[G] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                                (double)aa[d][kk], (double)xa[d][G][kk], acc[G], 0, 0,
                                                1 /* negate A */);
                                }
                                load_set(d, q + D < p ? q + D : p - 1);
                            }
                        }
                    }
                }
#pragma unroll
                for (int G = 0; G < W; ++G)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[G][r] = __builtin_fma(alpha, (double)bv[G][r], acc[G][r]);
                // diagonal block (identity past the order) and the reciprocals
                // of its diagonal
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = g + 4 * r;  // row of the block, column c
                    const int64_t gi = 16 * p + i;
                    double v = 0.0;
                    if (gi >= k) v = (i == c) ? 1.0 : 0.0;
                    else if (i == c) v = UNIT ? 1.0 : (double)dv[r];
                    else if (i > c) v = (double)dv[r];
                    Ls[w][c * 16 + i] = v;
                    if (!UNIT && i == c) Rs[w][c] = 1.0 / v;
                }
                // the columns' rows of the block
#pragma unroll
                for (int G = 0; G < W; ++G)
#pragma unroll
                    for (int r = 0; r < 4; ++r) Xs[w][G][g + 4 * r][c] = acc[G][r];
                wave_sync();
                // substitution (axpy order), pipelined by one row as in the
                // leaf solver, column c of group sg in this lane; the fast
                // divisions are redone in IEEE arithmetic for the whole block
                // if any operand of the wave left their guard (same result
                // wherever it held)
                double y[16];
                auto subst = [&](auto fast) {
                    double dg[16], rd[16], cur[16], nxt[16];
                    bool dok[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        y[i] = Xs[w][sg][i][c];
                        if (!UNIT) {
                            dg[i] = Ls[w][i * 16 + i];
                            rd[i] = Rs[w][i];
                            dok[i] = div_fast_divisor(dg[i]);
                        }
                    }
                    bool ok = true;
                    auto divide = [&](double a, int i) -> double {
                        if (UNIT) return a;
                        if (!decltype(fast)::value) return a / dg[i];
                        bool oki;
                        const double q = div_rn_fast(a, dg[i], rd[i], dok[i], oki);
                        ok = ok && oki;
                        return q;
                    };
#pragma unroll
                    for (int j = 1; j < 16; ++j) cur[j] = Ls[w][j];
                    double x = divide(y[0], 0);
                    y[0] = x;
#pragma unroll
                    for (int i = 0; i + 1 < 16; ++i) {
#pragma unroll
                        for (int j = i + 2; j < 16; ++j) nxt[j] = Ls[w][(i + 1) * 16 + j];
                        const double yn = __builtin_fma(-cur[i + 1], x, y[i + 1]);
                        const double xn = divide(yn, i + 1);
#pragma unroll
                        for (int j = i + 2; j < 16; ++j) y[j] = __builtin_fma(-cur[j], x, y[j]);
                        y[i + 1] = xn;
                        x = xn;
#pragma unroll
                        for (int j = i + 1; j < 16; ++j) asm volatile("" : "+v"(y[j]));
                        asm volatile("" ::: "memory");
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int j = i + 2; j < 16; ++j) cur[j] = nxt[j];
                    }
                    return ok;
                };
                if (!__all(subst(std::true_type()))) subst(std::false_type());
                if (W == 1) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double v01 = g == 0 ? y[4 * r] : y[4 * r + 1];
                        const double v23 = g == 2 ? y[4 * r + 2] : y[4 * r + 3];
                        acc[0][r] = g < 2 ? v01 : v23;
                    }
                } else {
                    // each group's solved column goes back through LDS to the
                    // accumulator layout of both groups
                    wave_sync();
                    if ((g & 1) == 0)
#pragma unroll
                        for (int i = 0; i < 16; ++i) Xs[w][sg][i][c] = y[i];
                    wave_sync();
#pragma unroll
                    for (int G = 0; G < W; ++G)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[G][r] = Xs[w][G][g + 4 * r][c];
                }
                wave_sync();  // Xs and Ls are reused by the next block
            }
            if (p < QL) {
                // the solved block for the later products, as stored (rounded
                // to the system's type: the same bits a read from memory gives)
#pragma unroll
                for (int G = 0; G < W; ++G)
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) XL[w][p][G][kk][lane] = (double)(TS)acc[G][kk];
            }
#pragma unroll
            for (int G = 0; G < W; ++G)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = 16 * p + g + 4 * r;
                    if (colok[G] && row < k) {
                        const TS v = (TS)acc[G][r];
                        Bw[bcol[G] + row * S.br] = v;
                        if (!__builtin_isfinite((double)v)) bad = 1;
                    }
                }
        }
        // the stores of this task are visible to its own later loads (same
        // wave, program order); flag a non-finite result of the system
        if (__any(bad) && lane == 0) atomicOr(&info[task.sys], 4);
    }
}

}  // namespace

hipError_t launch_batch_reset(int* counters, int* info, int64_t count, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(batch_reset_kernel, dim3((unsigned)blocks), dim3(256), 0, s, counters, info,
                       count);
    return hipGetLastError();
}

template <int W, int D>
void launch_batched_wd(int dtype, bool unit, const BatchSys* sys, const BatchTask* tasks,
                       const BatchQueues& qs, int* counters, int* info, double alpha, int grid,
                       hipStream_t s) {
    if (dtype == 0) {
        if (unit)
            hipLaunchKernelGGL((batched_kernel<double, true, W, D>), dim3(grid), dim3(256), 0, s,
                               sys, tasks, qs, counters, info, alpha);
        else
            hipLaunchKernelGGL((batched_kernel<double, false, W, D>), dim3(grid), dim3(256), 0, s,
                               sys, tasks, qs, counters, info, alpha);
    } else {
        if (unit)
            hipLaunchKernelGGL((batched_kernel<float, true, W, D>), dim3(grid), dim3(256), 0, s,
                               sys, tasks, qs, counters, info, alpha);
        else
            hipLaunchKernelGGL((batched_kernel<float, false, W, D>), dim3(grid), dim3(256), 0, s,
                               sys, tasks, qs, counters, info, alpha);
    }
}

hipError_t launch_batched(int dtype, bool unit, int groups, int depth, const BatchSys* sys,
                          const BatchTask* tasks, const BatchQueues& queues, int* counters,
                          int* info, double alpha, int grid, hipStream_t s) {
#define REDSEA_BATCHED_CASE(W, D)                                                              \
    if (groups == W && depth == D) {                                                           \
        launch_batched_wd<W, D>(dtype, unit, sys, tasks, queues, counters, info, alpha, grid, s); \
        return hipGetLastError();                                                              \
    }
    REDSEA_BATCHED_CASE(1, 1)
    REDSEA_BATCHED_CASE(1, 2)
    REDSEA_BATCHED_CASE(1, 4)
    REDSEA_BATCHED_CASE(2, 1)
    REDSEA_BATCHED_CASE(2, 2)
    REDSEA_BATCHED_CASE(2, 4)
#undef REDSEA_BATCHED_CASE
    return hipErrorInvalidValue;
}

}  // namespace redsea
