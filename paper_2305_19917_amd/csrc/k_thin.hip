// Thin right-hand sides: the whole forward substitution as one dataflow
// launch.
//
// With few right-hand sides the split of Sec. IV leaves the GPU idle: every
// leaf is a serial chain on a handful of CUs and every update a small
// product, each a separate launch on the critical path.  Here a task (row
// block i of 64 rows, group of up to 64 right-hand sides) belongs to one
// workgroup of a cooperative launch (all workgroups resident at once).  It
// starts from its rows of B and, for j = 0, 1, ..., i - 1, waits until block
// j of its group is solved (a counter of solved blocks in global memory, read
// and raised with agent-scope atomics), stages X_j in LDS and subtracts
// L_ij X_j on the matrix cores (v_mfma_f64_16x16x4f64, one 16-row slice of
// the block per wave).  Then it solves its 64 x 64 diagonal block in
// row-scaled form (the block and its right-hand sides divided by the
// diagonal, correctly rounded; unit-diagonal substitution after), stores X_i
// and raises the counter.  The products of a block with the blocks solved
// long before run while the blocks just before it are still being solved,
// so the critical path is the chain of diagonal solves plus one product per
// block.  When the tasks outnumber the resident workgroups, a persistent
// grid takes them from a queue in dependency order.
//
// Waits are bounded: a workgroup that waits longer than its limit raises a
// global abort flag and writes NaN for its block; every other waiting
// workgroup sees the abort flag and does the same, so the launch always ends.
#include <hip/hip_runtime.h>

#include <atomic>
#include <type_traits>

#include "fdiv.h"
#include "kernels.h"

namespace redsea {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kTB = 64;     // rows per block
constexpr int kTCols = 64;  // right-hand sides per task at most
// Right-hand sides per group: up to 256 right-hand sides, groups of 16 on
// the row-parallel solve (the groups of one launch are independent solves
// that each read the triangle; at these widths that costs less than the
// slower 16-row-step solve of a wider group); wider B in groups of 64.
constexpr int64_t kThinRowParMax = 256;  // groups of 16 up to this width
inline int64_t thin_group_width(int64_t nrhs) { return nrhs <= kThinRowParMax ? 16 : kTCols; }
// flags: [0] the task queue, [kAbortAt] abort, [kGroupFlags + 32 g] the
// solved-block counter of column group g (each in a cache line of its own)
constexpr int kAbortAt = 32;
constexpr int kGroupFlags = 64;
constexpr int kMaxDevices = 64;
constexpr int kStager = 4;             // the wave that waits for and stages solved blocks
constexpr int kThreads = 64 * (kStager + 1);

// Solved blocks travel through agent-scope stores and loads (written
// through to memory; a consumer's L2 never holds a line of X_j from before
// it was solved, since only block j's own workgroup reads those rows
// earlier).  Flags are read and raised with agent-scope read-modify-write
// atomics, which every XCD sees at once; a plain or agent-scope load of a
// flag can keep returning the consumer XCD's stale copy of its line until
// that line is evicted.  Acquire / release operations would be correct too,
// but their cache maintenance (an L2 invalidation per poll) is slower.  A
// block's stores are complete (waited for, then a workgroup barrier) before
// its flag is raised, and a consumer loads the block only after it has seen
// the flag.
template <typename T>
__device__ __forceinline__ T coherent_load(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void coherent_store(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// `zero` is a kernel argument equal to 0, so the compiler cannot turn the
// read-modify-write into a plain load
__device__ __forceinline__ int flag_read(int* p, int zero) {
    return __hip_atomic_fetch_add(p, zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_raise(int* p) {
    __hip_atomic_fetch_add(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void thin_flags_kernel(int* flags, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * 256)
        flags[i] = 0;
}

__device__ __forceinline__ double bcast_lane(double v, int src) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// a / d correctly rounded (the fast form where its guard holds; the IEEE
// division only on the rare lanes where it does not)
__device__ __forceinline__ double div_rn(double a, double d, double r) {
    bool ok;
    double q = div_rn_fast(a, d, r, div_fast_divisor(d), ok);
    if (__builtin_expect(!ok, 0)) q = a / d;
    return q;
}

// One task: a 64-row block of one group of gw right-hand sides (flags as
// laid out above; the blocks of a group finish in order, each needing its
// predecessor, so one counter per group says how many are solved).  Waves
// 0-3 own the block's rows; wave 4 (kStager) waits for solved blocks and
// stages them in LDS.  CPW > 0: the diagonal block's substitution runs with
// its rows across the lanes, CPW right-hand sides per wave; CPW = 0: in
// 16-row steps with one lane per right-hand side.
template <typename T, bool UNIT, int NCG, int CPW, bool PERSIST>
__global__ __launch_bounds__(kThreads, 1) void thin_kernel(TriView L, RhsView B, int64_t n,
                                                           int64_t nrhs, int ngroups, int gw, int* flags,
                                                           int64_t spin_limit, int zero) {
    constexpr int kXPer = kTB * 16 * NCG / 256;  // elements of a row block per row thread
    constexpr bool ROWPAR = CPW > 0;
    __shared__ double Xs[kTB][kTCols + 2];  // X_j of an update, then this block's rows
    __shared__ double Ls[kTB][kTB + 1];     // D^-1 L_ii strictly below the diagonal, else zero
    __shared__ double Ds[kTB], Rs[kTB];     // the diagonal and its reciprocals
    __shared__ int s_abort;
    const T* A = (const T*)L.base;
    T* Bp = (T*)B.base;
    // the wave index as a wave-uniform value: every branch on it is a scalar
    // branch, so a wave runs only its own role's code (no exec-masked pass
    // through the other's barriers and memory waits)
    const int tid0 = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid0 >> 6);
    const bool rows_wave = w < kStager;  // waves 0-3
    __shared__ int s_task;
    int* queue = flags;
    int* abort_flag = flags + kAbortAt;
    const int64_t nblk = (n + kTB - 1) / kTB;
    const int64_t ntasks = nblk * ngroups;
    auto tget = [&](int64_t r, int64_t col) -> double {
        return (double)A[L.off + r * L.tr + col * L.tc];
    };
    // Tasks (row block i, column group grp) are claimed in the order
    // t = i * ngroups + grp.  A task depends only on earlier row blocks of its
    // own group, which were claimed before it by resident workgroups, so the
    // earliest unfinished task can always proceed.
    // PERSIST: a grid of the resident workgroups loops over the queue;
    // otherwise every task has a workgroup of its own (t = blockIdx.x, the
    // same order) and the body runs once
  for (int64_t pass = 0;; ++pass) {
    int64_t t;
    if constexpr (PERSIST) {
        if (tid0 == 0) s_task = __hip_atomic_fetch_add(queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        t = s_task;
        __syncthreads();  // s_task is read before it is claimed again
    } else {
        t = pass == 0 ? (int64_t)blockIdx.x : ntasks;
    }
    if (t >= ntasks) break;  // uniform over the workgroup
    // the lane indexes as an opaque value per task: the address arithmetic
    // derived from them is recomputed in each pass instead of being hoisted
    // out of the loop and held in registers for the whole launch
    int tidv = tid0;
    asm volatile("" : "+v"(tidv));
    const int tid = tidv, lane = tid & 63, g = lane >> 4, c = lane & 15;
    const int64_t i = t / ngroups, grp = t % ngroups;
    const int64_t r0 = i * kTB;
    const int rows = (int)(n - r0 < kTB ? n - r0 : kTB);
    const int ncols = (int)(nrhs - grp * gw < gw ? nrhs - grp * gw : gw);
    const int64_t boff = B.off + grp * gw * B.bc;
    int* progress = flags + kGroupFlags + 32 * grp;  // solved blocks of this group
    auto bptr = [&](int64_t r, int64_t col) -> T* { return Bp + boff + r * B.br + col * B.bc; };

    // 1. Work that waits for nothing, done while earlier blocks are solved.
    // This wave's 16 rows of the block, in the accumulator layout (lane l,
    // register r: row g + 4r, column c of column group cg).
    v4d acc[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + g + 4 * r, col = 16 * cg + c;
            acc[cg][r] = (rows_wave && row < rows && col < ncols) ? (double)*bptr(r0 + row, col) : 0.0;
        }
    // The diagonal block (the identity past the order n), each row divided
    // by its diagonal element: the unit lower triangular D^-1 L_ii.
    if (tid < kTB) {
        const double d = (UNIT || tid >= rows) ? 1.0 : tget(r0 + tid, r0 + tid);
        Ds[tid] = d;
        Rs[tid] = 1.0 / d;
    }
    if (tid == 0) s_abort = 0;
    double dv[16];
    if (rows_wave) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k, rr = e % kTB, cc = e / kTB;
            dv[k] = (rr < rows && cc < rr) ? tget(r0 + rr, r0 + cc) : 0.0;
        }
    }
    __syncthreads();
    if (rows_wave) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k, rr = e % kTB, cc = e / kTB;
            Ls[rr][cc] = UNIT ? dv[k] : div_rn(dv[k], Ds[rr], Rs[rr]);
        }
    }
    __syncthreads();

    // 2. acc -= L_ij X_j for j < i, as each block is solved.  The row waves
    // hold the operands of L_ij (their 16 rows, 16 steps of four columns) in
    // a ring of three register buffers, loaded two updates ahead: the loads
    // take several microseconds, which this hides behind the block solves.
    // The stager's queue of memory operations holds only its polls and the
    // loads of X_j, so neither ever waits behind a load of L.
    // The loads are unconditional and untouched until their use, so all 16
    // stay in flight together: a row past the order n reads row n - 1
    // instead, which only feeds accumulator rows that are never stored.
    const int64_t arow = r0 + (16 * w + c < rows ? 16 * w + c : rows - 1);
    auto load_a = [&](int64_t j, T(&a)[16]) {
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) a[ks] = A[L.off + arow * L.tr + (j * kTB + 4 * ks + g) * L.tc];
    };
    // The prefetch is unconditional (past the last update it reloads block
    // i - 1): with a conditional one the compiler's wait before the products
    // has to cover the path without it, and then waits for the fresh loads.
    T ab0[16], ab1[16], ab2[16];  // L_ij is in buffer j mod 3
    // The two roles run separate loops (a wave takes one of them by a scalar
    // branch), each with the same two barriers per update; an abandoned wait
    // ends both after the first.
    bool aborted = false;
    if (!rows_wave) {
        int64_t known = 0;  // blocks known to be solved
        for (int64_t j = 0; j < i; ++j) {
            if (j >= known) {
                // Wait until block j is solved.  Only the next block's
                // workgroup is on the critical path; one that is d blocks
                // further down has d block solves of slack and polls about
                // every d * 0.4 us.  Every poll is an atomic on the one
                // counter, so this keeps its cache line free for the critical
                // reader.  The abort flag is looked at every 64 polls.
                const int64_t dist = i - j - 1;
                const int naps = (int)(dist < 16 ? dist : 16);
                int64_t spins = 0;
                for (;;) {
                    int v = 0;
                    if (lane == 0) v = flag_read(progress, zero);
                    v = __builtin_amdgcn_readfirstlane(v);
                    if (v > j) {
                        known = v;
                        break;
                    }
                    if ((++spins & 63) == 0) {
                        int ab = 0;
                        if (lane == 0) ab = flag_read(abort_flag, zero);
                        ab = __builtin_amdgcn_readfirstlane(ab);
                        if (ab != 0 || spins > spin_limit) {
                            if (lane == 0) {
                                flag_raise(abort_flag);
                                s_abort = 1;
                            }
                            break;
                        }
                    }
                    __builtin_amdgcn_s_sleep(1);
                    for (int t = 0; t < naps; ++t) __builtin_amdgcn_s_sleep(16);
                }
            }
            if (known > j) {
                // -X_j into LDS: lane = row, up to 32 loads in flight at once
                const int64_t gr = j * kTB + lane;
#pragma unroll
                for (int k0 = 0; k0 < 16 * NCG; k0 += 32) {
                    constexpr int kChunk = 16 * NCG < 32 ? 16 * NCG : 32;
                    double xv[kChunk];
#pragma unroll
                    for (int k = 0; k < kChunk; ++k)
                        xv[k] = (k0 + k < ncols && gr < n) ? (double)coherent_load(bptr(gr, k0 + k)) : 0.0;
#pragma unroll
                    for (int k = 0; k < kChunk; ++k) Xs[lane][k0 + k] = -xv[k];
                }
            }
            __syncthreads();  // X_j staged, or the wait abandoned
            if (s_abort != 0) {
                aborted = true;
                break;
            }
            __syncthreads();  // Xs is overwritten next
        }
    } else if (i > 0) {
        // one update: the prefetch of L_{i,j+2} into `pre`, then
        // acc += L_ij (-X_j) with L_ij from `cur`
        auto update = [&](int64_t j, T(&cur)[16], T(&pre)[16]) -> bool {
            load_a(j + 2 < i ? j + 2 : i - 1, pre);
            __syncthreads();  // X_j staged, or the wait abandoned
            if (s_abort != 0) return false;
            // the B operands read from LDS four steps at a time, ahead of
            // their products
#pragma unroll
            for (int k0 = 0; k0 < 16; k0 += 4) {
                double xb[4][NCG];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int cg = 0; cg < NCG; ++cg) xb[ks][cg] = Xs[4 * (k0 + ks) + g][16 * cg + c];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int cg = 0; cg < NCG; ++cg)
                        acc[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)cur[k0 + ks], xb[ks][cg],
                                                                      acc[cg], 0, 0, 0);
            }
            __syncthreads();  // Xs is overwritten next
            return true;
        };
        load_a(0, ab0);
        load_a(i > 1 ? 1 : 0, ab1);
        for (int64_t j = 0; j < i; j += 3) {
            if (!update(j, ab0, ab2) || (j + 1 < i && !update(j + 1, ab1, ab0)) ||
                (j + 2 < i && !update(j + 2, ab2, ab1))) {
                aborted = true;
                break;
            }
        }
    }

    // 3. The diagonal block: L_ii X_i = R_i as (D^-1 L_ii) X_i = D^-1 R_i, the
    // right-hand sides divided by the diagonal first (correctly rounded), so
    // each step of the substitution is a single fused multiply-add.
    if (!UNIT && rows_wave) {
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * w + g + 4 * r;
                acc[cg][r] = div_rn(acc[cg][r], Ds[row], Rs[row]);
            }
    }
    if constexpr (ROWPAR) {
        // wave w solves right-hand sides CPW w .. CPW w + CPW - 1, lane = row:
        // after row r is final it is broadcast, and every row below subtracts
        // its multiple (the rows at or above r multiply by the zero of
        // D^-1 L_ii there)
        if (rows_wave) {
#pragma unroll
            for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
                for (int r = 0; r < 4; ++r) Xs[16 * w + g + 4 * r][16 * cg + c] = acc[cg][r];
        }
        __syncthreads();
        if (rows_wave && CPW * w < ncols && !aborted) {
            // this lane's row of -D^-1 L_ii in registers: the substitution
            // then reads no memory
            double lrow[kTB - 1];
#pragma unroll
            for (int r = 0; r < kTB - 1; ++r) lrow[r] = -Ls[lane][r];
            double y[CPW];
#pragma unroll
            for (int k = 0; k < CPW; ++k) y[k] = Xs[lane][CPW * w + k];
#pragma unroll
            for (int r = 0; r < kTB - 1; ++r)
#pragma unroll
                for (int k = 0; k < CPW; ++k) y[k] = __builtin_fma(lrow[r], bcast_lane(y[k], r), y[k]);
#pragma unroll
            for (int k = 0; k < CPW; ++k) Xs[lane][CPW * w + k] = y[k];
        }
        __syncthreads();
    } else {
        // four 16-row steps: wave s hands its rows to LDS, wave 0 solves
        // them by substitution in axpy order (lane = right-hand side), the
        // row waves below subtract the product of their 16 x 16 block of
        // D^-1 L_ii with the new unknowns on the matrix cores
        const bool live = lane < ncols;
#pragma unroll
        for (int s = 0; s < kTB / 16; ++s) {
            const int b0 = 16 * s;
            if (w == s) {
#pragma unroll
                for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
                    for (int r = 0; r < 4; ++r) Xs[b0 + g + 4 * r][16 * cg + c] = acc[cg][r];
            }
            __syncthreads();
            if (w == 0 && !aborted) {
                double y[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) y[r] = live ? Xs[b0 + r][lane] : 0.0;
#pragma unroll
                for (int r = 0; r < 16; ++r)
#pragma unroll
                    for (int q = r + 1; q < 16; ++q) y[q] = __builtin_fma(-Ls[b0 + q][b0 + r], y[r], y[q]);
#pragma unroll
                for (int r = 0; r < 16; ++r) Xs[b0 + r][lane] = y[r];
            }
            __syncthreads();
            if (rows_wave && w > s) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const double a = -Ls[16 * w + c][b0 + 4 * ks + g];
#pragma unroll
                    for (int cg = 0; cg < NCG; ++cg)
                        acc[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            a, Xs[b0 + 4 * ks + g][16 * cg + c], acc[cg], 0, 0, 0);
                }
            }
        }
    }
    // X_i (NaN for an aborted block), stored along rows
    if (rows_wave) {
        const T nan = (T)__builtin_nan("");
#pragma unroll
        for (int k = 0; k < kXPer; ++k) {
            const int e = tid + 256 * k, rr = e % kTB, col = e / kTB;
            if (rr < rows && col < ncols)
                coherent_store(bptr(r0 + rr, col), aborted ? nan : (T)Xs[rr][col]);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this thread's stores are complete
    __syncthreads();                // ... and every other thread's
    if (tid == 0 && !aborted) flag_raise(progress);
  }
}

template <typename T, bool UNIT, int NCG, int CPW>
hipError_t thin_launch(const TriView& L, const RhsView& B, int64_t n, int64_t nrhs, int* flags,
                       hipStream_t s) {
    const int64_t nblk = (n + kTB - 1) / kTB;
    const int64_t gw = thin_group_width(nrhs);
    const int ngroups = (int)((nrhs + gw - 1) / gw);
    const int64_t ntasks = nblk * ngroups;
    const void* fn1 = (const void*)thin_kernel<T, UNIT, NCG, CPW, false>;
    const void* fnp = (const void*)thin_kernel<T, UNIT, NCG, CPW, true>;
    // resident workgroups per CU, asked once per device (the first query
    // costs more than a whole small solve)
    static std::atomic<int> per_cu_of[kMaxDevices];
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return hipErrorInvalidValue;
    int per_cu = per_cu_of[dev].load(std::memory_order_relaxed);
    if (per_cu == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fnp, kThreads, 0) != hipSuccess)
            return hipErrorInvalidValue;
        per_cu_of[dev].store(per_cu, std::memory_order_relaxed);
    }
    if (per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
    // every task a workgroup of its own when they all fit at once (one
    // column group: the whole latency chain in flight), else a persistent
    // grid of the resident workgroups working through the queue
    const int64_t resident = (int64_t)per_cu * cus;
    const int64_t grid = ntasks < resident ? ntasks : resident;
    const int64_t cnt = thin_flag_count(n, nrhs);
    hipLaunchKernelGGL(thin_flags_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       flags, cnt);
    const hipError_t fe = hipGetLastError();  // never run the solve on stale counters
    if (fe != hipSuccess) return fe;
    TriView l = L;
    RhsView b = B;
    int64_t nn = n, nr = nrhs, spin = (int64_t)1 << 22;
    int ng = ngroups, gwi = (int)gw;
    int* fl = flags;
    int zero = 0;
    void* args[] = {&l, &b, &nn, &nr, &ng, &gwi, &fl, &spin, &zero};
    return hipLaunchCooperativeKernel(grid == ntasks ? fn1 : fnp, dim3((unsigned)grid), dim3(kThreads),
                                      args, 0, s);
}

template <typename T, bool UNIT>
hipError_t thin_by_width(const TriView& L, const RhsView& B, int64_t n, int64_t nrhs, int* flags,
                         hipStream_t s) {
    if (nrhs <= 4) return thin_launch<T, UNIT, 1, 1>(L, B, n, nrhs, flags, s);
    if (nrhs <= 8) return thin_launch<T, UNIT, 1, 2>(L, B, n, nrhs, flags, s);
    if (nrhs <= kThinRowParMax) return thin_launch<T, UNIT, 1, 4>(L, B, n, nrhs, flags, s);
    return thin_launch<T, UNIT, 4, 0>(L, B, n, nrhs, flags, s);  // groups of 64
}

}  // namespace

int64_t thin_flag_count(int64_t, int64_t nrhs) {
    const int64_t gw = thin_group_width(nrhs);
    return kGroupFlags + 32 * ((nrhs + gw - 1) / gw);
}

hipError_t launch_thin(int dtype, const TriView& L, const RhsView& B, int64_t n, int64_t nrhs,
                       bool unit, int* flags, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    if (dtype == 0)
        return unit ? thin_by_width<double, true>(L, B, n, nrhs, flags, s)
                    : thin_by_width<double, false>(L, B, n, nrhs, flags, s);
    return unit ? thin_by_width<float, true>(L, B, n, nrhs, flags, s)
                : thin_by_width<float, false>(L, B, n, nrhs, flags, s);
}

}  // namespace redsea
