// Thin right-hand sides (up to 64): the whole forward substitution as one
// persistent dataflow launch.
//
// With few right-hand sides the split of Sec. IV leaves the GPU idle: every
// leaf is a serial chain on a handful of CUs and every update a small
// product, each a separate launch on the critical path.  Here row block i
// (64 rows) belongs to workgroup i of a cooperative launch (all workgroups
// resident at once).  The workgroup starts from its rows of B and, for j = 0,
// 1, ..., i - 1, waits until block j is solved (a readiness flag in global
// memory, agent-scope acquire / release atomics), stages X_j in LDS and
// subtracts L_ij X_j on the matrix cores (v_mfma_f64_16x16x4f64, one 16-row
// slice of the block per wave).  Then it solves its 64 x 64 diagonal block by
// substitution in axpy order, one lane per right-hand side, each unknown the
// correctly rounded quotient (fdiv.h), stores X_i and raises its flag.  The
// products of a block with the blocks solved long before run while the
// blocks just before it are still being solved, so the critical path is the
// chain of diagonal solves plus one product per block.
//
// Waits are bounded: a workgroup that waits longer than its limit (which only
// happens when the device cannot run all workgroups at once) raises a global
// abort flag, writes NaN for its block and publishes it; every other waiting
// workgroup sees the abort flag and does the same, so the launch always ends.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fdiv.h"
#include "kernels.h"

namespace redsea {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kTB = 64;     // rows per block
constexpr int kTCols = 64;  // right-hand sides at most

__device__ __forceinline__ int flag_acquire(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_release(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void thin_flags_kernel(int* flags, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * 256)
        flags[i] = 0;
}

// flags[0 .. nblk) readiness, flags[nblk] abort.
template <typename T, bool UNIT, int NCG>
__global__ __launch_bounds__(256, 1) void thin_kernel(TriView L, RhsView B, int64_t n, int ncols,
                                                      int* flags, int64_t spin_limit) {
    __shared__ double Xs[kTB][kTCols + 2];  // X_j of an update, then this block's rows
    __shared__ double Ls[kTB][kTB + 1];     // the diagonal block, Ls[row][col]
    __shared__ double Rs[kTB];              // 1 / diagonal
    __shared__ int s_go;
    const T* A = (const T*)L.base;
    T* Bp = (T*)B.base;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
    const int64_t nblk = (n + kTB - 1) / kTB;
    const int64_t i = blockIdx.x;
    const int64_t r0 = i * kTB;
    const int rows = (int)(n - r0 < kTB ? n - r0 : kTB);
    int* abort_flag = flags + nblk;
    auto tget = [&](int64_t r, int64_t col) -> double {
        return (double)A[L.off + r * L.tr + col * L.tc];
    };
    auto bptr = [&](int64_t r, int64_t col) -> T* { return Bp + B.off + r * B.br + col * B.bc; };

    // this wave's 16 rows of the block, in the accumulator layout (lane l,
    // register r: row g + 4r, column c of column group cg)
    v4d acc[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + g + 4 * r, col = 16 * cg + c;
            acc[cg][r] = (row < rows && col < ncols) ? (double)*bptr(r0 + row, col) : 0.0;
        }

    bool aborted = false;
    for (int64_t j = 0; j < i; ++j) {
        if (tid == 0) {
            int go = 1;
            int64_t spins = 0;
            while (flag_acquire(flags + j) == 0) {
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                    ++spins > spin_limit) {
                    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    go = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            s_go = go;
        }
        __syncthreads();
        if (!s_go) {  // uniform over the workgroup (read after the barrier)
            aborted = true;
            break;
        }
        // X_j into LDS (rows along consecutive threads)
        for (int e = tid; e < kTB * 16 * NCG; e += 256) {
            const int kk = e % kTB, col = e / kTB;
            const int64_t gr = j * kTB + kk;
            Xs[kk][col] = (col < ncols && gr < n) ? (double)*bptr(gr, col) : 0.0;
        }
        __syncthreads();
        // acc -= L_ij X_j in 16 steps of four columns of L_ij
        const int64_t arow = r0 + 16 * w + c;
        const bool arow_ok = 16 * w + c < rows;
#pragma unroll 4
        for (int ks = 0; ks < 16; ++ks) {
            const int64_t acol = j * kTB + 4 * ks + g;
            const double a = (arow_ok && acol < n) ? -tget(arow, acol) : 0.0;
#pragma unroll
            for (int cg = 0; cg < NCG; ++cg)
                acc[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Xs[4 * ks + g][16 * cg + c], acc[cg],
                                                              0, 0, 0);
        }
        __syncthreads();  // Xs is overwritten next
    }

    // the block's right-hand sides and its diagonal block into LDS (the
    // diagonal block is the identity past the order n)
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
        for (int r = 0; r < 4; ++r) Xs[16 * w + g + 4 * r][16 * cg + c] = acc[cg][r];
    for (int e = tid; e < kTB * kTB; e += 256) {
        const int rr = e % kTB, cc = e / kTB;
        double v = 0.0;
        if (rr >= rows || cc >= rows) v = (rr == cc) ? 1.0 : 0.0;
        else if (rr == cc) v = UNIT ? 1.0 : tget(r0 + rr, r0 + cc);
        else if (rr > cc) v = tget(r0 + rr, r0 + cc);
        Ls[rr][cc] = v;
        if (!UNIT && rr == cc) Rs[rr] = 1.0 / v;
    }
    __syncthreads();
    // substitution in axpy order: wave 0, lane = right-hand side, in four
    // 16-row steps held in registers; after a step its unknowns update the
    // rows below (each row with the step's unknowns in increasing order).
    // The fast divisions of a step are redone in IEEE arithmetic for the whole
    // wave if any operand left their guard (same quotient wherever it held).
    if (w == 0 && !aborted) {
#pragma unroll 1
        for (int sb = 0; sb < kTB / 16; ++sb) {
            const int b0 = 16 * sb;
            double y[16];
            auto step = [&](auto fast) {
#pragma unroll
                for (int r = 0; r < 16; ++r) y[r] = Xs[b0 + r][lane];
                bool ok = true;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    double x = y[r];
                    if (!UNIT) {
                        const double d = Ls[b0 + r][b0 + r];
                        if constexpr (decltype(fast)::value) {
                            bool oki;
                            x = div_rn_fast(y[r], d, Rs[b0 + r], div_fast_divisor(d), oki);
                            ok = ok && oki;
                        } else {
                            x = y[r] / d;
                        }
                    }
                    y[r] = x;
#pragma unroll
                    for (int q = r + 1; q < 16; ++q) y[q] = __builtin_fma(-Ls[b0 + q][b0 + r], x, y[q]);
                }
                return ok;
            };
            if (!__all(step(std::true_type()))) step(std::false_type());
#pragma unroll
            for (int r = 0; r < 16; ++r) Xs[b0 + r][lane] = y[r];
#pragma unroll 1
            for (int q = b0 + 16; q < kTB; ++q) {
                double t = Xs[q][lane];
#pragma unroll
                for (int r = 0; r < 16; ++r) t = __builtin_fma(-Ls[q][b0 + r], y[r], t);
                Xs[q][lane] = t;
            }
        }
    }
    __syncthreads();
    // X_i (NaN for an aborted block), stored along rows
    for (int e = tid; e < kTB * 16 * NCG; e += 256) {
        const int rr = e % kTB, col = e / kTB;
        if (rr < rows && col < ncols)
            *bptr(r0 + rr, col) = aborted ? (T)__builtin_nan("") : (T)Xs[rr][col];
    }
    __syncthreads();  // every store of the workgroup is complete
    if (tid == 0) {
        __threadfence();
        flag_release(flags + i, 1);
    }
}

template <typename T, bool UNIT, int NCG>
hipError_t thin_launch(const TriView& L, const RhsView& B, int64_t n, int ncols, int* flags,
                       hipStream_t s) {
    const void* fn = (const void*)thin_kernel<T, UNIT, NCG>;
    int per_cu = 0, cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess)
        return hipErrorInvalidValue;
    const int64_t nblk = (n + kTB - 1) / kTB;
    if (nblk > (int64_t)per_cu * cus) return hipErrorCooperativeLaunchTooLarge;
    int64_t cnt = nblk + 1;
    hipLaunchKernelGGL(thin_flags_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       flags, cnt);
    TriView l = L;
    RhsView b = B;
    int64_t nn = n, spin = (int64_t)1 << 22;
    int nc = ncols;
    int* fl = flags;
    void* args[] = {&l, &b, &nn, &nc, &fl, &spin};
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)nblk), dim3(256), args, 0, s);
}

template <typename T, bool UNIT>
hipError_t thin_by_groups(const TriView& L, const RhsView& B, int64_t n, int ncols, int* flags,
                          hipStream_t s) {
    switch ((ncols + 15) / 16) {
        case 1: return thin_launch<T, UNIT, 1>(L, B, n, ncols, flags, s);
        case 2: return thin_launch<T, UNIT, 2>(L, B, n, ncols, flags, s);
        case 3: return thin_launch<T, UNIT, 3>(L, B, n, ncols, flags, s);
        default: return thin_launch<T, UNIT, 4>(L, B, n, ncols, flags, s);
    }
}

}  // namespace

int64_t thin_flag_count(int64_t n) { return (n + kTB - 1) / kTB + 1; }

hipError_t launch_thin(int dtype, const TriView& L, const RhsView& B, int64_t n, int64_t ncols,
                       bool unit, int* flags, hipStream_t s) {
    if (n <= 0 || ncols <= 0) return hipSuccess;
    if (ncols > kTCols) return hipErrorInvalidValue;
    if (dtype == 0)
        return unit ? thin_by_groups<double, true>(L, B, n, (int)ncols, flags, s)
                    : thin_by_groups<double, false>(L, B, n, (int)ncols, flags, s);
    return unit ? thin_by_groups<float, true>(L, B, n, (int)ncols, flags, s)
                : thin_by_groups<float, false>(L, B, n, (int)ncols, flags, s);
}

}  // namespace redsea
