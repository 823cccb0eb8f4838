// Persistent batched solver: many independent triangular systems of uneven
// order and right-hand-side count in one launch (the solve of Sec. IV per
// system; spec batching pattern).
//
// Work is a list of tasks (system, tile of up to 16 right-hand sides), sorted
// longest-first on the host.  Each workgroup repeatedly claims the next task
// from a counter and solves it alone: the system's order is at most kmax
// (<= 1024), so the whole 16-column panel of B stays in LDS while the
// workgroup runs the right-looking blocked substitution over 16-row blocks:
//   wave 0 solves the 16 x 16 diagonal block of every column by substitution
//   (one IEEE division per row), then all four waves update the blocks below
//   on the matrix cores (v_mfma_f64_16x16x4f64), each wave a different block.
// A task never depends on another, so the result does not depend on which
// workgroup ran it.
#include <hip/hip_runtime.h>

#include "batched.h"

namespace redsea {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void batch_reset_kernel(int* counter, int* info, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        info[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

template <typename TS, bool UNIT>
__global__ __launch_bounds__(256) void batched_kernel(const BatchSys* __restrict__ sys,
                                                      const BatchTask* __restrict__ tasks,
                                                      int ntasks, int* __restrict__ counter,
                                                      int* __restrict__ info, double alpha) {
    extern __shared__ double Pn[];  // [rows][16], rows = padded order of the task's system
    __shared__ double Ld[16 * 16];  // diagonal block, element (j, i) at Ld[i*16 + j]
    __shared__ int claimed;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;
    for (;;) {
        if (tid == 0) claimed = atomicAdd(counter, 1);
        __syncthreads();
        const int t = claimed;
        __syncthreads();
        if (t >= ntasks) break;  // uniform: every thread read the same value
        const BatchTask task = tasks[t];
        const BatchSys S = sys[task.sys];
        const TS* A = (const TS*)S.a;
        TS* B = (TS*)S.b;
        const int64_t k = S.k, c0 = task.c0;
        const int w = (int)(S.nrhs - c0 < 16 ? S.nrhs - c0 : 16);
        const int nblk = (int)((k + 15) / 16), kp = nblk * 16;
        // load the panel (rows past k and columns past w are zero)
        for (int idx = tid; idx < kp * 16; idx += 256) {
            const int i = idx % kp, j = idx / kp;
            double v = 0.0;
            if (i < k && j < w) {
                v = (double)B[S.b_off + i * S.br + (c0 + j) * S.bc];
                if (alpha != 1.0) v = alpha * v;
            }
            Pn[i * 16 + j] = v;
        }
        __syncthreads();
        if (alpha != 0.0) {
            for (int q = 0; q < nblk; ++q) {
                if (wave == 0) {
                    // stage the diagonal block (identity past the order)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = g + 4 * r, jj = c;  // element (i, jj) of the block
                        const int64_t gi = 16 * q + i, gj = 16 * q + jj;
                        double v = 0.0;
                        if (gi >= k) v = (i == jj) ? 1.0 : 0.0;
                        else if (i == jj) v = UNIT ? 1.0 : (double)A[S.a_off + gi * S.tr + gj * S.tc];
                        else if (i > jj) v = (double)A[S.a_off + gi * S.tr + gj * S.tc];
                        Ld[jj * 16 + i] = v;
                    }
                    wave_sync();
                    if (g == 0) {
                        double y[16];
#pragma unroll
                        for (int i = 0; i < 16; ++i) y[i] = Pn[(16 * q + i) * 16 + c];
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            double x = y[i];
                            if (!UNIT) x = x / Ld[i * 16 + i];
                            y[i] = x;
#pragma unroll
                            for (int j = i + 1; j < 16; ++j) y[j] = __builtin_fma(-Ld[i * 16 + j], x, y[j]);
                        }
#pragma unroll
                        for (int i = 0; i < 16; ++i) Pn[(16 * q + i) * 16 + c] = y[i];
                    }
                }
                __syncthreads();
                for (int p = q + 1 + wave; p < nblk; p += 4) {
                    v4d f;
#pragma unroll
                    for (int r = 0; r < 4; ++r) f[r] = Pn[(16 * p + g + 4 * r) * 16 + c];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const int64_t gi = 16 * p + c, gj = 16 * q + 4 * kk + g;
                        const double a = gi < k ? -(double)A[S.a_off + gi * S.tr + gj * S.tc] : 0.0;
                        const double b = Pn[(16 * q + 4 * kk + g) * 16 + c];
                        f = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, f, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) Pn[(16 * p + g + 4 * r) * 16 + c] = f[r];
                }
                __syncthreads();
            }
        }
        // store, flagging non-finite results of the system
        int bad = 0;
        for (int idx = tid; idx < kp * 16; idx += 256) {
            const int i = idx % kp, j = idx / kp;
            if (i < k && j < w) {
                const TS v = (TS)Pn[i * 16 + j];
                B[S.b_off + i * S.br + (c0 + j) * S.bc] = v;
                if (!__builtin_isfinite((double)v)) bad = 1;
            }
        }
        if (bad) atomicOr(&info[task.sys], 4);
        __syncthreads();  // the panel is free for the next task
    }
}

}  // namespace

hipError_t launch_batch_reset(int* counter, int* info, int64_t count, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(batch_reset_kernel, dim3((unsigned)blocks), dim3(256), 0, s, counter, info,
                       count);
    return hipGetLastError();
}

size_t batched_lds_bytes(int64_t kmax) { return (size_t)((kmax + 15) / 16) * 16 * 16 * 8; }

hipError_t launch_batched(int dtype, bool unit, const BatchSys* sys, const BatchTask* tasks,
                          int ntasks, int* counter, int* info, int64_t kmax, double alpha,
                          int grid, hipStream_t s) {
    const size_t lds = batched_lds_bytes(kmax);
    if (dtype == 0) {
        if (unit)
            hipLaunchKernelGGL((batched_kernel<double, true>), dim3(grid), dim3(256), lds, s, sys,
                               tasks, ntasks, counter, info, alpha);
        else
            hipLaunchKernelGGL((batched_kernel<double, false>), dim3(grid), dim3(256), lds, s, sys,
                               tasks, ntasks, counter, info, alpha);
    } else {
        if (unit)
            hipLaunchKernelGGL((batched_kernel<float, true>), dim3(grid), dim3(256), lds, s, sys,
                               tasks, ntasks, counter, info, alpha);
        else
            hipLaunchKernelGGL((batched_kernel<float, false>), dim3(grid), dim3(256), lds, s, sys,
                               tasks, ntasks, counter, info, alpha);
    }
    return hipGetLastError();
}

hipError_t batched_set_lds_limit(int dtype, bool unit, size_t bytes) {
    const void* f;
    if (dtype == 0) f = unit ? (const void*)batched_kernel<double, true> : (const void*)batched_kernel<double, false>;
    else f = unit ? (const void*)batched_kernel<float, true> : (const void*)batched_kernel<float, false>;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace redsea
