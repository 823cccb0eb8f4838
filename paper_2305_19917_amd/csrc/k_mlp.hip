// Kernels of the learned schedule picker and of the tuner's data generator.
//
// The picker is a 3-layer FP32 MLP (4 -> 64 -> 64 -> 45, ReLU) regressing the
// log time of each candidate schedule.  Training and inference run on these
// hand-written kernels: one thread per output element, every reduction over
// the batch done by one thread in a fixed order, so results are
// deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "picker.h"

namespace redsea {

namespace {

// ------------------------------------------------------------------ MLP

// out[b][o] = act(sum_i W[o][i] in[b][i] + bias[o]),  W is O x I row-major
template <bool RELU>
__global__ __launch_bounds__(256) void linear_kernel(const float* __restrict__ W,
                                                     const float* __restrict__ bias,
                                                     const float* __restrict__ in, int I, int O,
                                                     int64_t nb, float* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nb * O) return;
    const int64_t b = idx / O;
    const int o = (int)(idx % O);
    float acc = bias[o];
    for (int i = 0; i < I; ++i) acc = __builtin_fmaf(W[o * I + i], in[b * I + i], acc);
    out[idx] = RELU ? (acc > 0.f ? acc : 0.f) : acc;
}

// dY = 2 mask (Y - T) / count, count = sum(mask) (computed by every thread
// in the same order, so it is the same value everywhere)
__global__ __launch_bounds__(256) void dloss_kernel(const float* __restrict__ Y,
                                                    const float* __restrict__ T,
                                                    const float* __restrict__ mask, int64_t total,
                                                    const float* __restrict__ count,
                                                    float* __restrict__ dY) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const float cnt = count[0] > 0.f ? count[0] : 1.f;
    dY[idx] = mask[idx] > 0.f ? 2.f * (Y[idx] - T[idx]) / cnt : 0.f;
}

// loss = sum mask (Y - T)^2 / sum mask, one workgroup, fixed reduction tree
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ Y,
                                                   const float* __restrict__ T,
                                                   const float* __restrict__ mask, int64_t total,
                                                   float* __restrict__ count,
                                                   float* __restrict__ loss) {
    __shared__ float s_err[256], s_cnt[256];
    float e = 0.f, c = 0.f;
    for (int64_t i = threadIdx.x; i < total; i += 256) {
        if (mask[i] > 0.f) {
            const float d = Y[i] - T[i];
            e = __builtin_fmaf(d, d, e);
            c += 1.f;
        }
    }
    s_err[threadIdx.x] = e;
    s_cnt[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_err[threadIdx.x] += s_err[threadIdx.x + w];
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        count[0] = s_cnt[0];
        loss[0] = s_cnt[0] > 0.f ? s_err[0] / s_cnt[0] : 0.f;
    }
}

// dW[o][i] = sum_b dOut[b][o] in[b][i];  db[o] = sum_b dOut[b][o]
__global__ __launch_bounds__(256) void wgrad_kernel(const float* __restrict__ dOut,
                                                    const float* __restrict__ in, int I, int O,
                                                    int64_t nb, float* __restrict__ dW,
                                                    float* __restrict__ db) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx < O * I) {
        const int o = idx / I, i = idx % I;
        float acc = 0.f;
        for (int64_t b = 0; b < nb; ++b) acc = __builtin_fmaf(dOut[b * O + o], in[b * I + i], acc);
        dW[idx] = acc;
    } else if (idx < O * I + O) {
        const int o = idx - O * I;
        float acc = 0.f;
        for (int64_t b = 0; b < nb; ++b) acc += dOut[b * O + o];
        db[o] = acc;
    }
}

// dIn[b][i] = (sum_o dOut[b][o] W[o][i]) * (act[b][i] > 0)
__global__ __launch_bounds__(256) void dgrad_kernel(const float* __restrict__ dOut,
                                                    const float* __restrict__ W,
                                                    const float* __restrict__ act, int I, int O,
                                                    int64_t nb, float* __restrict__ dIn) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nb * I) return;
    const int64_t b = idx / I;
    const int i = (int)(idx % I);
    float acc = 0.f;
    for (int o = 0; o < O; ++o) acc = __builtin_fmaf(dOut[b * O + o], W[o * I + i], acc);
    dIn[idx] = act[idx] > 0.f ? acc : 0.f;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int n, float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ generator

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014)
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double unit_draw(uint64_t seed, uint64_t i, uint64_t j) {
    const uint64_t h = mix64(seed ^ mix64(i * 0x100000001B3ull + j));
    return (double)(h >> 11) * 0x1.0p-53;  // [0, 1)
}

// strict lower part U(-1, 1); row sums of |L| into rows[i]
__global__ __launch_bounds__(256) void gen_lower_kernel(double* __restrict__ A, int64_t lda,
                                                        int64_t n, uint64_t seed,
                                                        double* __restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double sum = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double v = 0.0;
        if (j < i) {
            v = 2.0 * unit_draw(seed, (uint64_t)i, (uint64_t)j) - 1.0;
            sum += fabs(v);
        }
        if (j != i) A[i + j * lda] = v;
    }
    rows[i] = sum;
}

// diagonal: 1 + row sum (c <= 0) or c (1 + max row sum)
__global__ __launch_bounds__(256) void gen_diag_kernel(double* __restrict__ A, int64_t lda,
                                                       int64_t n, double c,
                                                       const double* __restrict__ rows) {
    __shared__ double red[256];
    double mx = 0.0;
    if (c > 0.0) {
        for (int64_t i = threadIdx.x; i < n; i += 256) mx = rows[i] > mx ? rows[i] : mx;
        red[threadIdx.x] = mx;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w && red[threadIdx.x + w] > red[threadIdx.x])
                red[threadIdx.x] = red[threadIdx.x + w];
            __syncthreads();
        }
        mx = red[0];
    }
    for (int64_t i = threadIdx.x; i < n; i += 256)
        A[i + i * lda] = c > 0.0 ? c * (1.0 + mx) : 1.0 + rows[i];
}

// right-hand sides: approximately N(0, 1) (Box-Muller on two draws)
__global__ __launch_bounds__(256) void gen_rhs_kernel(double* __restrict__ B, int64_t ldb,
                                                      int64_t m, int64_t n, uint64_t seed) {
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx % m, j = idx / m;
        const double u1 = unit_draw(seed ^ 0x5555ull, (uint64_t)i, (uint64_t)j) + 0x1.0p-54;
        const double u2 = unit_draw(seed ^ 0xAAAAull, (uint64_t)i, (uint64_t)j);
        B[i + j * ldb] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

__global__ __launch_bounds__(256) void narrow_kernel(const double* __restrict__ src, int64_t total,
                                                     float* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * 256)
        dst[i] = (float)src[i];
}

unsigned blocks_for(int64_t total) {
    int64_t b = (total + 255) / 256;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (unsigned)b;
}

}  // namespace

hipError_t mlp_forward_dev(const float* P, const float* X, int64_t nb, float* H1, float* H2,
                           float* Y, hipStream_t s) {
    const MlpShape S;
    const float* W1 = P + S.w1();
    const float* b1 = P + S.b1();
    const float* W2 = P + S.w2();
    const float* b2 = P + S.b2();
    const float* W3 = P + S.w3();
    const float* b3 = P + S.b3();
    hipLaunchKernelGGL(linear_kernel<true>, dim3(blocks_for(nb * S.h1)), dim3(256), 0, s, W1, b1, X,
                       S.in, S.h1, nb, H1);
    hipLaunchKernelGGL(linear_kernel<true>, dim3(blocks_for(nb * S.h2)), dim3(256), 0, s, W2, b2, H1,
                       S.h1, S.h2, nb, H2);
    hipLaunchKernelGGL(linear_kernel<false>, dim3(blocks_for(nb * S.out)), dim3(256), 0, s, W3, b3,
                       H2, S.h2, S.out, nb, Y);
    return hipGetLastError();
}

hipError_t mlp_grad_dev(const float* P, const float* X, const float* T, const float* mask,
                        int64_t nb, float* G, float* loss, float* scratch, hipStream_t s) {
    const MlpShape S;
    float* H1 = scratch;
    float* H2 = H1 + nb * S.h1;
    float* Y = H2 + nb * S.h2;
    float* dY = Y + nb * S.out;
    float* dH2 = dY + nb * S.out;
    float* dH1 = dH2 + nb * S.h2;
    float* count = dH1 + nb * S.h1;
    hipError_t e = mlp_forward_dev(P, X, nb, H1, H2, Y, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, Y, T, mask, nb * S.out, count, loss);
    hipLaunchKernelGGL(dloss_kernel, dim3(blocks_for(nb * S.out)), dim3(256), 0, s, Y, T, mask,
                       nb * S.out, count, dY);
    // layer 3
    hipLaunchKernelGGL(wgrad_kernel, dim3((S.out * S.h2 + S.out + 255) / 256), dim3(256), 0, s, dY,
                       H2, S.h2, S.out, nb, G + S.w3(), G + S.b3());
    hipLaunchKernelGGL(dgrad_kernel, dim3(blocks_for(nb * S.h2)), dim3(256), 0, s, dY, P + S.w3(),
                       H2, S.h2, S.out, nb, dH2);
    // layer 2
    hipLaunchKernelGGL(wgrad_kernel, dim3((S.h2 * S.h1 + S.h2 + 255) / 256), dim3(256), 0, s, dH2,
                       H1, S.h1, S.h2, nb, G + S.w2(), G + S.b2());
    hipLaunchKernelGGL(dgrad_kernel, dim3(blocks_for(nb * S.h1)), dim3(256), 0, s, dH2, P + S.w2(),
                       H1, S.h1, S.h2, nb, dH1);
    // layer 1
    hipLaunchKernelGGL(wgrad_kernel, dim3((S.h1 * S.in + S.h1 + 255) / 256), dim3(256), 0, s, dH1,
                       X, S.in, S.h1, nb, G + S.w1(), G + S.b1());
    return hipGetLastError();
}

hipError_t mlp_adam_dev(float* P, const float* G, float* M, float* V, int64_t step, float lr,
                        float b1, float b2, float eps, hipStream_t s) {
    const MlpShape S;
    const int n = S.count();
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, P, G, M, V, n, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t gen_system_dev(double* A, int64_t lda, int64_t n, double c, uint64_t seed,
                          double* rows, hipStream_t s) {
    hipLaunchKernelGGL(gen_lower_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, lda,
                       n, seed, rows);
    hipLaunchKernelGGL(gen_diag_kernel, dim3(1), dim3(256), 0, s, A, lda, n, c, rows);
    return hipGetLastError();
}

hipError_t gen_rhs_dev(double* B, int64_t ldb, int64_t m, int64_t n, uint64_t seed,
                       hipStream_t s) {
    hipLaunchKernelGGL(gen_rhs_kernel, dim3(blocks_for(m * n)), dim3(256), 0, s, B, ldb, m, n, seed);
    return hipGetLastError();
}

hipError_t narrow_dev(const double* src, int64_t total, float* dst, hipStream_t s) {
    hipLaunchKernelGGL(narrow_kernel, dim3(blocks_for(total)), dim3(256), 0, s, src, total, dst);
    return hipGetLastError();
}

}  // namespace redsea
