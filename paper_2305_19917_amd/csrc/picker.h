// Learned schedule picker: network shape, device kernels, host inference.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace redsea {

// 4 -> 64 -> 64 -> 45, parameters packed W1, b1, W2, b2, W3, b3 (row-major).
// Inputs: log2 n, log2 nrhs, dtype, log10 kappa (normalised).
struct MlpShape {
    static constexpr int in = 4, h1 = 64, h2 = 64, out = 45;
    constexpr int w1() const { return 0; }
    constexpr int b1() const { return h1 * in; }
    constexpr int w2() const { return b1() + h1; }
    constexpr int b2() const { return w2() + h2 * h1; }
    constexpr int w3() const { return b2() + h2; }
    constexpr int b3() const { return w3() + out * h2; }
    constexpr int count() const { return b3() + out; }
};

// forward into H1 (nb x 64), H2 (nb x 64), Y (nb x 45)
hipError_t mlp_forward_dev(const float* P, const float* X, int64_t nb, float* H1, float* H2,
                           float* Y, hipStream_t s);
// scratch: nb * (64 + 64 + 45 + 45 + 64 + 64) + 1 floats
hipError_t mlp_grad_dev(const float* P, const float* X, const float* T, const float* mask,
                        int64_t nb, float* G, float* loss, float* scratch, hipStream_t s);
hipError_t mlp_adam_dev(float* P, const float* G, float* M, float* V, int64_t step, float lr,
                        float b1, float b2, float eps, hipStream_t s);

// tuner data generation
hipError_t gen_system_dev(double* A, int64_t lda, int64_t n, double c, uint64_t seed,
                          double* rows, hipStream_t s);
hipError_t gen_rhs_dev(double* B, int64_t ldb, int64_t m, int64_t n, uint64_t seed, hipStream_t s);
hipError_t narrow_dev(const double* src, int64_t total, float* dst, hipStream_t s);

// host-side picker used by AUTO solves; returns -1 without weights
int pick_candidate(int dtype, int64_t n, int64_t nrhs, double kappa, int* confident);
void decode_candidate(int idx, int* variant, int* nb, int* precision);

}  // namespace redsea
