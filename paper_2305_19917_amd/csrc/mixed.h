// Launchers of the mixed-precision kernels (k_mixed.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace redsea {

hipError_t launch_convert_tri(int to_bf16, const double* a, int64_t lda, int64_t k, int uplo,
                              bool unit, void* dst, hipStream_t s);
// dst (row-major, ld ldd) := BF16 of M = op(A) restricted to A's stored
// triangle (zero elsewhere, padding columns included; unit diagonal one).
hipError_t launch_convert_rows_bf16(const double* a, int64_t lda, int64_t k, int uplo, bool unit,
                                   bool op_trans, void* dst, int64_t ldd, hipStream_t s);
hipError_t launch_scale_to_f32(const double* src, int64_t ld, int64_t m, int64_t n,
                               const double* inv, bool rhs_rows, double alpha, float* dst,
                               int64_t ldd, hipStream_t s);
hipError_t launch_update(double* x, int64_t ldx, int64_t m, int64_t n, const float* d, int64_t ldd,
                         const double* scale, bool rhs_rows, bool accumulate, hipStream_t s);
hipError_t launch_copy_scaled(const double* src, int64_t lds, int64_t m, int64_t n, double alpha,
                              double* dst, int64_t ldd, hipStream_t s);
hipError_t launch_rhs_max(const double* a, int64_t ld, int64_t m, int64_t n, bool rhs_rows,
                          double scale, double* out, hipStream_t s);
hipError_t launch_tri_rowsum(const double* a, int64_t lda, int64_t k, bool a_trans, bool lower,
                             bool unit, double* out, hipStream_t s);
hipError_t launch_gemm_bf16(bool a_trans, bool rhs_trans, const GemmArgs& g, hipStream_t s);

}  // namespace redsea
