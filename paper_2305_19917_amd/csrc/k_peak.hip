// Matrix-core throughput probe: every wave of a full grid runs eight
// independent accumulation chains of 16x16x4 MFMAs (FP64 or FP32) and writes
// one checksum per lane, so the measured rate is the achievable MFMA peak of
// the device under the clock it holds while the matrix cores are busy.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "redsea.h"

namespace redsea {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(256) void mfma_peak_kernel(int64_t iters, T* out) {
    typedef typename std::conditional<sizeof(T) == 8, v4d, v4f>::type acc_t;
    const int lane = threadIdx.x & 63;
    // distinct operands per chain, so that no two chains can be merged
    T a[8], b[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = T(1) + T(lane + 64 * i) * T(1e-4);
        b[i] = T(1) - T(lane + 64 * i) * T(1e-4);
    }
    acc_t acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = acc_t{0, 0, 0, 0};
    // 16 steps per trip, so that any register moves the loop back-edge needs
    // are amortised over 128 MFMAs
    for (int64_t it = 0; it < iters; it += 16) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if constexpr (sizeof(T) == 8)
                    acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[i], acc[i], 0, 0, 0);
                else
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[i], acc[i], 0, 0, 0);
            }
    }
    T s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace
}  // namespace redsea

extern "C" int64_t redsea_mfma_peak(int dtype, int64_t iters, void* out, int64_t out_elems,
                                    void* stream_ptr) {
    hipStream_t stream = (hipStream_t)stream_ptr;
    using namespace redsea;
    const int64_t grid = 4096;  // 16 workgroups of four waves per CU
    if ((dtype != REDSEA_F64 && dtype != REDSEA_F32) || iters <= 0) return -1;
    iters = (iters + 15) / 16 * 16;  // whole trips of the unrolled loop
    if (out == nullptr || out_elems < grid * 256) return -3;
    if (dtype == REDSEA_F64)
        hipLaunchKernelGGL(mfma_peak_kernel<double>, dim3((unsigned)grid), dim3(256), 0, stream,
                           iters, (double*)out);
    else
        hipLaunchKernelGGL(mfma_peak_kernel<float>, dim3((unsigned)grid), dim3(256), 0, stream,
                           iters, (float*)out);
    if (hipGetLastError() != hipSuccess) return -100;
    // flops: waves x iterations x 8 chains x 16*16*4*2
    return grid * 4 * iters * 8 * 2048;
}
