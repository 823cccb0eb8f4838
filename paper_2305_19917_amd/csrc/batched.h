// Persistent batched solver: device descriptors and launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace redsea {

// One system in canonical form (forward substitution, lower T of order k):
// T(i, j) = a[a_off + i*tr + j*tc], B(i, j) = b[b_off + i*br + j*bc].
struct BatchSys {
    const void* a;
    int64_t a_off, tr, tc;
    void* b;
    int64_t b_off, br, bc;
    int64_t k, nrhs;
};

// A tile of up to 16 right-hand sides [c0, c0 + 16) of system `sys`.
struct BatchTask {
    int32_t sys;
    int32_t c0;
};

constexpr int64_t kBatchMaxOrder = 1024;  // panel of 16 columns in LDS

hipError_t launch_batch_reset(int* counter, int* info, int64_t count, hipStream_t s);
hipError_t launch_batched(int dtype, bool unit, const BatchSys* sys, const BatchTask* tasks,
                          int ntasks, int* counter, int* info, int64_t kmax, double alpha,
                          int grid, hipStream_t s);

}  // namespace redsea
