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

// Task queues, one per XCD: the tasks of a system all sit in one queue, so
// the column tiles of a system run on one XCD and share its triangle in that
// XCD's L2.  A workgroup claims from the queue of its XCD (workgroups are
// dispatched to the XCDs round-robin) and then from the others in turn, so
// every task is claimed exactly once wherever it runs.  Counters are 32 ints
// apart (one cache line each).
constexpr int kBatchQueues = 8;
constexpr int kBatchCounterInts = 32 * kBatchQueues;
struct BatchQueues {
    int start[kBatchQueues];  // first task of each queue in the task array
    int count[kBatchQueues];
};

hipError_t launch_batch_reset(int* counters, int* info, int64_t count, hipStream_t s);
// groups: column groups of 16 per task (1 or 2; with 2 a wave solves 32
// right-hand sides and each block of the triangle it loads feeds both).
// depth: steps of the left-looking product whose operands are in flight (1,
// 2 or 4).  Neither changes the arithmetic: results are bitwise the same.
hipError_t launch_batched(int dtype, bool unit, int groups, int depth, const BatchSys* sys,
                          const BatchTask* tasks, const BatchQueues& queues, int* counters,
                          int* info, double alpha, int grid, hipStream_t s);

// Task shapes the batched solver can run (index = tile option - 1):
// {column groups per task, operand prefetch depth, workgroups of four waves
// per CU}.
constexpr int kBatchTiles = 12;
constexpr int kBatchTileGroups[kBatchTiles] = {1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2};
constexpr int kBatchTileDepth[kBatchTiles] = {1, 1, 2, 2, 4, 4, 1, 1, 2, 2, 4, 4};
constexpr int kBatchTileWgPerCu[kBatchTiles] = {2, 4, 2, 4, 2, 4, 2, 4, 2, 4, 2, 4};
constexpr int kBatchTileDefault = 1;

}  // namespace redsea
