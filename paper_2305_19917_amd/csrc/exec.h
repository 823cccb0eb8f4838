// Executor internals shared by the entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/redsea.h"
#include "kernels.h"
#include "plan.h"

namespace redsea {

// A solve in canonical form: forward substitution with the lower-triangular
// T of order k on nrhs right-hand sides.
struct Canon {
    int dtype;
    bool unit;
    bool op_trans;   // the left problem's matrix is A^T (storage layout "T")
    bool rhs_trans;  // right-hand sides are rows of B (right side)
    bool reverse;    // backward substitution, indices reversed
    int64_t k, nrhs;
    const void* A;
    int64_t lda;
    void* B;
    int64_t ldb;
    TriView tri;
    RhsView rhs;
    // BF16 products (mixed precision): the products read the BF16 copy A16 of
    // M = op_eff(A) stored by rows (M(i, j) at A16[j + i*lda16]) and round X
    // to BF16 as they read it; leaves stay on A (FP32).
    bool gemm_bf16 = false;
    const void* A16 = nullptr;
    int64_t lda16 = 0;
};

Canon canonicalize(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                   const void* A, int64_t lda, void* B, int64_t ldb);
GemmArgs gemm_args(const Canon& c, int64_t r0, int64_t R, int64_t c0, int64_t K);
const std::vector<Task>& plan_for(int variant, int64_t k, int64_t nb, int64_t kleaf);
// Library workspace for one stream (see api.cpp): `ptr` stays valid, and no
// other host thread may regrow it, while the lease is held.
struct WsLease {
    std::unique_lock<std::mutex> lock;
    void* ptr = nullptr;
};
int workspace(int slot, size_t bytes, hipStream_t s, WsLease& out);
// Bytes of packed diagonal blocks execute() needs for this solve.
size_t packed_bytes(const Canon& c, int64_t nb);
// Runs the solve on stream s.  packed: device memory of packed_bytes(c, nb)
// bytes for the diagonal blocks, or null to take it from the workspace.
// thin_flags: device memory of thin_flag_count ints for the one-launch thin
// solve when `packed` is given (without it, a caller-owned-memory solve
// takes the split schedule); ignored when packed is null.
int execute(const Canon& c, int variant, int64_t nb, hipStream_t s, void* packed = nullptr,
            int* thin_flags = nullptr);
// Kernel timing trace (redsea_trace_begin / redsea_trace_end).
bool trace_on();
void trace_push(int kind, double flops, hipEvent_t e0, hipEvent_t e1);

// Runs `launch` and, when tracing, records events around it on stream s.
template <typename F>
hipError_t traced(int kind, double flops, hipStream_t s, F&& launch) {
    if (!trace_on()) return launch();
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return hipErrorOutOfMemory;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hipErrorOutOfMemory;
    }
    (void)hipEventRecord(e0, s);
    hipError_t e = launch();
    (void)hipEventRecord(e1, s);
    trace_push(kind, flops, e0, e1);
    return e;
}

int check_args(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
               const void* A, int64_t lda, const void* B, int64_t ldb, bool need_a);
int pick_nb(int requested, int64_t k);
int tuned_candidate(int dtype, int64_t k, int64_t nrhs, double kappa, hipStream_t s);
int mixed_solve(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
                const double* A, int64_t lda, double* B, int64_t ldb, int inner, double tol,
                int max_iter, void* work, size_t work_bytes, redsea_mixed_stats* stats,
                const redsea_opts* opts, hipStream_t s);

}  // namespace redsea
