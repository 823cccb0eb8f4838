// Host side of the batched solve: validation, canonical descriptors, the
// longest-first task order, and the plan object whose run is launches only
// (so it can be captured in a hipGraph and replayed).  Systems of order above
// kBatchMaxOrder are left to the single-system path, whose recursive
// schedule suits them better than one wave per 16 columns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <vector>

#include "../../include/redsea.h"
#include "batched.h"
#include "exec.h"
#include "kernels.h"

struct redsea_batch_plan {
    int dtype = 0;
    bool unit = false;
    double alpha = 1.0;
    int64_t count = 0;
    int ntasks = 0;
    int64_t kmax = 0;
    int grid = 0;
    int device = 0;
    redsea::BatchSys* d_sys = nullptr;
    redsea::BatchTask* d_tasks = nullptr;
    int* d_counter = nullptr;
    // systems above the panel limit, solved by the single-system path
    std::vector<redsea::Canon> big;
    std::vector<int64_t> big_index;
    int variant = 1, nb = 128;
    // packed diagonal blocks of the large systems (solved one after another
    // on the run's stream, so one buffer of the largest size serves all);
    // owned by the plan so that a run allocates nothing
    void* packed = nullptr;
};

namespace redsea {

namespace {

int validate(int dtype, int side, int uplo, int trans, int diag, int64_t count, const int64_t* m,
             const int64_t* n, double alpha, const void* const* A, const int64_t* lda,
             void* const* B, const int64_t* ldb) {
    if (dtype != REDSEA_F64 && dtype != REDSEA_F32) return -1;
    if (side != REDSEA_LEFT && side != REDSEA_RIGHT) return -2;
    if (uplo != REDSEA_LOWER && uplo != REDSEA_UPPER) return -3;
    if (trans != REDSEA_NOTRANS && trans != REDSEA_TRANS && trans != REDSEA_CONJTRANS) return -4;
    if (diag != REDSEA_NONUNIT && diag != REDSEA_UNIT) return -5;
    if (count < 0) return -6;
    if (count == 0) return 0;
    if (!m) return -7;
    if (!n) return -8;
    if (!A) return -10;
    if (!lda) return -11;
    if (!B) return -12;
    if (!ldb) return -13;
    for (int64_t i = 0; i < count; ++i) {
        if (m[i] < 0) return -7;
        if (n[i] < 0) return -8;
        const int64_t ka = side == REDSEA_LEFT ? m[i] : n[i];
        if (lda[i] < std::max<int64_t>(1, ka)) return -11;
        if (ldb[i] < std::max<int64_t>(1, m[i])) return -13;
        if (m[i] > 0 && n[i] > 0) {
            if (alpha != 0.0 && A[i] == nullptr) return -10;
            if (B[i] == nullptr) return -12;
        }
    }
    return 0;
}

}  // namespace

}  // namespace redsea

using namespace redsea;

extern "C" {

int redsea_batched_plan_create(int dtype, int side, int uplo, int trans, int diag, int64_t count,
                               const int64_t* m, const int64_t* n, double alpha,
                               const void* const* A, const int64_t* lda, void* const* B,
                               const int64_t* ldb, const redsea_opts* opts,
                               redsea_batch_plan** out) {
    if (!out) return -15;
    *out = nullptr;
    int rc = validate(dtype, side, uplo, trans, diag, count, m, n, alpha, A, lda, B, ldb);
    if (rc) return rc;
    if (opts && (opts->variant < 0 || opts->variant > 3)) return -14;
    redsea_batch_plan* P = new redsea_batch_plan;
    P->dtype = dtype;
    P->unit = diag == REDSEA_UNIT;
    P->alpha = alpha;
    P->count = count;
    if (opts && opts->variant) P->variant = opts->variant;
    if (opts && opts->nb) P->nb = opts->nb;
    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return REDSEA_ERR_HIP;
    }
    std::vector<BatchSys> sys;  // indexed by the system's position in the batch
    std::vector<std::pair<double, BatchTask>> work;
    for (int64_t i = 0; i < count; ++i) {
        if (m[i] == 0 || n[i] == 0) continue;
        Canon c = canonicalize(dtype, side, uplo, trans, diag, m[i], n[i], A[i], lda[i], B[i], ldb[i]);
        if (c.k > kBatchMaxOrder) {
            P->big.push_back(c);
            P->big_index.push_back(i);
            continue;
        }
        BatchSys d;
        d.a = c.tri.base;
        d.a_off = c.tri.off;
        d.tr = c.tri.tr;
        d.tc = c.tri.tc;
        d.b = c.rhs.base;
        d.b_off = c.rhs.off;
        d.br = c.rhs.br;
        d.bc = c.rhs.bc;
        d.k = c.k;
        d.nrhs = c.nrhs;
        const int32_t id = (int32_t)i;
        P->kmax = std::max(P->kmax, c.k);
        for (int64_t c0 = 0; c0 < c.nrhs; c0 += 16) {
            const double w = (double)std::min<int64_t>(16, c.nrhs - c0);
            const double kp = (double)((c.k + 15) / 16 * 16);
            // longest-processing-time first: the chain of k divisions plus the
            // k^2 w / 2 update work, both per tile
            work.push_back({kp * kp * 16.0 / 2.0 + 600.0 * kp + w, BatchTask{id, (int32_t)c0}});
        }
        sys.resize(std::max<size_t>(sys.size(), (size_t)i + 1));
        sys[i] = d;
    }
    size_t big_bytes = 0;
    for (const Canon& c : P->big) big_bytes = std::max(big_bytes, packed_bytes(c, pick_nb(P->nb, c.k)));
    if (big_bytes > 0 && hipMalloc(&P->packed, big_bytes) != hipSuccess) {
        (void)hipGetLastError();
        P->packed = nullptr;
        redsea_batched_plan_destroy(P);
        return REDSEA_ERR_ALLOC;
    }
    std::stable_sort(work.begin(), work.end(),
                     [](const std::pair<double, BatchTask>& x, const std::pair<double, BatchTask>& y) {
                         return x.first > y.first;
                     });
    std::vector<BatchTask> tasks;
    tasks.reserve(work.size());
    for (auto& w : work) tasks.push_back(w.second);
    P->ntasks = (int)tasks.size();
    if (sys.empty()) sys.resize(1);
    bool ok = hipMalloc(&P->d_sys, sys.size() * sizeof(BatchSys)) == hipSuccess &&
              hipMalloc(&P->d_tasks, std::max<size_t>(1, tasks.size()) * sizeof(BatchTask)) ==
                  hipSuccess &&
              hipMalloc(&P->d_counter, sizeof(int)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        redsea_batched_plan_destroy(P);
        return REDSEA_ERR_ALLOC;
    }
    if (hipMemcpy(P->d_sys, sys.data(), sys.size() * sizeof(BatchSys), hipMemcpyHostToDevice) !=
            hipSuccess ||
        (!tasks.empty() && hipMemcpy(P->d_tasks, tasks.data(), tasks.size() * sizeof(BatchTask),
                                     hipMemcpyHostToDevice) != hipSuccess)) {
        redsea_batched_plan_destroy(P);
        return REDSEA_ERR_HIP;
    }
    // persistent grid: eight resident waves per CU (two workgroups of four);
    // each wave claims tasks on its own
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess)
        cus = 256;
    P->grid = std::max(1, std::min((P->ntasks + 3) / 4, cus * 2));
    *out = P;
    return REDSEA_OK;
}

int redsea_batched_plan_run(redsea_batch_plan* P, int* info, void* stream) {
    if (!P) return -1;
    if (P->count > 0 && !info) return -2;
    if (P->count == 0) return REDSEA_OK;
    hipStream_t s = (hipStream_t)stream;
    if (launch_batch_reset(P->d_counter, info, P->count, s) != hipSuccess) return REDSEA_ERR_HIP;
    if (P->ntasks > 0 &&
        launch_batched(P->dtype, P->unit, P->d_sys, P->d_tasks, P->ntasks, P->d_counter, info,
                       std::max<int64_t>(P->kmax, 16), P->alpha, P->grid, s) != hipSuccess)
        return REDSEA_ERR_HIP;
    for (size_t i = 0; i < P->big.size(); ++i) {
        const Canon& c = P->big[i];
        const int64_t rows = c.rhs_trans ? c.nrhs : c.k, cols = c.rhs_trans ? c.k : c.nrhs;
        if (P->alpha != 1.0 &&
            launch_scale(P->dtype, c.B, rows, cols, c.ldb, P->alpha, s) != hipSuccess)
            return REDSEA_ERR_HIP;
        if (P->alpha != 0.0) {
            int rc = execute(c, P->variant, pick_nb(P->nb, c.k), s, P->packed);
            if (rc) return rc;
        }
        if (launch_check_finite(P->dtype, c.B, rows, cols, c.ldb, info + P->big_index[i],
                                REDSEA_ERR_NONFINITE, s) != hipSuccess)
            return REDSEA_ERR_HIP;
    }
    return REDSEA_OK;
}

void redsea_batched_plan_destroy(redsea_batch_plan* P) {
    if (!P) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(P->device);
    (void)hipDeviceSynchronize();
    if (P->d_sys) (void)hipFree(P->d_sys);
    if (P->d_tasks) (void)hipFree(P->d_tasks);
    if (P->d_counter) (void)hipFree(P->d_counter);
    if (P->packed) (void)hipFree(P->packed);
    (void)hipSetDevice(cur);
    delete P;
}

int redsea_trsm_batched(int dtype, int side, int uplo, int trans, int diag, int64_t count,
                        const int64_t* m, const int64_t* n, double alpha,
                        const void* const* A, const int64_t* lda, void* const* B,
                        const int64_t* ldb, int* info, const redsea_opts* opts, void* stream) {
    int rc = validate(dtype, side, uplo, trans, diag, count, m, n, alpha, A, lda, B, ldb);
    if (rc) return rc;
    if (count == 0) return REDSEA_OK;
    if (!info) return -14;
    if (opts && (opts->variant < 0 || opts->variant > 3)) return -15;
    if (opts && !(opts->nb == 0 || opts->nb == 16 || opts->nb == 32 || opts->nb == 64 ||
                  opts->nb == 128 || opts->nb == 256 || opts->nb == 512))
        return -15;
    redsea_batch_plan* P = nullptr;
    rc = redsea_batched_plan_create(dtype, side, uplo, trans, diag, count, m, n, alpha, A, lda, B,
                                    ldb, opts, &P);
    if (rc) return rc;
    rc = redsea_batched_plan_run(P, info, stream);
    redsea_batched_plan_destroy(P);  // waits for the launch before freeing descriptors
    return rc;
}

}  // extern "C"
