// Host side of the batched solve: validation, canonical descriptors, the
// longest-first task order, and the plan object whose run is launches only
// (so it can be captured in a hipGraph and replayed).  Systems of order above
// kBatchMaxOrder are left to the single-system path, whose recursive
// schedule suits them better than one wave per 16 columns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/redsea.h"
#include "batched.h"
#include "exec.h"
#include "kernels.h"
#include "picker.h"

struct redsea_batch_plan {
    int dtype = 0;
    bool unit = false;
    double alpha = 1.0;
    int64_t count = 0;
    int ntasks = 0;
    int64_t kmax = 0;
    int grid = 0;
    int tile = redsea::kBatchTileDefault;  // task shape (1-based index into kBatchTiles)
    int device = 0;
    redsea::BatchSys* d_sys = nullptr;
    redsea::BatchTask* d_tasks = nullptr;
    redsea::BatchQueues queues{};
    int* d_counter = nullptr;  // kBatchCounterInts ints
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

// Tile choices of the autotuner, per device and batch signature (data type,
// unit diagonal, and the rounded log2 of the system count, of the largest and
// median orders and of the median right-hand-side count).
typedef std::tuple<int, int, int, int, int, int, int> BatchSig;
std::mutex g_bt_mu;
std::map<BatchSig, int> g_bt;

int batch_signature(int dtype, int diag, int64_t count, const int64_t* m, const int64_t* n,
                    int side, BatchSig* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return REDSEA_ERR_HIP;
    std::vector<int64_t> ks, rs;
    for (int64_t i = 0; i < count; ++i) {
        if (m[i] == 0 || n[i] == 0) continue;
        ks.push_back(side == REDSEA_LEFT ? m[i] : n[i]);
        rs.push_back(side == REDSEA_LEFT ? n[i] : m[i]);
    }
    auto lg = [](double v) { return (int)std::lround(std::log2(std::max(v, 1.0))); };
    int kmax = 0, kmed = 0, rmed = 0;
    if (!ks.empty()) {
        std::sort(ks.begin(), ks.end());
        std::sort(rs.begin(), rs.end());
        kmax = lg((double)ks.back());
        kmed = lg((double)ks[ks.size() / 2]);
        rmed = lg((double)rs[rs.size() / 2]);
    }
    *out = BatchSig(dev, dtype * 2 + (diag == REDSEA_UNIT), lg((double)ks.size()), kmax, kmed, rmed,
                    0);
    return REDSEA_OK;
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
    if (opts && (opts->tile < 0 || opts->tile > kBatchTiles)) return -14;
    // task shape: the caller's, else the autotuner's for this kind of batch
    // (tuned now when REDSEA_TUNE=1 and not yet known), else the default
    int tile = opts ? opts->tile : 0;
    if (tile == 0) {
        BatchSig sig;
        if ((rc = batch_signature(dtype, diag, count, m, n, side, &sig))) return rc;
        {
            std::lock_guard<std::mutex> lock(g_bt_mu);
            auto it = g_bt.find(sig);
            if (it != g_bt.end()) tile = it->second;
        }
        const char* e = std::getenv("REDSEA_TUNE");
        if (tile == 0 && e && std::atoi(e) == 1) {
            std::vector<int64_t> ks(count), rs(count);
            for (int64_t i = 0; i < count; ++i) {
                ks[i] = side == REDSEA_LEFT ? m[i] : n[i];
                rs[i] = side == REDSEA_LEFT ? n[i] : m[i];
            }
            int best = 0;
            rc = redsea_batched_tune(dtype, diag, count, ks.data(), rs.data(), 2, nullptr, &best);
            if (rc) return rc;
            tile = best;
        }
        if (tile == 0) tile = kBatchTileDefault;
    }
    redsea_batch_plan* P = new redsea_batch_plan;
    P->tile = tile;
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
        const int64_t width = 16 * kBatchTileGroups[tile - 1];
        for (int64_t c0 = 0; c0 < c.nrhs; c0 += width) {
            const double w = (double)std::min<int64_t>(width, c.nrhs - c0);
            const double kp = (double)((c.k + 15) / 16 * 16);
            // longest-processing-time first: the chain of k divisions plus the
            // k^2 w / 2 update work, both per tile
            work.push_back({kp * kp * (double)width / 2.0 + 600.0 * kp + w,
                            BatchTask{id, (int32_t)c0}});
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
    // One queue per XCD: systems go to the queues longest-first, each to the
    // least loaded so far (their tiles stay together); each queue is then
    // ordered longest task first.
    std::vector<double> sys_work(sys.size(), 0.0);
    for (auto& w : work) sys_work[(size_t)w.second.sys] += w.first;
    std::vector<int32_t> order;
    for (size_t i = 0; i < sys_work.size(); ++i)
        if (sys_work[i] > 0.0) order.push_back((int32_t)i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return sys_work[(size_t)x] > sys_work[(size_t)y]; });
    std::vector<int> queue_of(sys.size(), 0);
    double load[kBatchQueues] = {};
    for (int32_t i : order) {
        int q = 0;
        for (int u = 1; u < kBatchQueues; ++u)
            if (load[u] < load[q]) q = u;
        queue_of[(size_t)i] = q;
        load[q] += sys_work[(size_t)i];
    }
    std::stable_sort(work.begin(), work.end(),
                     [](const std::pair<double, BatchTask>& x, const std::pair<double, BatchTask>& y) {
                         return x.first > y.first;
                     });
    std::vector<BatchTask> tasks;
    tasks.reserve(work.size());
    for (int q = 0; q < kBatchQueues; ++q) {
        P->queues.start[q] = (int)tasks.size();
        for (auto& w : work)
            if (queue_of[(size_t)w.second.sys] == q) tasks.push_back(w.second);
        P->queues.count[q] = (int)tasks.size() - P->queues.start[q];
    }
    P->ntasks = (int)tasks.size();
    if (sys.empty()) sys.resize(1);
    bool ok = hipMalloc(&P->d_sys, sys.size() * sizeof(BatchSys)) == hipSuccess &&
              hipMalloc(&P->d_tasks, std::max<size_t>(1, tasks.size()) * sizeof(BatchTask)) ==
                  hipSuccess &&
              hipMalloc(&P->d_counter, kBatchCounterInts * sizeof(int)) == hipSuccess;
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
    P->grid = std::max(1, std::min((P->ntasks + 3) / 4, cus * kBatchTileWgPerCu[tile - 1]));
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
        launch_batched(P->dtype, P->unit, kBatchTileGroups[P->tile - 1],
                       kBatchTileDepth[P->tile - 1], P->d_sys, P->d_tasks,
                       P->queues, P->d_counter, info, P->alpha, P->grid, s) != hipSuccess)
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

int redsea_batched_tune(int dtype, int diag, int64_t count, const int64_t* k, const int64_t* nrhs,
                        int reps, double* ms, int* best) {
    if (dtype != REDSEA_F64 && dtype != REDSEA_F32) return -1;
    if (diag != REDSEA_NONUNIT && diag != REDSEA_UNIT) return -2;
    if (count < 0) return -3;
    if (count > 0 && !k) return -4;
    if (count > 0 && !nrhs) return -5;
    if (reps < 1) return -6;
    if (!best) return -8;
    for (int64_t i = 0; i < count; ++i) {
        if (k[i] < 0) return -4;
        if (nrhs[i] < 0) return -5;
    }
    *best = kBatchTileDefault;
    if (count == 0) return REDSEA_OK;
    // generated systems of the batch's shapes (left, lower, no transpose;
    // strict part uniform in (-1, 1), diagonal 1 + sum |row|), one buffer
    const size_t es = dtype == REDSEA_F64 ? 8 : 4;
    std::vector<size_t> aoff(count), boff(count);
    size_t atot = 0, btot = 0;
    int64_t kmax = 1;
    for (int64_t i = 0; i < count; ++i) {
        aoff[i] = atot;
        boff[i] = btot;
        atot += (size_t)k[i] * k[i];
        btot += (size_t)k[i] * nrhs[i];
        kmax = std::max(kmax, k[i]);
    }
    double *A64 = nullptr, *B64 = nullptr, *rows = nullptr;
    void *A = nullptr, *B0 = nullptr, *B = nullptr;
    int* info = nullptr;
    auto cleanup = [&]() {
        if (A64) (void)hipFree(A64);
        if (B64) (void)hipFree(B64);
        if (rows) (void)hipFree(rows);
        if (dtype != REDSEA_F64 && A) (void)hipFree(A);
        if (dtype != REDSEA_F64 && B0) (void)hipFree(B0);
        if (B) (void)hipFree(B);
        if (info) (void)hipFree(info);
    };
    bool ok = hipMalloc(&A64, std::max<size_t>(atot, 1) * 8) == hipSuccess &&
              hipMalloc(&B64, std::max<size_t>(btot, 1) * 8) == hipSuccess &&
              hipMalloc(&rows, (size_t)kmax * 8) == hipSuccess &&
              hipMalloc(&B, std::max<size_t>(btot, 1) * es) == hipSuccess &&
              hipMalloc(&info, (size_t)count * sizeof(int)) == hipSuccess;
    if (ok && dtype != REDSEA_F64)
        ok = hipMalloc(&A, std::max<size_t>(atot, 1) * 4) == hipSuccess &&
             hipMalloc(&B0, std::max<size_t>(btot, 1) * 4) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        cleanup();
        return REDSEA_ERR_ALLOC;
    }
    hipStream_t s = nullptr;
    for (int64_t i = 0; i < count; ++i) {
        if (k[i] == 0 || nrhs[i] == 0) continue;
        if (gen_system_dev(A64 + aoff[i], k[i], k[i], 0.0, 7000 + 2 * (uint64_t)i, rows, s) !=
                hipSuccess ||
            gen_rhs_dev(B64 + boff[i], k[i], k[i], nrhs[i], 7001 + 2 * (uint64_t)i, s) != hipSuccess) {
            cleanup();
            return REDSEA_ERR_HIP;
        }
    }
    if (dtype == REDSEA_F64) {
        A = A64;
        B0 = B64;
    } else if (narrow_dev(A64, (int64_t)atot, (float*)A, s) != hipSuccess ||
               narrow_dev(B64, (int64_t)btot, (float*)B0, s) != hipSuccess) {
        cleanup();
        return REDSEA_ERR_HIP;
    }
    std::vector<const void*> ap(count);
    std::vector<void*> bp(count);
    for (int64_t i = 0; i < count; ++i) {
        ap[i] = (const char*)A + aoff[i] * es;
        bp[i] = (char*)B + boff[i] * es;
    }
    std::vector<int64_t> ld(count);
    for (int64_t i = 0; i < count; ++i) ld[i] = std::max<int64_t>(1, k[i]);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return REDSEA_ERR_HIP;
    }
    int rc = REDSEA_OK;
    double best_ms = -1.0;
    for (int t = 1; t <= kBatchTiles && rc == REDSEA_OK; ++t) {
        redsea_opts o{0, 0, 0, 0.0, t};
        redsea_batch_plan* P = nullptr;
        rc = redsea_batched_plan_create(dtype, REDSEA_LEFT, REDSEA_LOWER, REDSEA_NOTRANS, diag,
                                        count, k, nrhs, 1.0, ap.data(), ld.data(), bp.data(),
                                        ld.data(), &o, &P);
        if (rc) break;
        std::vector<float> tv;
        for (int r = 0; r <= reps && rc == REDSEA_OK; ++r) {
            if (hipMemcpyAsync(B, B0, std::max<size_t>(btot, 1) * es, hipMemcpyDeviceToDevice, s) !=
                hipSuccess) {
                rc = REDSEA_ERR_HIP;
                break;
            }
            (void)hipEventRecord(e0, s);
            rc = redsea_batched_plan_run(P, info, s);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) rc = REDSEA_ERR_HIP;
            float el = 0.f;
            (void)hipEventElapsedTime(&el, e0, e1);
            if (r > 0) tv.push_back(el);  // the first run warms up
        }
        redsea_batched_plan_destroy(P);
        if (rc) break;
        std::sort(tv.begin(), tv.end());
        const double med = tv[tv.size() / 2];
        if (ms) ms[t - 1] = med;
        if (best_ms < 0 || med < best_ms) {  // ties keep the lower index
            best_ms = med;
            *best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cleanup();
    if (rc) return rc;
    // remember the pick for batches of this kind
    BatchSig sig;
    if (batch_signature(dtype, diag, count, k, nrhs, REDSEA_LEFT, &sig) == REDSEA_OK) {
        std::lock_guard<std::mutex> lock(g_bt_mu);
        g_bt[sig] = *best;
    }
    return REDSEA_OK;
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
    if (opts && (opts->tile < 0 || opts->tile > kBatchTiles)) return -15;
    redsea_batch_plan* P = nullptr;
    rc = redsea_batched_plan_create(dtype, side, uplo, trans, diag, count, m, n, alpha, A, lda, B,
                                    ldb, opts, &P);
    if (rc) return rc;
    rc = redsea_batched_plan_run(P, info, stream);
    redsea_batched_plan_destroy(P);  // waits for the launch before freeing descriptors
    return rc;
}

}  // extern "C"
