// Mixed-precision solve with FP64 iterative refinement.
//
// The solve of op(A) X = alpha B (paper Sec. IV, with the models of Sec. V
// for its structure) is computed with low-precision arithmetic and its
// accuracy restored in FP64:
//   X0  = low-precision solve of RN32(alpha B)
//   loop: R = alpha B - op(A) X        (FP64, triangle-masked product)
//         eta = max_j ||R_j|| / (||op(A)|| ||X_j|| + ||alpha B_j||)
//         stop when eta <= tol;  fall back to the FP64 solve on stagnation
//         (eta > eta_prev / 2), a non-finite eta, or max_iter corrections
//         D = low-precision solve of RN32(R_j / ||R_j||)   (per right-hand side)
//         X += ||R_j|| D                (FP64)
// Low precision is FP32 throughout (inner = 1), or BF16 products with FP32
// accumulation and FP32-stored leaves (inner = 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/redsea.h"
#include "exec.h"
#include "kernels.h"
#include "mixed.h"
#include "ozaki.h"

namespace redsea {

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
// Leading dimensions of the low-precision working copies: the BF16 matrix is
// stored by rows padded to 8 elements and the FP32 right-hand sides by columns
// padded to 4, so rows / columns start on 16-byte boundaries (the BF16
// product's 16-byte operand loads).
int64_t ld16(int64_t k) { return (k + 7) / 8 * 8; }
int64_t ldw(int64_t m) { return (m + 3) / 4 * 4; }

struct MixedLayout {
    size_t a32, a16, b0, r, w32, rnorm, xnorm, bnorm, scal, rowsum, ozm, ozx, total;
};

MixedLayout layout(int64_t m, int64_t n, int64_t k, int64_t nrhs, bool bf16, bool ozaki) {
    MixedLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.a32 = take((size_t)k * k * 4);
    L.a16 = take(bf16 ? (size_t)k * ld16(k) * 2 : 0);
    L.b0 = take((size_t)m * n * 8);
    L.r = take((size_t)m * n * 8);
    L.w32 = take((size_t)ldw(m) * n * 4);
    L.rnorm = take((size_t)nrhs * 8);
    L.xnorm = take((size_t)nrhs * 8);
    L.bnorm = take((size_t)nrhs * 8);
    L.scal = take((size_t)nrhs * 8);
    L.rowsum = take((size_t)k * 8);
    L.ozm = take(ozaki ? ozaki_m_bytes(k) : 0);
    L.ozx = take(ozaki ? ozaki_x_bytes(k, nrhs) : 0);
    L.total = off;
    return L;
}

// Pinned host staging for the per-iteration norm read-back, one buffer per
// (device, stream) like the device workspace.  The caller holds the lease
// (the entry's lock) for the whole solve; every copy into the buffer is
// waited for before the solve returns, so growth can free the old one.
struct PinEntry {
    std::mutex mu;
    double* ptr = nullptr;
    size_t doubles = 0;
};
std::mutex g_pin_mu;
std::map<std::pair<int, uintptr_t>, std::unique_ptr<PinEntry>> g_pin;

int pinned(size_t doubles, hipStream_t s, std::unique_lock<std::mutex>& held, double** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return REDSEA_ERR_HIP;
    PinEntry* e = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_pin_mu);
        auto& p = g_pin[{dev, (uintptr_t)s}];
        if (!p) p.reset(new PinEntry);
        e = p.get();
    }
    std::unique_lock<std::mutex> lock(e->mu);
    if (e->doubles < doubles) {
        if (e->ptr) (void)hipHostFree(e->ptr);
        e->ptr = nullptr;
        e->doubles = 0;
        if (hipHostMalloc((void**)&e->ptr, doubles * 8, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            e->ptr = nullptr;
            return REDSEA_ERR_ALLOC;
        }
        e->doubles = doubles;
    }
    held = std::move(lock);
    *out = e->ptr;
    return REDSEA_OK;
}

#define HIPCHK(x)                                         \
    do {                                                  \
        if ((x) != hipSuccess) return REDSEA_ERR_HIP;     \
    } while (0)

}  // namespace

int mixed_solve(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
                const double* A, int64_t lda, double* B, int64_t ldb, int inner, double tol,
                int max_iter, void* work, size_t work_bytes, redsea_mixed_stats* stats,
                const redsea_opts* opts, hipStream_t s) {
    const bool bf16 = (inner & 3) == 2;
    const bool ozaki = (inner & REDSEA_RESIDUAL_INT8) != 0;
    const bool right = side == REDSEA_RIGHT;
    const Canon c64 = canonicalize(REDSEA_F64, side, uplo, trans, diag, m, n, A, lda, B, ldb);
    const int64_t k = c64.k, nrhs = c64.nrhs;
    const bool unit = diag == REDSEA_UNIT;
    const MixedLayout L = layout(m, n, k, nrhs, bf16, ozaki);
    char* ws = (char*)work;
    WsLease lease;
    if (ws) {
        if (work_bytes < L.total) return -16;
    } else {
        int rc = workspace(1, L.total, s, lease);
        if (rc) return rc;
        ws = (char*)lease.ptr;
    }
    float* a32 = (float*)(ws + L.a32);
    void* a16 = ws + L.a16;
    double* b0 = (double*)(ws + L.b0);
    double* r = (double*)(ws + L.r);
    float* w32 = (float*)(ws + L.w32);
    double* rnorm = (double*)(ws + L.rnorm);
    double* xnorm = (double*)(ws + L.xnorm);
    double* bnorm = (double*)(ws + L.bnorm);
    double* scal = (double*)(ws + L.scal);
    double* rowsum = (double*)(ws + L.rowsum);
    void* ozm = ws + L.ozm;
    void* ozx = ws + L.ozx;
    double* host = nullptr;
    std::unique_lock<std::mutex> pin_lock;
    int rc = pinned((size_t)3 * nrhs + (size_t)k, s, pin_lock, &host);
    if (rc) return rc;
    double* h_r = host;
    double* h_x = host + nrhs;
    double* h_aux = host + 2 * nrhs;  // bnorm, then scales
    double* h_row = host + 3 * nrhs;

    const int variant = opts && opts->variant ? opts->variant : VAR_RECURSIVE;
    const int nb = pick_nb(opts ? opts->nb : 0, k);
    const bool m_lower = !c64.reverse;

    // low-precision copies of the triangle, FP64 copy of B, norms of op(A), alpha B
    HIPCHK(launch_convert_tri(0, A, lda, k, uplo, unit, a32, s));
    if (bf16) HIPCHK(launch_convert_rows_bf16(A, lda, k, uplo, unit, c64.op_trans, a16, ld16(k), s));
    // integer residue planes of op(A) for the emulated residual
    if (ozaki) HIPCHK(ozaki_split_m(A, lda, k, uplo, c64.op_trans, unit, ozm, s));
    HIPCHK(launch_copy_scaled(B, ldb, m, n, 1.0, b0, m, s));
    HIPCHK(launch_tri_rowsum(A, lda, k, c64.op_trans, m_lower, unit, rowsum, s));
    HIPCHK(launch_rhs_max(b0, m, m, n, right, std::fabs(alpha), bnorm, s));
    HIPCHK(hipMemcpyAsync(h_row, rowsum, (size_t)k * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_aux, bnorm, (size_t)nrhs * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double anorm = 0.0;
    for (int64_t i = 0; i < k; ++i) anorm = (h_row[i] > anorm || h_row[i] != h_row[i]) ? h_row[i] : anorm;
    std::vector<double> bn(h_aux, h_aux + nrhs);

    auto low_solve = [&]() -> int {
        Canon c32 = canonicalize(REDSEA_F32, side, uplo, trans, diag, m, n, a32, k, w32, ldw(m));
        c32.gemm_bf16 = bf16;
        c32.A16 = a16;
        c32.lda16 = ld16(k);
        return execute(c32, variant, nb, s);
    };

    // X0
    HIPCHK(launch_scale_to_f32(b0, m, m, n, nullptr, right, alpha, w32, ldw(m), s));
    if ((rc = low_solve())) return rc;
    HIPCHK(launch_update(B, ldb, m, n, w32, ldw(m), nullptr, right, false, s));

    const GemmArgs rg{k, nrhs, k, A, lda, B, ldb, r, m};
    double eta = INFINITY, prev = INFINITY;
    int iters = 0;
    bool fell_back = false;
    for (;;) {
        // R = alpha B0 - op(A) X: FP64 products, or the exact integer
        // emulation (as accurate as an FP64 product)
        if (ozaki) {
            HIPCHK(ozaki_product(ozm, m_lower ? 1 : 2, k, nrhs, right, alpha, -1.0, B, ldb, b0, m,
                                 r, m, ozx, s));
        } else {
            HIPCHK(launch_copy_scaled(b0, m, m, n, 1.0, r, m, s));
            HIPCHK(launch_trmm(0, c64.op_trans, right, m_lower ? 1 : 2, unit, alpha, -1.0, rg, s));
        }
        HIPCHK(launch_rhs_max(r, m, m, n, right, 1.0, rnorm, s));
        HIPCHK(launch_rhs_max(B, ldb, m, n, right, 1.0, xnorm, s));
        HIPCHK(hipMemcpyAsync(h_r, rnorm, (size_t)nrhs * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h_x, xnorm, (size_t)nrhs * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        eta = 0.0;
        for (int64_t j = 0; j < nrhs; ++j) {
            const double den = anorm * h_x[j] + bn[j];
            double e = den > 0 ? h_r[j] / den : (h_r[j] > 0 ? INFINITY : 0.0);
            if (!(e == e) || !std::isfinite(h_r[j]) || !std::isfinite(h_x[j])) e = INFINITY;
            eta = std::max(eta, e);
        }
        if (eta <= tol) break;
        if (!std::isfinite(eta) || iters >= max_iter || (iters > 0 && eta > 0.5 * prev)) {
            fell_back = true;
            break;
        }
        prev = eta;
        // D = low solve of R / ||R||, X += ||R|| D
        for (int64_t j = 0; j < nrhs; ++j) h_aux[j] = h_r[j] > 0 ? 1.0 / h_r[j] : 0.0;
        HIPCHK(hipMemcpyAsync(scal, h_aux, (size_t)nrhs * 8, hipMemcpyHostToDevice, s));
        HIPCHK(launch_scale_to_f32(r, m, m, n, scal, right, 1.0, w32, ldw(m), s));
        if ((rc = low_solve())) return rc;
        HIPCHK(launch_update(B, ldb, m, n, w32, ldw(m), rnorm, right, true, s));
        ++iters;
    }
    if (fell_back) {
        // FP64 solve from the kept copy of B
        HIPCHK(launch_copy_scaled(b0, m, m, n, alpha, B, ldb, s));
        Canon c = canonicalize(REDSEA_F64, side, uplo, trans, diag, m, n, A, lda, B, ldb);
        if ((rc = execute(c, variant, nb, s))) return rc;
    }
    if (stats) {
        stats->iterations = iters;
        stats->eta = eta;
        stats->fell_back = fell_back ? 1 : 0;
    }
    return REDSEA_OK;
}

size_t mixed_workspace_bytes(int side, int64_t m, int64_t n, int inner) {
    if (m <= 0 || n <= 0) return 0;
    const int64_t k = side == REDSEA_RIGHT ? n : m;
    const int64_t nrhs = side == REDSEA_RIGHT ? m : n;
    return layout(m, n, k, nrhs, (inner & 3) == 2, (inner & REDSEA_RESIDUAL_INT8) != 0).total;
}

}  // namespace redsea

using namespace redsea;

extern "C" {

size_t redsea_trsm_mixed_workspace_bytes(int side, int64_t m, int64_t n, int inner) {
    return mixed_workspace_bytes(side, m, n, (inner & 3) == 0 ? inner | 1 : inner);
}

int redsea_trsm_mixed(int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                      double alpha, const double* A, int64_t lda, double* B, int64_t ldb,
                      int inner, double tol, int max_iter, void* work, size_t work_bytes,
                      redsea_mixed_stats* stats, void* stream) {
    if (side != REDSEA_LEFT && side != REDSEA_RIGHT) return -1;
    if (uplo != REDSEA_LOWER && uplo != REDSEA_UPPER) return -2;
    if (trans != REDSEA_NOTRANS && trans != REDSEA_TRANS && trans != REDSEA_CONJTRANS) return -3;
    if (diag != REDSEA_NONUNIT && diag != REDSEA_UNIT) return -4;
    if (m < 0) return -5;
    if (n < 0) return -6;
    const int64_t ka = side == REDSEA_LEFT ? m : n;
    if (lda < std::max<int64_t>(1, ka)) return -9;
    if (ldb < std::max<int64_t>(1, m)) return -11;
    if ((inner & ~(3 | REDSEA_RESIDUAL_INT8)) || (inner & 3) == 3) return -12;
    if (stats) {
        stats->iterations = 0;
        stats->eta = 0.0;
        stats->fell_back = 0;
    }
    if (m == 0 || n == 0) return REDSEA_OK;
    if (alpha != 0.0 && A == nullptr) return -8;
    if (B == nullptr) return -10;
    hipStream_t s = (hipStream_t)stream;
    if (alpha == 0.0)
        return launch_scale(REDSEA_F64, B, m, n, ldb, 0.0, s) == hipSuccess ? REDSEA_OK
                                                                          : REDSEA_ERR_HIP;
    if ((inner & 3) == 0) inner |= 1;
    if (!(tol > 0.0)) tol = 1e-12;
    if (max_iter <= 0) max_iter = (inner & 3) == 1 ? 5 : 10;
    return mixed_solve(side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb, inner, tol, max_iter,
                       work, work_bytes, stats, nullptr, s);
}

}  // extern "C"
