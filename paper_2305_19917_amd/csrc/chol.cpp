// Cholesky factorisation (redsea_potrf) on the library's solve and products.
//
// The paper names the Cholesky factorisation as the next application of its
// triangular solver (Sec. VIII).  The factorisation is split as the solve is
// in the recursive model (Sec. V-A): with A = [A11 A21^T; A21 A22], n1 rows in
// A11,
//     A11 = L11 L11^T            (recursively),
//     L21 = A21 L11^{-T}         (redsea_trsm, right side: the library's
//                                 triangular solve with n - n1 right-hand
//                                 sides),
//     A22 := A22 - L21 L21^T     (one triangle of tiles on the matrix cores),
//     A22 = L22 L22^T            (recursively),
// down to diagonal blocks of order nb or less, each factored by one workgroup
// (the block in registers, its columns passed on through LDS).  n1 is half the order rounded up to a multiple of nb, so every
// leaf but the last has order nb and the big solves and products come first.
// An upper factorisation A = U^T U runs the same steps on U = L^T through the
// transposed storage: the solve becomes U11^T U12 = A12 (left side) and the
// update A22 -= U12^T U12.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "exec.h"
#include "kernels.h"

namespace redsea {

namespace {

struct CholCtx {
    int dtype;
    bool upper;
    int64_t lda;
    int nb;
    int* info;
    hipStream_t s;
    size_t es;  // element bytes
};

// Address of entry (i, j) of the matrix stored at a0.
char* at(const CholCtx& c, char* a0, int64_t i, int64_t j) {
    return a0 + (size_t)(i + j * c.lda) * c.es;
}

int factor(const CholCtx& c, char* a0, int64_t r0, int64_t n) {
    char* a = at(c, a0, r0, r0);
    if (n <= c.nb) {
        const int64_t sr = c.upper ? c.lda : 1, sc = c.upper ? 1 : c.lda;
        const double fl = (double)n * n * n / 3.0;
        return traced(REDSEA_KERNEL_CHOL_LEAF, fl, c.s, [&] {
                   return launch_potrf_leaf(c.dtype, a, sr, sc, (int)n, r0, c.info, c.s);
               }) == hipSuccess
                   ? REDSEA_OK
                   : REDSEA_ERR_HIP;
    }
    const int64_t n1 = ((n / 2 + c.nb - 1) / c.nb) * c.nb, n2 = n - n1;
    int rc = factor(c, a0, r0, n1);
    if (rc) return rc;
    // panel: L21 = A21 L11^{-T} (lower) or U12 = U11^{-T} A12 (upper)
    const redsea_opts o{REDSEA_VARIANT_RECURSIVE, 0, REDSEA_PREC_NATIVE, 0.0, 0};
    char* panel = c.upper ? at(c, a0, r0, r0 + n1) : at(c, a0, r0 + n1, r0);
    rc = c.upper ? redsea_trsm(c.dtype, REDSEA_LEFT, REDSEA_UPPER, REDSEA_TRANS, REDSEA_NONUNIT, n1,
                               n2, 1.0, a, c.lda, panel, c.lda, &o, c.s)
                 : redsea_trsm(c.dtype, REDSEA_RIGHT, REDSEA_LOWER, REDSEA_TRANS, REDSEA_NONUNIT,
                               n2, n1, 1.0, a, c.lda, panel, c.lda, &o, c.s);
    if (rc) return rc;
    // trailing update of one triangle of A22: C(i, j) -= sum_k P(i, k) P(j, k)
    // for i <= j in the product's coordinates, which is the stored triangle
    char* a22 = at(c, a0, r0 + n1, r0 + n1);
    GemmArgs g{n2, n2, n1, panel, c.lda, panel, c.lda, a22, c.lda};
    const double fl = (double)n2 * n2 * n1;
    if (traced(REDSEA_KERNEL_SYRK, fl, c.s,
               [&] { return launch_syrk(c.dtype, c.upper, !c.upper, g, c.s); }) != hipSuccess)
        return REDSEA_ERR_HIP;
    return factor(c, a0, r0 + n1, n2);
}

}  // namespace

}  // namespace redsea

using namespace redsea;

extern "C" int redsea_potrf(int dtype, int uplo, int64_t n, void* A, int64_t lda, int nb,
                            int* info, void* stream) {
    if (dtype != REDSEA_F64 && dtype != REDSEA_F32) return -1;
    if (uplo != REDSEA_LOWER && uplo != REDSEA_UPPER) return -2;
    if (n < 0) return -3;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (!(nb == 0 || nb == 32 || nb == 64 || nb == 128)) return -6;
    if (!info) return -7;
    if (n > 0 && !A) return -4;
    hipStream_t s = (hipStream_t)stream;
    const int leaf = nb ? nb : kCholLeafDefault;
    // the panel solves take the per-stream buffer, which a graph must not
    // capture: refuse before anything is enqueued
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return REDSEA_ERR_HIP;
    if (cap != hipStreamCaptureStatusNone && n > leaf) return REDSEA_ERR_UNSUPPORTED;
    if (launch_info_clear(info, s) != hipSuccess) return REDSEA_ERR_HIP;
    if (n == 0) return REDSEA_OK;
    CholCtx c{dtype, uplo == REDSEA_UPPER, lda, leaf, info, s,
              dtype == REDSEA_F64 ? sizeof(double) : sizeof(float)};
    return factor(c, (char*)A, 0, n);
}
