/*
 * CPU oracle for the Cholesky factorisation (TEST INFRASTRUCTURE ONLY).
 *
 * Nothing in the GPU library links, includes or calls this file; only the
 * test suite and the measurement scripts load it.  It shares no code with the
 * HIP path.
 *
 * The paper names the Cholesky factorisation as the next application of its
 * triangular solver (Sec. VIII).  Its result has a plain definition: for a
 * symmetric positive definite A, the unique lower-triangular L with a
 * positive diagonal and L L^T = A.  Equating column j of L L^T with column j
 * of A, in increasing j, gives every entry of L from entries already known:
 *
 *     l_jj = sqrt(a_jj - sum_{k<j} l_jk^2),
 *     l_ij = (a_ij - sum_{k<j} l_ik l_jk) / l_jj        (i > j),
 *
 * and that is what oracle_potrf computes: each sum in increasing k, every
 * multiply and subtract separately rounded (the file is built with
 * -ffp-contract=off), IEEE square root and division.  The bracket under the
 * square root is the pivot of column j; when it is not positive (or NaN) the
 * leading minor of order j + 1 is not positive definite, the function
 * returns j + 1 and leaves columns j and later as they were (columns before
 * j hold the factor).  uplo = 1 factors A = U^T U with U = L^T read from and
 * written to the upper triangle.  The other strict triangle is neither read
 * nor written.
 *
 * oracle_chol_residual gives, for listed entries (i, j) of the stored
 * triangle, r_ij = a_ij - (F F^T)_ij with the sum by Dot2 (TwoProduct via
 * fma and TwoSum, Ogita, Rump and Oishi, "Accurate sum and dot product", SIAM
 * J. Sci. Comput. 26(6), 2005, Algorithm 5.3; restated here, this file owns
 * its copy) and d_ij = (|F| |F|^T)_ij, the quantities of the componentwise
 * backward-error bound of Cholesky (Higham, "Accuracy and Stability of
 * Numerical Algorithms", 2nd ed., Thm 10.3: |A - L L^T| <= gamma_{n+1} |L||L^T|).
 *
 * Flag encoding: uplo 0 = lower, 1 = upper.  Column-major, lda >= n.
 */
#include <math.h>
#include <stdint.h>

/* Entry (i, j) of the lower factor's storage: L(i, j) itself for uplo 0,
 * U(j, i) for uplo 1. */
static int64_t at(int uplo, int64_t i, int64_t j, int64_t lda) {
    return uplo == 0 ? i + j * lda : j + i * lda;
}

int oracle_potrf(int uplo, int64_t n, double* a, int64_t lda) {
    for (int64_t j = 0; j < n; ++j) {
        double piv = a[at(uplo, j, j, lda)];
        for (int64_t k = 0; k < j; ++k) {
            const double l = a[at(uplo, j, k, lda)];
            piv = piv - l * l;
        }
        if (!(piv > 0.0)) return (int)(j + 1);
        const double ljj = sqrt(piv);
        for (int64_t i = j + 1; i < n; ++i) {
            double s = a[at(uplo, i, j, lda)];
            for (int64_t k = 0; k < j; ++k) s = s - a[at(uplo, i, k, lda)] * a[at(uplo, j, k, lda)];
            a[at(uplo, i, j, lda)] = s / ljj;
        }
        a[at(uplo, j, j, lda)] = ljj;
    }
    return 0;
}

static void two_sum(double a, double b, double* s, double* e) {
    const double x = a + b;
    const double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* Entries (pi[p], pj[p]) of the lower storage, pi >= pj, of A and of the
 * computed factor F (same uplo): r[p] = A - F F^T there (Dot2), d[p] =
 * (|F||F|^T) there (plain). */
void oracle_chol_residual(int uplo, int64_t n, const double* a, int64_t lda, const double* f,
                          int64_t ldf, int64_t npairs, const int64_t* pi, const int64_t* pj,
                          double* r, double* d) {
    (void)n;
    for (int64_t p = 0; p < npairs; ++p) {
        const int64_t i = pi[p], j = pj[p];
        /* Dot2 of a_ij - sum_{k<=j} f_ik f_jk: start from a_ij, add -f_ik f_jk */
        double s = a[at(uplo, i, j, lda)], c = 0.0, mag = 0.0;
        for (int64_t k = 0; k <= j; ++k) {
            const double x = f[at(uplo, i, k, ldf)], y = f[at(uplo, j, k, ldf)];
            const double h = -(x * y);
            const double l = fma(-x, y, -h); /* -(x y) = h + l exactly */
            double t, q;
            two_sum(s, h, &t, &q);
            s = t;
            c = c + (q + l);
            mag = mag + fabs(x) * fabs(y);
        }
        r[p] = s + c;
        d[p] = mag;
    }
}
