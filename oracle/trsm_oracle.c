/*
 * CPU oracle for the dense triangular solve with many right-hand sides.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the HIP path.
 *
 * What it computes is the plain definition of the result.  The paper
 * (Sec. IV) poses L x = b with L dense lower-triangular and extends it to many
 * right-hand sides b sharing one L; its recursive, iterative and blocked
 * models (Sec. V-A, V-B, V-C) only reorder the sums of that solve.  The
 * library follows BLAS xTRSM semantics on top of that:
 *     side = left :  op(A) X = alpha B
 *     side = right:  X op(A) = alpha B
 * with op(A) = A or A^T, A lower or upper, unit or non-unit diagonal, and X
 * overwriting B.  The oracle therefore is textbook substitution on op(A),
 * written with explicit index maps, not a replay of the method:
 *
 *   trsm_plain   : substitution in axpy (column) form, one IEEE division per
 *                  unknown, separate multiply and subtract (built with
 *                  -ffp-contract=off so no fused multiply-add is formed).
 *   trsm_comp    : dot form x_i = (b_i - sum_j t_ij x_j) / t_ii with the sum
 *                  evaluated by Dot2 (TwoProduct via fma + TwoSum, Ogita, Rump
 *                  and Oishi, "Accurate sum and dot product", SIAM J. Sci.
 *                  Comput. 26(6), 2005, Algorithm 5.3), rounded once before
 *                  the division.
 *   residual_comp: R = alpha B - op(A) X (left) or alpha B - X op(A) (right),
 *                  every entry by Dot2 with alpha*b taken as an exact product,
 *                  so R is as accurate as if computed in twice the working
 *                  precision and rounded once.
 *   opnorm       : infinity norm (max row sum) or one norm (max column sum)
 *                  of op(A), honouring the triangle and the unit diagonal.
 *
 * Work is split over right-hand sides only (columns for the left side, rows
 * for the right side).  Each right-hand side is processed by one thread with
 * the same operation order, so results do not depend on the thread count.
 *
 * Flag encoding (same integers as the public header, restated here on
 * purpose so the oracle owns its own copy):
 *   side 0 = left, 1 = right;  uplo 0 = lower, 1 = upper;
 *   trans 0 = no transpose, 1 or 2 = transpose;  diag 0 = non-unit, 1 = unit.
 * All matrices are column-major with leading dimensions >= their row count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* op(A) as an index map.                                              */
/* ------------------------------------------------------------------ */

typedef struct {
    const double* a;
    int64_t lda;
    int uplo;  /* storage triangle of A            */
    int trans; /* 0: op(A) = A, 1: op(A) = A^T     */
    int unit;  /* 1: diagonal taken as one, unread */
} opmat;

/* Element (i, j) of op(A) as a mathematical matrix: zero outside its
 * triangle, one on the diagonal when unit, otherwise the stored entry. */
static double op_at(const opmat* M, int64_t i, int64_t j) {
    int64_t r = M->trans ? j : i; /* row/col in the stored A */
    int64_t c = M->trans ? i : j;
    if (r == c) return M->unit ? 1.0 : M->a[r + c * M->lda];
    if (M->uplo == 0 && r < c) return 0.0;
    if (M->uplo == 1 && r > c) return 0.0;
    return M->a[r + c * M->lda];
}

/* op(A) is lower triangular iff (A lower and not transposed) or
 * (A upper and transposed). */
static int op_is_lower(const opmat* M) { return (M->uplo == 0) != (M->trans != 0); }

/* ------------------------------------------------------------------ */
/* Error-free transformations (Ogita, Rump, Oishi 2005, Sec. 2-3).     */
/* ------------------------------------------------------------------ */

static void two_sum(double a, double b, double* s, double* e) {
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static void two_prod(double a, double b, double* p, double* e) {
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* Dot2 accumulator: the running value is p + s with p the rounded sum and s
 * the accumulated error terms. */
typedef struct {
    double p, s;
} dot2;

static void dot2_init(dot2* d) { d->p = 0.0; d->s = 0.0; }

static void dot2_add_prod(dot2* d, double x, double y) {
    double h, r, q;
    two_prod(x, y, &h, &r);
    two_sum(d->p, h, &d->p, &q);
    d->s = d->s + (q + r);
}

static double dot2_result(const dot2* d) { return d->p + d->s; }

/* ------------------------------------------------------------------ */
/* One right-hand side.                                                */
/*                                                                     */
/* T is the triangular matrix of the vector system T y = c that one     */
/* right-hand side reduces to:                                          */
/*   left side : T = op(A),   y = column j of X, c = alpha * column j   */
/*   right side: T = op(A)^T, y = row i of X,    c = alpha * row i      */
/* t_at(i, j) reads T through the op(A) map.                            */
/* ------------------------------------------------------------------ */

typedef struct {
    opmat M;
    int transposed; /* 1: T = op(A)^T */
} trimat;

static double t_at(const trimat* T, int64_t i, int64_t j) {
    return T->transposed ? op_at(&T->M, j, i) : op_at(&T->M, i, j);
}

static int t_is_lower(const trimat* T) {
    int lower = op_is_lower(&T->M);
    return T->transposed ? !lower : lower;
}

/* Plain substitution, axpy form, on a strided vector y of length m.  On
 * entry y holds c, on exit the solution. */
static void subst_axpy(const trimat* T, int64_t m, double* y, int64_t inc) {
    if (t_is_lower(T)) {
        for (int64_t k = 0; k < m; ++k) {
            double xk = y[k * inc];
            if (!T->M.unit) xk = xk / t_at(T, k, k);
            y[k * inc] = xk;
            for (int64_t i = k + 1; i < m; ++i) {
                double prod = t_at(T, i, k) * xk;
                y[i * inc] = y[i * inc] - prod;
            }
        }
    } else {
        for (int64_t k = m - 1; k >= 0; --k) {
            double xk = y[k * inc];
            if (!T->M.unit) xk = xk / t_at(T, k, k);
            y[k * inc] = xk;
            for (int64_t i = 0; i < k; ++i) {
                double prod = t_at(T, i, k) * xk;
                y[i * inc] = y[i * inc] - prod;
            }
        }
    }
}

/* Compensated substitution, dot form. */
static void subst_dot2(const trimat* T, int64_t m, double* y, int64_t inc) {
    if (t_is_lower(T)) {
        for (int64_t i = 0; i < m; ++i) {
            dot2 d;
            dot2_init(&d);
            dot2_add_prod(&d, y[i * inc], 1.0);
            for (int64_t j = 0; j < i; ++j) dot2_add_prod(&d, -t_at(T, i, j), y[j * inc]);
            double s = dot2_result(&d);
            y[i * inc] = T->M.unit ? s : s / t_at(T, i, i);
        }
    } else {
        for (int64_t i = m - 1; i >= 0; --i) {
            dot2 d;
            dot2_init(&d);
            dot2_add_prod(&d, y[i * inc], 1.0);
            for (int64_t j = i + 1; j < m; ++j) dot2_add_prod(&d, -t_at(T, i, j), y[j * inc]);
            double s = dot2_result(&d);
            y[i * inc] = T->M.unit ? s : s / t_at(T, i, i);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Threading over right-hand sides.                                    */
/* ------------------------------------------------------------------ */

typedef struct {
    int side, mode; /* mode 0 plain, 1 compensated */
    trimat T;
    int64_t m, n; /* B is m x n */
    double alpha;
    double* b;
    int64_t ldb;
    int64_t lo, hi; /* right-hand sides [lo, hi) */
} solve_job;

static void solve_rhs_range(const solve_job* J) {
    for (int64_t r = J->lo; r < J->hi; ++r) {
        double* y;
        int64_t len, inc;
        if (J->side == 0) { y = J->b + r * J->ldb; len = J->m; inc = 1; }
        else { y = J->b + r; len = J->n; inc = J->ldb; }
        if (J->alpha == 0.0) {
            for (int64_t i = 0; i < len; ++i) y[i * inc] = 0.0;
            continue;
        }
        if (J->alpha != 1.0)
            for (int64_t i = 0; i < len; ++i) y[i * inc] = J->alpha * y[i * inc];
        if (J->mode == 0) subst_axpy(&J->T, len, y, inc);
        else subst_dot2(&J->T, len, y, inc);
    }
}

static void* solve_thread(void* arg) {
    solve_rhs_range((const solve_job*)arg);
    return NULL;
}

static int run_split(solve_job* base, int64_t nrhs, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > nrhs) nthreads = (int)(nrhs > 0 ? nrhs : 1);
    pthread_t tid[256];
    solve_job jobs[256];
    int64_t chunk = (nrhs + nthreads - 1) / nthreads;
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *base;
        jobs[t].lo = (int64_t)t * chunk;
        jobs[t].hi = jobs[t].lo + chunk < nrhs ? jobs[t].lo + chunk : nrhs;
        if (jobs[t].lo >= jobs[t].hi) break;
        if (t == 0) continue; /* the caller's thread takes chunk 0 */
        if (pthread_create(&tid[t], NULL, solve_thread, &jobs[t]) != 0) {
            for (int u = 1; u < t; ++u) pthread_join(tid[u], NULL);
            return -1;
        }
        started = t;
    }
    if (jobs[0].lo < jobs[0].hi) solve_rhs_range(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
    return 0;
}

static int solve_common(int mode, int side, int uplo, int trans, int diag, int64_t m,
                        int64_t n, double alpha, const double* a, int64_t lda, double* b,
                        int64_t ldb, int nthreads) {
    if (m <= 0 || n <= 0) return 0;
    solve_job J;
    memset(&J, 0, sizeof J);
    J.side = side;
    J.mode = mode;
    J.T.M.a = a;
    J.T.M.lda = lda;
    J.T.M.uplo = uplo;
    J.T.M.trans = trans != 0;
    J.T.M.unit = diag != 0;
    J.T.transposed = side == 1;
    J.m = m;
    J.n = n;
    J.alpha = alpha;
    J.b = b;
    J.ldb = ldb;
    return run_split(&J, side == 0 ? n : m, nthreads);
}

/* Plain substitution: B := alpha op(A)^{-1} B (left) or alpha B op(A)^{-1}
 * (right). */
int oracle_trsm_plain(int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                      double alpha, const double* a, int64_t lda, double* b, int64_t ldb,
                      int nthreads) {
    return solve_common(0, side, uplo, trans, diag, m, n, alpha, a, lda, b, ldb, nthreads);
}

/* Compensated (Dot2) substitution, same contract as oracle_trsm_plain. */
int oracle_trsm_comp(int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                     double alpha, const double* a, int64_t lda, double* b, int64_t ldb,
                     int nthreads) {
    return solve_common(1, side, uplo, trans, diag, m, n, alpha, a, lda, b, ldb, nthreads);
}

/* ------------------------------------------------------------------ */
/* Compensated residual.                                               */
/* ------------------------------------------------------------------ */

typedef struct {
    int side;
    opmat M;
    int64_t m, n;
    double alpha;
    const double *b, *x;
    int64_t ldb, ldx;
    double* r;
    int64_t ldr;
    int64_t lo, hi;
} resid_job;

static void resid_range(const resid_job* J) {
    int64_t k = J->side == 0 ? J->m : J->n; /* order of op(A) */
    for (int64_t c = J->lo; c < J->hi; ++c) {
        for (int64_t i = 0; i < J->m; ++i) {
            /* left : r_ic = alpha b_ic - sum_p op(A)_ip x_pc
             * right: r_ic = alpha b_ic - sum_p x_ip op(A)_pc */
            dot2 d;
            dot2_init(&d);
            dot2_add_prod(&d, J->alpha, J->b[i + c * J->ldb]);
            for (int64_t p = 0; p < k; ++p) {
                double t = J->side == 0 ? op_at(&J->M, i, p) : op_at(&J->M, p, c);
                double xv = J->side == 0 ? J->x[p + c * J->ldx] : J->x[i + p * J->ldx];
                if (t != 0.0) dot2_add_prod(&d, -t, xv);
            }
            J->r[i + c * J->ldr] = dot2_result(&d);
        }
    }
}

static void* resid_thread(void* arg) {
    resid_range((const resid_job*)arg);
    return NULL;
}

/* R := alpha B - op(A) X (left) or alpha B - X op(A) (right); B, X, R are
 * m x n.  Columns are split across threads. */
int oracle_residual_comp(int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                         double alpha, const double* a, int64_t lda, const double* b,
                         int64_t ldb, const double* x, int64_t ldx, double* r, int64_t ldr,
                         int nthreads) {
    if (m <= 0 || n <= 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > n) nthreads = (int)n;
    resid_job base;
    memset(&base, 0, sizeof base);
    base.side = side;
    base.M.a = a;
    base.M.lda = lda;
    base.M.uplo = uplo;
    base.M.trans = trans != 0;
    base.M.unit = diag != 0;
    base.m = m;
    base.n = n;
    base.alpha = alpha;
    base.b = b;
    base.x = x;
    base.ldb = ldb;
    base.ldx = ldx;
    base.r = r;
    base.ldr = ldr;
    pthread_t tid[256];
    resid_job jobs[256];
    int64_t chunk = (n + nthreads - 1) / nthreads;
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = base;
        jobs[t].lo = (int64_t)t * chunk;
        jobs[t].hi = jobs[t].lo + chunk < n ? jobs[t].lo + chunk : n;
        if (jobs[t].lo >= jobs[t].hi) break;
        if (t == 0) continue;
        if (pthread_create(&tid[t], NULL, resid_thread, &jobs[t]) != 0) {
            for (int u = 1; u < t; ++u) pthread_join(tid[u], NULL);
            return -1;
        }
        started = t;
    }
    if (jobs[0].lo < jobs[0].hi) resid_range(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Norms of op(A).                                                     */
/* ------------------------------------------------------------------ */

/* which = 0: infinity norm (max over rows of the absolute row sum);
 * which = 1: one norm (max over columns of the absolute column sum). */
double oracle_opnorm(int uplo, int trans, int diag, int64_t k, const double* a, int64_t lda,
                     int which) {
    opmat M;
    M.a = a;
    M.lda = lda;
    M.uplo = uplo;
    M.trans = trans != 0;
    M.unit = diag != 0;
    double best = 0.0;
    for (int64_t i = 0; i < k; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < k; ++j) s += fabs(which == 0 ? op_at(&M, i, j) : op_at(&M, j, i));
        if (s > best || s != s) best = s;
    }
    return best;
}
