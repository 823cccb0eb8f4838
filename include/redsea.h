/*
 * redsea.h -- C interface of libredsea, a dense triangular solver with many
 * right-hand sides for AMD MI355X (gfx950).
 *
 * The computation is the one the ReDSEa paper (arXiv 2305.19917) maps and
 * schedules: the triangular system L x = b of Sec. IV, extended to many
 * right-hand sides that share L, solved by splitting L into a top-left
 * triangle, a bottom-left rectangle and a bottom-right triangle (solve, then
 * update the lower right-hand sides with a matrix product, then solve),
 * arranged in the recursive, iterative or blocked models of computation of
 * Sec. V-A, V-B and V-C.  On top of that the library follows BLAS xTRSM
 * semantics:
 *
 *     side = REDSEA_LEFT :  op(A) X = alpha B      (A is m x m)
 *     side = REDSEA_RIGHT:  X op(A) = alpha B      (A is n x n)
 *
 * with B an m x n matrix that X overwrites, op(A) = A or A^T, A lower or
 * upper triangular (only that triangle is read), and a unit diagonal that is
 * never read when diag = REDSEA_UNIT.
 *
 * Conventions shared by every entry point:
 *   - All matrices are column-major.  Matrix pointers are DEVICE pointers
 *     (memory from hipMalloc or a PyTorch CUDA/HIP tensor) unless a comment
 *     says HOST.  The caller owns every buffer it passes; the library never
 *     frees or retains them beyond the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls are asynchronous on that stream unless stated otherwise.
 *   - Return value (LAPACK info style):
 *        0        success;
 *       -i        argument number i (1-based) is invalid: a bad enum value,
 *                 m or n < 0, lda < max(1, order of A), ldb < max(1, m), or
 *                 a NULL pointer where data must be read or written;
 *       >0        runtime failure, see redsea_status_string():
 *                 REDSEA_ERR_HIP (a HIP call failed), REDSEA_ERR_ALLOC
 *                 (device memory could not be obtained), REDSEA_ERR_NOCONV
 *                 (iterative refinement did not converge and the FP64
 *                 fallback is disabled), REDSEA_ERR_NONFINITE (non-finite
 *                 value in a mixed-precision result),
 *                 REDSEA_ERR_UNSUPPORTED (a valid combination this build
 *                 does not implement).
 *   - Quick return: m == 0 or n == 0 succeeds without touching memory.
 *     alpha == 0 sets B to zero without reading A.
 *   - As in BLAS there is no singularity check: a zero on a non-unit
 *     diagonal propagates Inf/NaN into X.
 */
#ifndef REDSEA_H
#define REDSEA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { REDSEA_LEFT = 0, REDSEA_RIGHT = 1 } redsea_side;
typedef enum { REDSEA_LOWER = 0, REDSEA_UPPER = 1 } redsea_uplo;
/* For real data the conjugate transpose equals the transpose. */
typedef enum { REDSEA_NOTRANS = 0, REDSEA_TRANS = 1, REDSEA_CONJTRANS = 2 } redsea_trans;
typedef enum { REDSEA_NONUNIT = 0, REDSEA_UNIT = 1 } redsea_diag;
/* REDSEA_BF16 is accepted by redsea_gemm_update only: a BF16 matrix operand
 * with FP32 right-hand sides and result (the product of the BF16 refinement
 * mode). */
typedef enum { REDSEA_F64 = 0, REDSEA_F32 = 1, REDSEA_BF16 = 2 } redsea_dtype;

/* Model of computation (paper Sec. V). */
typedef enum {
    REDSEA_VARIANT_AUTO = 0,
    REDSEA_VARIANT_RECURSIVE = 1, /* Sec. V-A: halve into TS, GEMM, TS down to the leaf size */
    REDSEA_VARIANT_ITERATIVE = 2, /* Sec. V-B: fixed leaf size, one GEMM panel after each leaf */
    REDSEA_VARIANT_BLOCKED = 3    /* Sec. V-C: r-1 rounds of equal leaf-size GEMM blocks */
} redsea_variant;

typedef enum {
    REDSEA_PREC_AUTO = 0,
    REDSEA_PREC_NATIVE = 1,   /* arithmetic in the data type            */
    REDSEA_PREC_FP32_IR = 2,  /* FP32 solves + FP64 refinement (F64 only) */
    REDSEA_PREC_BF16_IR = 3   /* BF16 products + FP64 refinement (F64 only) */
} redsea_precision;

/* Solver options; a NULL pointer means every field AUTO.  nb is the leaf
 * (diagonal block) order; 0 = AUTO, otherwise one of 16, 32, 64, 128, 256,
 * 512.  kappa is the caller's estimate of the condition number of op(A); it
 * only informs the automatic choice, never the arithmetic.  When variant, nb
 * and precision are all AUTO the learned picker chooses them (see
 * redsea_pick); if kappa is then 0 (unknown) the library computes
 * max|a_ii| / min|a_ii| (a lower bound on the condition number of a
 * triangular matrix; 1 for a unit diagonal) on the device and waits for that
 * value, so an AUTO call with kappa = 0 synchronizes the stream once.  An
 * AUTO nb beside a fixed variant or precision is 256 for order(A) > 128,
 * else 128.  tile only concerns the batched solver (see redsea_batched_tune)
 * and is ignored elsewhere. */
typedef struct {
    int variant;   /* redsea_variant   */
    int nb;        /* leaf size or 0   */
    int precision; /* redsea_precision */
    double kappa;  /* condition estimate or 0 */
    int tile;      /* batched solves: task shape 1..REDSEA_BATCH_TILES, 0 = AUTO */
} redsea_opts;

enum {
    REDSEA_OK = 0,
    REDSEA_ERR_HIP = 1,
    REDSEA_ERR_ALLOC = 2,
    REDSEA_ERR_NOCONV = 3,
    REDSEA_ERR_NONFINITE = 4,
    REDSEA_ERR_UNSUPPORTED = 5,
    REDSEA_ERR_TOO_LARGE = 6 /* exceeds the fixed scratch of redsea_trsm_noalloc */
};

/*
 * Solve op(A) X = alpha B (left) or X op(A) = alpha B (right) in place.
 *
 * Follows the three-stage split of Sec. IV applied recursively, iteratively
 * or in blocked rounds (Sec. V) as selected by opts.  A recursive solve with
 * at most 256 right-hand sides (where it was measured faster than every
 * split schedule) runs instead as one cooperative dataflow launch over
 * 64-row blocks and groups of 16 right-hand sides, and AUTO solves of such
 * widths take it; the environment variable REDSEA_THIN=1 / 0 takes it for
 * every width / never.  dtype gives the element
 * type of A and B (double or float).  Argument numbers for the -i return:
 * dtype 1, side 2, uplo 3, trans 4, diag 5, m 6, n 7, alpha 8, A 9, lda 10,
 * B 11, ldb 12, opts 13, stream 14.  Temporary device memory (at most
 * 1.5 * order(A) * nb elements plus a few KB: the packed diagonal blocks) is
 * taken from a buffer the library keeps per (device, stream) until the
 * process ends.  It grows in stream order (hipFreeAsync of the old buffer,
 * hipMallocAsync of the new one, both on `stream`), so calls on different
 * streams may run concurrently and calls on one stream never wait for the
 * device.  A call on a stream that is being captured into a HIP graph returns
 * REDSEA_ERR_UNSUPPORTED (a cached buffer could be freed before the graph is
 * replayed); a batched plan (below) owns its memory and may be captured.
 */
int redsea_trsm(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                double alpha, const void* A, int64_t lda, void* B, int64_t ldb,
                const redsea_opts* opts, void* stream);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as redsea_trsm (same arguments, numbers and kernels; for a given
 * variant and nb the result is bitwise that of redsea_trsm) in native
 * precision only, with its scratch memory (the packed diagonal blocks, or
 * the flags of the one-launch solve for thin right-hand sides) in a
 * fixed device array of REDSEA_NOALLOC_SCRATCH_BYTES that the library holds
 * on each device it runs on until the process ends.  It calls no hipMalloc,
 * hipFree or other allocating routine and never waits for the device, so it
 * may be captured into a graph; the first call on a device looks up the
 * array's address (hipGetSymbolAddress), so make one call there before
 * capturing, an empty one (m = 0) will do.  variant AUTO means recursive, nb AUTO is 256
 * above order 128, else 128 (no picker, no tuner); precision AUTO or NATIVE,
 * and REDSEA_ERR_UNSUPPORTED for the refinement modes.  A problem whose
 * packed diagonal blocks exceed the array (FP64 with nb 256: order above
 * about 11000) returns REDSEA_ERR_TOO_LARGE before any device work.  Every
 * call on one device shares that device's array: calls that overlap in time
 * on one device (different streams, or several host threads) race and must
 * be ordered by the caller.  Argument numbers as in redsea_trsm.
 */
#define REDSEA_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int redsea_trsm_noalloc(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                        double alpha, const void* A, int64_t lda, void* B, int64_t ldb,
                        const redsea_opts* opts, void* stream);

/*
 * Variable-size batch of independent solves sharing flags and alpha
 * (thousands of uneven systems in one launch; each system is the solve of
 * Sec. IV).
 * m, n, lda, ldb: HOST arrays of `count` entries.  A, B: HOST arrays of
 * `count` DEVICE pointers.  info: DEVICE int array of `count` entries that
 * receives 0 or REDSEA_ERR_NONFINITE for a system whose result holds a
 * non-finite value.  Systems of order up to 1024 are solved together by one
 * persistent launch (tasks of up to 16 right-hand sides, longest first);
 * larger ones by the single-system path on the same stream.  The return
 * value is 0, the -i code of the first invalid argument (for the per-system
 * arrays, i is the array's position), or a runtime failure code.  Argument
 * numbers: dtype 1, side 2, uplo 3, trans 4, diag 5, count 6, m 7, n 8,
 * alpha 9, A 10, lda 11, B 12, ldb 13, info 14, opts 15, stream 16.  This
 * one-shot form builds a plan, runs it and frees it, which waits for the
 * device; repeated batches should use the plan calls below.
 */
int redsea_trsm_batched(int dtype, int side, int uplo, int trans, int diag, int64_t count,
                        const int64_t* m, const int64_t* n, double alpha,
                        const void* const* A, const int64_t* lda, void* const* B,
                        const int64_t* ldb, int* info, const redsea_opts* opts, void* stream);

/*
 * Batched plan: the host work of redsea_trsm_batched (argument checks,
 * canonical descriptors, task order, one synchronous upload) done once, so
 * that redsea_batched_plan_run() is kernel launches only and may be captured
 * in a hipGraph and replayed: every device buffer a run uses (descriptors,
 * task list, the packed diagonal blocks of systems above order 1024) is
 * allocated by create and owned by the plan.  The plan keeps the device
 * pointers it was created with; the caller keeps those buffers alive and
 * unchanged in shape.
 * create: arguments 1-13 as in redsea_trsm_batched, opts 14, out 15 (HOST
 * pointer receiving the plan).  run: plan 1, info 2 (DEVICE int[count]),
 * stream 3; calls of one plan must not overlap in time.  destroy waits for
 * the device and frees the plan (NULL is ignored).
 */
typedef struct redsea_batch_plan redsea_batch_plan;
int redsea_batched_plan_create(int dtype, int side, int uplo, int trans, int diag, int64_t count,
                               const int64_t* m, const int64_t* n, double alpha,
                               const void* const* A, const int64_t* lda, void* const* B,
                               const int64_t* ldb, const redsea_opts* opts,
                               redsea_batch_plan** out);
int redsea_batched_plan_run(redsea_batch_plan* plan, int* info, void* stream);
void redsea_batched_plan_destroy(redsea_batch_plan* plan);

/*
 * Triangular matrix product (BLAS xTRMM extended to an output operand):
 *     side = REDSEA_LEFT :  C := beta C + alpha op(A) B      (A is m x m)
 *     side = REDSEA_RIGHT:  C := beta C + alpha B op(A)      (A is n x n)
 * with B and C m x n (they must not overlap), A triangular (only its uplo
 * triangle is read; a unit diagonal is never read), C not read when beta is
 * 0.  It is the product the update stage of the split (Sec. IV) performs
 * when the whole triangle multiplies, and with beta = alpha_b, alpha = -1,
 * B = X it is the residual alpha_b B - op(A) X of a solve.  method
 * REDSEA_TRMM_MFMA: products on the matrix cores in dtype (FP64 or FP32),
 * only the tiles that meet the triangle.  method REDSEA_TRMM_INT8 (FP64
 * only): the product is emulated exactly in integer arithmetic (Ozaki scheme
 * II: rows of op(A) and columns of B rounded to 53-bit integers after
 * power-of-two scaling, 16 modular products on the INT8 matrix cores,
 * Chinese-remainder reconstruction), so its error is that of rounding each
 * row / column to 53 bits relative to its largest entry -- the accuracy of an
 * FP64 product, not FP64 arithmetic.  Workspace (INT8 method: about
 * 16 (k^2 + 2 k nrhs) bytes, k the order of A) comes from the per-stream
 * buffer described at redsea_trsm.  Argument numbers: dtype 1, side 2, uplo 3,
 * trans 4, diag 5, m 6, n 7, alpha 8, A 9, lda 10, B 11, ldb 12, beta 13,
 * C 14, ldc 15, method 16, stream 17.
 */
enum { REDSEA_TRMM_MFMA = 0, REDSEA_TRMM_INT8 = 1 };
int redsea_trmm(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                double beta, void* C, int64_t ldc, int method, void* stream);

/*
 * Cholesky factorisation of a symmetric positive definite n x n matrix in
 * place (LAPACK xPOTRF semantics): A = L L^T with L lower (uplo REDSEA_LOWER)
 * or A = U^T U with U upper (REDSEA_UPPER).  Only the uplo triangle of A is
 * read, and the factor overwrites it; the other strict triangle is neither
 * read nor written.  The paper names this factorisation as the next
 * application of its solver (Sec. VIII); here it is built on that solver.
 * The matrix is split as the recursive model splits a solve (Sec. V-A):
 * factor A11 (order n1, half of n rounded up to a multiple of nb), solve
 * L21 L11^T = A21 with redsea_trsm, update A22 -= L21 L21^T on the matrix
 * cores (only the tiles of the stored triangle), factor A22; blocks of order
 * nb or less are factored by one workgroup (the block held in registers,
 * each column passed on through LDS).  nb: 0 (AUTO, 128), 32, 64 or 128.  info: DEVICE int that receives 0, or i > 0 when the leading minor
 * of order i is not positive definite; the factorisation then stops (later
 * diagonal blocks are skipped), the factor's first i - 1 columns are final
 * and the rest of the triangle is unspecified.  Read info after the stream
 * has completed the call.  Temporary memory is that of redsea_trsm (the
 * per-stream buffer): on a stream being captured into a graph, an order
 * above nb returns REDSEA_ERR_UNSUPPORTED before anything is enqueued.
 * Argument numbers: dtype 1, uplo 2, n 3, A 4, lda 5, nb 6, info 7,
 * stream 8.
 */
int redsea_potrf(int dtype, int uplo, int64_t n, void* A, int64_t lda, int nb, int* info,
                 void* stream);

/*
 * Autotuner of the batched solver's task shape (the library picks the task
 * shape with its own tuner rather than a fixed rule).  Candidates t = 1..12 are
 * {16, 32} right-hand sides per wave task (a task of 32 uses each loaded
 * block of the triangle for two groups of 16, halving reads of the matrix)
 * x {1, 2, 4} steps of the left-looking product with operands in flight
 * x {2, 4} workgroups of four waves per CU in the persistent grid, in that
 * nesting order (t = 1: 16 columns, depth 1, 2 workgroups per CU); every
 * candidate does the same arithmetic on every column, so the result does not
 * depend on the pick.  Generates, on the device, left / lower
 * / no-transpose systems of the given orders k[i] and right-hand-side counts
 * nrhs[i] (HOST arrays; strict lower part uniform in (-1, 1), diagonal
 * 1 + sum |row|), times every candidate (median of `reps` after a warm-up),
 * writes the milliseconds to ms[0..11] (HOST, optional) and the fastest
 * candidate to *best (ties: the lower index), and remembers that pick for
 * later batches of the same kind on this device (data type, unit diagonal,
 * and the rounded log2 of the system count, of the largest and median orders
 * and of the median right-hand-side count).  Batched calls with opts->tile = 0
 * use a remembered pick, else tune first when the environment variable
 * REDSEA_TUNE is 1, else take candidate 1.  Synchronous; allocates and frees
 * its own device memory.  Argument numbers: dtype 1, diag 2, count 3, k 4,
 * nrhs 5, reps 6, ms 7, best 8.
 */
enum { REDSEA_BATCH_TILES = 12 };
int redsea_batched_tune(int dtype, int diag, int64_t count, const int64_t* k, const int64_t* nrhs,
                        int reps, double* ms, int* best);

/* Statistics of one mixed-precision solve (host struct). */
typedef struct {
    int iterations; /* refinement corrections applied            */
    double eta;     /* last normwise backward error estimate      */
    int fell_back;  /* 1 if the FP64 solve produced the result     */
} redsea_mixed_stats;

/*
 * FP64 solve computed with low-precision inner solves and FP64 iterative
 * refinement (FP64 accuracy from faster low-precision solves): X0 from an
 * FP32 (inner = 1) or BF16-product (inner = 2) solve, then repeated
 * R = alpha B - op(A) X in FP64
 * (with inner | REDSEA_RESIDUAL_INT8: by the exact integer emulation of
 * redsea_trmm's REDSEA_TRMM_INT8 method, a labelled variant),
 * a low-precision correction solve and X += D in FP64, until the normwise
 * backward error is at most tol (tol <= 0 means 1e-12) or max_iter
 * (<= 0: 5 for FP32, 10 for BF16) is reached; on stagnation or no
 * convergence it falls back to the FP64 solve.  inner = 0 (or a bare
 * REDSEA_RESIDUAL_INT8) means FP32; any other value returns -12.
 * work/work_bytes: optional DEVICE workspace of at least
 * redsea_trsm_mixed_workspace_bytes(side, m, n, inner) bytes (the same inner
 * code, flag included); NULL uses the library's per-(device, stream) buffer
 * as redsea_trsm does.  stats: optional HOST struct.  This call synchronizes
 * the stream once per refinement step to read the convergence test.
 * Argument numbers:
 * side 1, uplo 2, trans 3, diag 4, m 5, n 6, alpha 7, A 8, lda 9, B 10,
 * ldb 11, inner 12, tol 13, max_iter 14, work 15, work_bytes 16, stats 17,
 * stream 18.
 */
enum { REDSEA_RESIDUAL_INT8 = 16 };
int redsea_trsm_mixed(int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                      double alpha, const double* A, int64_t lda, double* B, int64_t ldb,
                      int inner, double tol, int max_iter, void* work, size_t work_bytes,
                      redsea_mixed_stats* stats, void* stream);

/* Bytes of device workspace redsea_trsm_mixed needs for this shape. */
size_t redsea_trsm_mixed_workspace_bytes(int side, int64_t m, int64_t n, int inner);

/* Static, human-readable text for a return code. */
const char* redsea_status_string(int code);

/*
 * Schedule inspection (HOST only, no device work): writes the task list the
 * planner builds for a lower-triangular order-m solve with leaf size nb and
 * the given variant, in canonical (forward-substitution) coordinates.
 * Each task is 6 int64 values {kind, row0, rows, col0, cols, round}:
 *   kind 0 = leaf solve of rows [row0, row0+rows);
 *   kind 1 = product update B[row0:row0+rows] -= T[row0:.., col0:col0+cols] X[col0:..];
 *   round  = launch group (tasks with equal round run in one launch).
 * Returns the number of tasks (also when it exceeds max_tasks, in which case
 * only max_tasks are written), or a negative -i for an invalid argument.
 * Follows the recursive split of Sec. V-A, the iterative panels of Sec. V-B
 * and the blocked rounds of Sec. V-C.
 */
int64_t redsea_schedule(int variant, int64_t m, int nb, int64_t* tasks, int64_t max_tasks);

/*
 * Product update C := C - op(A) op(X), the matrix-matrix product that the
 * update stage of the split (Sec. IV, stage 2; Sec. V-A for many right-hand
 * sides) performs, on the same MFMA kernels the solver uses.  op(A) is M x K:
 * A[i + k*lda] (transa = 0) or A[k + i*lda] (transa = 1).  transx = 0: X is
 * K x N at X[k + j*ldx] and C is M x N at C[i + j*ldc]; transx = 1: both are
 * stored transposed, X[j + k*ldx] and C[j + i*ldc].  dtype REDSEA_F64 and
 * REDSEA_F32: A, X and C of that type.  dtype REDSEA_BF16: A holds BF16
 * values, X and C FP32; each X value is rounded to BF16 (nearest even) and
 * the products of BF16 values are accumulated in FP32 before C is updated
 * (the product of the BF16 refinement mode).  tile selects a kernel tile
 * configuration (0 .. 17) or -1 for the default (BF16: -1 only).  Argument numbers:
 * dtype 1, transa 2, transx 3, M 4, N 5, K 6, A 7, lda 8, X 9, ldx 10, C 11,
 * ldc 12, tile 13, stream 14.  Asynchronous on stream.
 */
int redsea_gemm_update(int dtype, int transa, int transx, int64_t M, int64_t N, int64_t K,
                       const void* A, int64_t lda, const void* X, int64_t ldx, void* C,
                       int64_t ldc, int tile, void* stream);

/*
 * Kernel timing trace (HOST calls).  Between redsea_trace_begin() and
 * redsea_trace_end() every kernel the solver launches is bracketed by HIP
 * events on its stream.  redsea_trace_end() waits for those events and
 * writes, for each kernel class k < nkinds (REDSEA_KERNEL_*), the number of
 * launches, their summed duration in milliseconds and their summed
 * algorithmic flops (product: 2*M*N*K; leaf: rows^2 * right-hand sides;
 * Cholesky block of order b: b^3 / 3; triangular update: n^2 k for an n x n
 * triangle and k columns).
 * The three output arrays are HOST arrays of nkinds entries owned by the
 * caller.  Returns 0, -4 for bad arrays, or REDSEA_ERR_HIP.  Tracing adds a
 * pair of event records per launch; it is meant for measurement, not for
 * production calls.
 */
enum {
    REDSEA_KERNEL_PACK = 0,       /* diagonal-block packing            */
    REDSEA_KERNEL_LEAF = 1,       /* leaf solve (Sec. V white triangles) */
    REDSEA_KERNEL_GEMM = 2,       /* one product update (grey rectangle) */
    REDSEA_KERNEL_GEMM_GROUP = 3, /* one blocked round of products       */
    REDSEA_KERNEL_THIN = 4,       /* whole solve as one dataflow launch  */
    REDSEA_KERNEL_CHOL_LEAF = 5,  /* Cholesky of one diagonal block      */
    REDSEA_KERNEL_SYRK = 6,       /* Cholesky trailing update, one triangle */
    REDSEA_KERNEL_CLASSES = 7
};
void redsea_trace_begin(void);
int redsea_trace_end(int64_t* launches, double* ms, double* flops, int nkinds);

/*
 * Candidate schedules of the picker: index = 15*(variant-1) + 3*nb_index +
 * precision_index with variant in {recursive, iterative, blocked}, nb in
 * {32, 64, 128, 256, 512} and precision in {native, FP32+IR, BF16+IR}: 45
 * candidates.  redsea_candidate decodes an index (returns -1 if out of
 * range).  HOST call.
 */
enum { REDSEA_CANDIDATES = 45 };
int redsea_candidate(int index, int* variant, int* nb, int* precision);

/*
 * Exhaustive autotuner for one shape (the timings it produces train the
 * picker, and the picker falls back to it).  Generates a
 * left/lower/no-transpose system of order n with nrhs right-hand sides on the
 * device (strict lower part uniform in (-1, 1) from a counter-based hash of
 * (seed, i, j); diagonal 1 + sum|row| when c <= 0, else the constant
 * c * (1 + max row sum), which sets the condition number), then times each
 * listed candidate in the given order: `reps` runs after one warm-up, B
 * restored between runs, median in milliseconds written to ms[i] (-1 for a
 * candidate that does not apply, e.g. refinement for FP32 data); a candidate
 * whose warm-up run already takes more than three times the best median so
 * far is not repeated and reports that one run.  cand: HOST array of ncand indices.
 * Synchronous; allocates and frees its own device buffers.  Argument
 * numbers: dtype 1, n 2, nrhs 3, c 4, seed 5, reps 6, cand 7, ncand 8, ms 9,
 * stream 10.
 */
int redsea_tune_shape(int dtype, int64_t n, int64_t nrhs, double c, uint64_t seed, int reps,
                      const int* cand, int ncand, double* ms, void* stream);

/*
 * Learned picker: a 3-layer FP32 MLP (5 -> 64 -> 64 -> 45, ReLU) that maps
 * (log2 n, log2 nrhs, dtype, log10 kappa, log2 batch), normalised, to the
 * predicted log time of each candidate.  Parameters are packed as W1 (64x5,
 * row-major), b1, W2 (64x64), b2, W3 (45x64), b3: redsea_mlp_param_count()
 * floats.  All pointers below are DEVICE pointers; X is nb x 5 row-major
 * (already normalised), Y, T and mask are nb x 45.  The kernels are
 * deterministic (no atomics).
 *   forward: Y = MLP(X).
 *   grad   : gradient of the masked mean squared error
 *            sum(mask (Y - T)^2) / sum(mask) into grad (packed like params)
 *            and the loss into loss[0].
 *   adam   : one Adam step (bias-corrected, step >= 1) on params with moment
 *            buffers m, v (packed like params, zero-initialised by the caller).
 * Argument numbers follow the declaration order.
 */
int redsea_mlp_param_count(void);
int redsea_mlp_forward(const float* params, const float* X, int64_t nb, float* Y, void* stream);
int redsea_mlp_grad(const float* params, const float* X, const float* T, const float* mask,
                    int64_t nb, float* grad, float* loss, void* stream);
int redsea_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr,
                    float beta1, float beta2, float eps, void* stream);

/*
 * Picker decision for a solve (HOST call, no device work): the candidate
 * index the library would use for a left solve of order n with nrhs
 * right-hand sides, data type dtype and condition estimate kappa (<= 0:
 * unknown), or -1 when no trained weights are loaded.  Outside the range of
 * orders and widths the network was trained on it is not consulted and the
 * default schedule is returned (recursive, native precision, nb 256 above
 * order 128, else 128).  *confident is set to 1 when the shape is inside
 * the training range and the best two predictions differ by more than 5 %.  Weights come from the file named by
 * REDSEA_MLP_WEIGHTS, else picker_weights.txt next to the library;
 * redsea_mlp_load(path) loads a file explicitly (returns 0 or -1).
 */
int redsea_pick(int dtype, int64_t n, int64_t nrhs, double kappa, int* confident);
int redsea_mlp_load(const char* path);

/* Diagnostic, not part of the solver: the achievable matrix-core rate.
 * Launches, asynchronously on `stream`, 4096 workgroups of four waves, each
 * wave running eight independent chains of `iters` (rounded up to a multiple
 * of 16) 16x16x4 MFMAs in `dtype`
 * (REDSEA_F64 or REDSEA_F32), and writes one checksum per thread to `out`
 * (device, caller-owned, at least 4096*256 elements of `dtype`).  Returns the
 * number of floating-point operations performed, so that flops / elapsed time
 * measured by the caller with events on `stream` is the achieved rate; -1 for
 * a bad dtype or iters <= 0, -3 for a missing or short `out`, -100 when the
 * launch fails.  The MI355X datasheet roofs are 78.6 (FP64) and 157.3 (FP32)
 * TFLOP/s. */
int64_t redsea_mfma_peak(int dtype, int64_t iters, void* out, int64_t out_elems, void* stream);

/* Library version as "major.minor.patch+build", build being the first 12 hex
 * digits of the SHA-256 of the sources it was compiled from. */
const char* redsea_version(void);

#ifdef __cplusplus
}
#endif

#endif /* REDSEA_H */
