// Host-side launchers of the HIP kernels (gfx950).  Every launcher returns
// the hipError_t of its launch.  Matrix coordinates are canonical: T is the
// lower-triangular operator of a forward substitution, element (i, j) at
// A + a_off + i * tr + j * tc (strides may be negative); B rows likewise.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace redsea {

// Canonical view of the triangular operand: T(i, j) = base[off + i*tr + j*tc].
struct TriView {
    const void* base;
    int64_t off, tr, tc;
};

// Canonical view of the right-hand sides: B(i, j) = base[off + i*br + j*bc].
struct RhsView {
    void* base;
    int64_t off, br, bc;
};

// Elements of one packed leaf block: the nb x nb square, for nb = 256
// followed by its 120 off-diagonal 16 x 16 blocks in MFMA A-operand order.
inline int64_t leaf_block_elems(int nb) {
    return (int64_t)nb * nb + (nb == 256 ? 120 * 256 : 0);
}

// Copies the diagonal blocks of T into `packed`: block p (rows
// [p*nb, p*nb+nb)) becomes, at p * leaf_block_elems(nb), an nb x nb
// column-major square whose lower triangle holds T and whose rows past m are
// the identity (for nb = 256 followed by the negated off-diagonal 16 x 16
// blocks in MFMA A-operand order).  nblk blocks.  unit: the diagonal is taken
// as one and not read.
hipError_t launch_pack_diag(int dtype, const TriView& T, int64_t m, int nb, int64_t first_blk,
                            int64_t nblk, bool unit, void* packed, hipStream_t s);

// Solves the leaf at rows [row0, row0+rows) for all ncols columns, reading the
// packed leaf block `pblk` (leaf_block_elems(nb) elements, nb one of 16, 32,
// 64, 128, 256; rows <= nb).  unit: skip the division.
hipError_t launch_leaf(int dtype, int nb, const void* pblk, int64_t rows, const RhsView& B,
                       int64_t row0, int64_t ncols, bool unit, hipStream_t s);

// Plain-layout product update in the library's storage coordinates:
//   C(i, j) -= sum_k A(i, k) X(k, j),  i < M, j < N, k < K
// A(i, k) = a[i + k*lda] (a_trans = false) or a[k + i*lda] (a_trans = true);
// X(k, j) = x[k + j*ldx] and C(i, j) = c[i + j*ldc] (rhs_trans = false) or
// x[j + k*ldx] and c[j + i*ldc] (rhs_trans = true).
struct GemmArgs {
    int64_t M, N, K;
    const void* a;
    int64_t lda;
    const void* x;
    int64_t ldx;
    void* c;
    int64_t ldc;
};

// Triangular product C := beta C + gamma M X with M the k x k triangle of the
// library's storage coordinates: M(i, j) = a[i + j*lda] (a_trans false) or
// a[j + i*lda]; lower (tri = 1) or upper (tri = 2) part only, unit diagonal
// taken as one and not read; C is not read when beta is 0.  dtype 0 (FP64)
// or 1 (FP32).  M = N rows/cols of the args; X and C as in a product update.
// With gamma = -1 this is the residual R = beta B - M X of a solve.
hipError_t launch_trmm(int dtype, bool a_trans, bool rhs_trans, int tri, bool unit, double beta,
                       double gamma, const GemmArgs& g, hipStream_t s);
// Product update restricted to one triangle: C(i, j) -= sum_k A(i, k) X(k, j)
// for i <= j only (M == N; the entries with i > j are neither read nor
// written), layouts as in a product update, with a_trans != rhs_trans: the
// two layouts in which X = A^T stored as A (x = a, ldx = lda) makes this the
// trailing update A22 -= L21 L21^T of a lower Cholesky factorisation (a_trans
// false: C's i <= j is the storage's lower triangle) or A22 -= U12^T U12 of an
// upper one (a_trans true).  Any other operands are allowed too.
hipError_t launch_syrk(int dtype, bool a_trans, bool rhs_trans, const GemmArgs& g, hipStream_t s);
// tile < 0 picks the default tile configuration for the shape.
hipError_t launch_gemm(int dtype, bool a_trans, bool rhs_trans, const GemmArgs& g, hipStream_t s,
                       int tile = -1);
int gemm_tile_count();
int gemm_default_tile(int dtype, int64_t M, int64_t N, int64_t K);

// Several independent products of the same layouts in one launch (a blocked
// round, Sec. V-C).  The descriptors travel as kernel arguments, so at most
// kMaxGroup per launch; no two of them may write the same rows of C.
constexpr int kMaxGroup = 48;
struct GemmGroup {
    int count;
    GemmArgs g[kMaxGroup];
};
hipError_t launch_gemm_group(int dtype, bool a_trans, bool rhs_trans, const GemmGroup& grp,
                             hipStream_t s, int tile = -1);

// B(i, j) := alpha * B(i, j) over an m x n column-major matrix (alpha == 0
// writes zeros without reading B).
hipError_t launch_scale(int dtype, void* b, int64_t m, int64_t n, int64_t ldb, double alpha,
                        hipStream_t s);

// out[0] := max |T(i, i)|, out[1] := min |T(i, i)| over i < k (device doubles).
hipError_t launch_diag_extremes(int dtype, const TriView& T, int64_t k, double* out,
                                hipStream_t s);

// The whole canonical solve as one persistent dataflow launch over tasks
// (64-row block, group of up to 64 right-hand sides), cooperative so that
// every workgroup is resident; blocks wait on per-group counters of solved
// blocks in `flags`, which must hold thin_flag_count(n, nrhs) ints of device
// memory.
int64_t thin_flag_count(int64_t n, int64_t nrhs);
hipError_t launch_thin(int dtype, const TriView& L, const RhsView& B, int64_t n, int64_t ncols,
                       bool unit, int* flags, hipStream_t s);

// Cholesky factorisation of one diagonal block of order b <= kCholLeafMax in
// place: the lower factor L of the block whose entry (i, j), i >= j, is at
// a[i*sr + j*sc] (sr = 1, sc = lda for a lower factorisation; sr = lda, sc = 1
// reads an upper one's U = L^T).  Only that triangle is read or written.
// info: device int; a block does nothing when *info != 0 on entry, and sets
// *info = col0 + j + 1 when the pivot of its column j is not positive.
constexpr int kCholLeafMax = 128;
constexpr int kCholLeafDefault = 128;  // leaf order when the caller leaves nb at 0
hipError_t launch_potrf_leaf(int dtype, void* a, int64_t sr, int64_t sc, int b, int64_t col0,
                             int* info, hipStream_t s);
// info[0] := 0 (a kernel, not a memset, so it may sit in captured work).
hipError_t launch_info_clear(int* info, hipStream_t s);

// info[0] := 0 if every entry of the m x n matrix is finite, else `code`.
hipError_t launch_check_finite(int dtype, const void* b, int64_t m, int64_t n, int64_t ldb,
                               int* info, int code, hipStream_t s);

}  // namespace redsea
