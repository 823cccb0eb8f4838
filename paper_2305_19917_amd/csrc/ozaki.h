// FP64-accurate residual by exact integer emulation (Ozaki scheme II:
// Ozaki, Uchino, Imamura, "Ozaki Scheme II: A GEMM-oriented emulation of
// floating-point matrix multiplication using an integer modular technique").
//
// For R = alpha B0 - M X with M a k x k triangle:
//   1. rows of M and columns of X are scaled by powers of two and rounded to
//      integers of at most 53 bits: M'_i = rint(2^e_i M_i), X'_j = rint(2^f_j X_j);
//   2. M' X' is an integer below k 2^106 in magnitude, so it is determined by
//      its residues modulo 16 pairwise coprime moduli p_l <= 256 whose
//      product P exceeds 2^125;
//   3. for each modulus the residues (symmetric, in [-128, 127]) of M' and X'
//      are multiplied exactly on the INT8 matrix cores (INT32 accumulation;
//      k 128^2 < 2^31) and the result reduced modulo p_l;
//   4. the Chinese remainder theorem rebuilds M' X' exactly in multi-word
//      integer arithmetic, and Y = 2^(-e_i - f_j) M' X' is rounded to FP64.
// The only approximation is step 1 (each element rounded to 53 bits relative
// to its row or column maximum), so Y is as accurate as an FP64 product.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace redsea {

constexpr int kOzN = 16;  // moduli

// Moduli and Chinese-remainder weights w_l = (P/p_l) * ((P/p_l)^-1 mod p_l)
// mod P, as little-endian 32-bit limbs; passed to kernels by value.
struct OzakiConst {
    int p[kOzN];
    float invp[kOzN];   // 1 / p_l rounded to FP32 (product residues)
    double invpd[kOzN]; // 1 / p_l rounded to FP64 (53-bit integer residues)
    uint32_t w[kOzN][4];
    uint32_t P[4];
    uint32_t halfP[4];  // floor(P / 2)
    double Pd;          // P rounded to FP64
};
const OzakiConst& ozaki_const();

// Bytes of the workspace planes for an order-k triangle and nrhs columns.
size_t ozaki_m_bytes(int64_t k);        // residue planes of M (+ row exponents)
size_t ozaki_x_bytes(int64_t k, int64_t nrhs);  // planes of X and of the products (+ exponents)

// Residue planes of M = op(A) (storage coordinates, as in launch_residual):
// M(i, j) = a[i + j*lda] (a_trans false) or a[j + i*lda], restricted to the
// stored triangle of A (uplo), unit diagonal as one.  Writes, into `ws`
// (ozaki_m_bytes), the row exponents and 16 int8 planes by rows.
hipError_t ozaki_split_m(const double* a, int64_t lda, int64_t k, int uplo, bool a_trans,
                         bool unit, void* ws, hipStream_t s);

// R := beta C0 + gamma M X with M from ozaki_split_m (lower: tri = 1, upper:
// 2; beta == 0: C0 is not read).  X(k, j) = x[k + j*ldx] (rhs_trans false) or
// x[j + k*ldx]; C0 and R the same way with their own leading dimensions (R
// may be C0).  xws: ozaki_x_bytes.
hipError_t ozaki_product(const void* mws, int tri, int64_t k, int64_t nrhs, bool rhs_trans,
                         double beta, double gamma, const double* x, int64_t ldx,
                         const double* c0, int64_t ldc0, double* r, int64_t ldr, void* xws,
                         hipStream_t s);

}  // namespace redsea
