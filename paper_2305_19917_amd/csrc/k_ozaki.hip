// Exact integer emulation of the FP64 residual product (Ozaki scheme II):
// splitting kernels, the modular INT8 products on v_mfma_i32_16x16x64_i8,
// and the Chinese-remainder reconstruction.  See ozaki.h for the method.
#include <hip/hip_runtime.h>

#include <cmath>
#include <climits>
#include <mutex>

#include "ozaki.h"
#include "tiles.h"

namespace redsea {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned __int128 u128;

constexpr int kSentinel = INT_MIN;  // exponent of a row / column holding Inf or NaN

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
int64_t ld_m(int64_t k) { return (k + 15) / 16 * 16; }  // bytes per plane row of M
int64_t ld_x(int64_t k) { return (k + 15) / 16 * 16; }  // bytes per plane column of X
int64_t ld_r(int64_t k) { return (k + 3) / 4 * 4; }     // bytes per plane column of the products

// Exponent e with 2^52 <= mx 2^e < 2^53 (0 for a zero maximum, the sentinel
// for a non-finite one).
__device__ __forceinline__ int scale_exp(double mx) {
    if (!(mx <= 1.7976931348623157e308)) return kSentinel;  // Inf or NaN
    if (mx == 0.0) return 0;
    int ex = 0;
    (void)frexp(mx, &ex);  // mx = f 2^ex, f in [0.5, 1)
    return 53 - ex;
}

// Symmetric residue in [-128, 127] of the integer-valued q (|q| <= 2^53)
// modulo p <= 256: t = floor(q / p) from a rounded reciprocal (off by at most
// one), q - t p exactly by one fused multiply-add, then the corrections.
__device__ __forceinline__ int sym_residue(double q, int p, double invp) {
    const double t = floor(q * invp);
    double r = fma(-t, (double)p, q);
    if (r < 0.0) r += p;
    if (r >= p) r -= p;
    int ri = (int)r;
    return ri >= 128 ? ri - p : ri;
}

// ---------------------------------------------------------------- M planes

// e[i] for row i of M (max |M(i, j)| over the stored triangle, unit diagonal
// as one).  Row i of M is a row of A (a_trans false: strided, 64 rows per
// workgroup, lanes on rows, the eight waves splitting the columns) or a
// column of A (a_trans: contiguous, one wave per row).
__device__ __forceinline__ bool m_stored(int64_t i, int64_t j, int uplo, bool a_trans) {
    const int64_t r = a_trans ? j : i, c = a_trans ? i : j;
    return uplo == 0 ? r >= c : r <= c;
}

__global__ __launch_bounds__(512) void m_rowexp_kernel(const double* __restrict__ a, int64_t lda,
                                                       int64_t k, int uplo, int a_trans, int unit,
                                                       int* __restrict__ e) {
    __shared__ double part[8][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double mx = 0.0;
    int64_t i;
    if (!a_trans) {
        i = (int64_t)blockIdx.x * 64 + lane;
        const int64_t per = (k + 7) / 8, ja = w * per, jb = ja + per < k ? ja + per : k;
        if (i < k)
            for (int64_t j = ja; j < jb; ++j) {
                if (!m_stored(i, j, uplo, false)) continue;
                const double v = (j == i && unit) ? 1.0 : fabs(a[i + j * lda]);
                mx = (v > mx || v != v) ? v : mx;
            }
        part[w][lane] = mx;
        __syncthreads();
        if (w == 0 && i < k) {
#pragma unroll
            for (int q = 1; q < 8; ++q) {
                const double v = part[q][lane];
                mx = (v > mx || v != v) ? v : mx;
            }
            e[i] = scale_exp(mx);
        }
    } else {
        i = (int64_t)blockIdx.x * 8 + w;
        if (i >= k) return;  // uniform over the wave
        for (int64_t j = lane; j < k; j += 64) {
            if (!m_stored(i, j, uplo, true)) continue;
            const double v = (j == i && unit) ? 1.0 : fabs(a[j + i * lda]);
            mx = (v > mx || v != v) ? v : mx;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double v = __shfl_xor(mx, o);
            mx = (v > mx || v != v) ? v : mx;
        }
        if (lane == 0) e[i] = scale_exp(mx);
    }
}

// Plane l, row i, byte j := symmetric residue of rint(2^e_i M(i, j)) modulo
// p_l (zero outside the stored triangle and in the padding columns j >= k).
// 64 x 64 tiles of M pass through LDS so that A is read along its contiguous
// index and the planes are written along j.
__global__ __launch_bounds__(256) void m_split_kernel(const double* __restrict__ a, int64_t lda,
                                                      int64_t k, int uplo, int a_trans, int unit,
                                                      const int* __restrict__ e,
                                                      signed char* __restrict__ planes,
                                                      int64_t ldm, int64_t plane_bytes,
                                                      OzakiConst C) {
    __shared__ double t[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    auto m_at = [&](int64_t i, int64_t j) -> double {
        if (i >= k || j >= k || !m_stored(i, j, uplo, a_trans)) return 0.0;
        if (i == j && unit) return 1.0;
        return a_trans ? a[j + i * lda] : a[i + j * lda];
    };
    for (int q = ty; q < 64; q += 4) {
        if (!a_trans) t[tx][q] = m_at(i0 + tx, j0 + q);
        else t[q][tx] = m_at(i0 + q, j0 + tx);
    }
    __syncthreads();
    for (int q = ty; q < 64; q += 4) {
        const int64_t i = i0 + q, j = j0 + tx;
        if (i >= k || j >= ldm) continue;
        const int ei = e[i];
        const double v = ei == kSentinel ? 0.0 : rint(ldexp(t[q][tx], ei));
#pragma unroll
        for (int l = 0; l < kOzN; ++l)
            planes[l * plane_bytes + i * ldm + j] = (signed char)sym_residue(v, C.p[l], C.invpd[l]);
    }
}

// ---------------------------------------------------------------- X planes

// One workgroup per column j of X: f[j] from the column maximum, then plane
// l, column j, byte kk := residue of rint(2^f_j X(kk, j)) (zero for kk >= k).
__global__ __launch_bounds__(256) void x_split_kernel(const double* __restrict__ x, int64_t ldx,
                                                      int64_t k, int rhs_trans,
                                                      int* __restrict__ f,
                                                      signed char* __restrict__ planes,
                                                      int64_t ldp, int64_t plane_bytes,
                                                      OzakiConst C) {
    __shared__ double red[256];
    const int64_t j = blockIdx.x;
    auto x_at = [&](int64_t kk) -> double { return rhs_trans ? x[j + kk * ldx] : x[kk + j * ldx]; };
    double mx = 0.0;
    for (int64_t kk = threadIdx.x; kk < k; kk += 256) {
        const double v = fabs(x_at(kk));
        mx = (v > mx || v != v) ? v : mx;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    const int fj = scale_exp(red[0]);
    if (threadIdx.x == 0) f[j] = fj;
    for (int64_t kk = threadIdx.x; kk < ldp; kk += 256) {
        const double v = (kk < k && fj != kSentinel) ? rint(ldexp(x_at(kk), fj)) : 0.0;
#pragma unroll
        for (int l = 0; l < kOzN; ++l)
            planes[l * plane_bytes + j * ldp + kk] = (signed char)sym_residue(v, C.p[l], C.invpd[l]);
    }
}

// ---------------------------------------------------------------- products

// For modulus l = blockIdx.y: Q_l(i, j) := (sum_kk Mres_l(i, kk) Xres_l(kk, j))
// mod p_l in [0, p_l), over the rows of the triangle (tri 1: kk <= i, 2:
// kk >= i; the planes are zero outside it, so only whole k-stages outside are
// skipped).  Both operands are k-contiguous int8, brought straight into LDS
// by 16-byte buffer loads (a chunk past the rows, columns or K reads zero),
// two stages of 64 k, one barrier per stage; chunk q of row (column) m sits
// at slot 4m + (q ^ (m/4 % 4)), so a fragment read (16 rows, one chunk) hits
// 16 different 16-byte bank groups.  The INT32 sums are exact (|sum| <= k
// 128^2 < 2^31).
template <int BM, int BN, int WM, int WN>
struct I8Cfg {
    static constexpr int NW = WM * WN, NT = 64 * NW, SM = BM / WM, SN = BN / WN;
    static constexpr int FM = SM / 16, FN = SN / 16;
    static constexpr int A_LOADS = BM * 4 / 64, X_LOADS = BN * 4 / 64;
    static constexpr int A_BYTES = BM * 64, X_BYTES = BN * 64, STAGE = A_BYTES + X_BYTES;
    static_assert(A_LOADS % NW == 0 && X_LOADS % NW == 0, "loads per wave");
};

typedef __attribute__((address_space(3))) void* lds_ptr_i8_t;
constexpr unsigned kI8Oob = 0x7FFFFFF0u;
constexpr int kI8Bk = 64;

template <typename D>
__device__ __forceinline__ void i8_stage(const signed char* pa, int64_t lda, int64_t mlim,
                                         const signed char* px, int64_t ldx, int64_t nlim,
                                         int64_t klim, char* st, int wave, int lane) {
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc((void*)pa, 0, (int)kI8Oob, 0x00020000);
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc((void*)px, 0, (int)kI8Oob, 0x00020000);
#pragma unroll
    for (int u = 0; u < D::A_LOADS / D::NW; ++u) {
        const int q = u * D::NW + wave;
        const int slot = 64 * q + lane, m = slot >> 2, kq = (slot & 3) ^ ((m >> 2) & 3);
        const unsigned voff = (m < mlim && 16 * kq < klim) ? (unsigned)(16 * kq + m * lda) : kI8Oob;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr_i8_t)(st + q * 1024), 16, voff, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < D::X_LOADS / D::NW; ++u) {
        const int q = u * D::NW + wave;
        const int slot = 64 * q + lane, n = slot >> 2, kq = (slot & 3) ^ ((n >> 2) & 3);
        const unsigned voff = (n < nlim && 16 * kq < klim) ? (unsigned)(16 * kq + n * ldx) : kI8Oob;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_ptr_i8_t)(st + D::A_BYTES + q * 1024), 16,
                                                 voff, 0, 0, 0);
    }
}

template <int BM, int BN, int WM, int WN, int TRI>
__global__ __launch_bounds__(64 * WM * WN, 2) void ozaki_gemm_kernel(
    const signed char* __restrict__ mplanes, int64_t ldm, int64_t m_plane,
    const signed char* __restrict__ xplanes, int64_t ldxp, int64_t x_plane,
    unsigned char* __restrict__ qplanes, int64_t ldq, int64_t q_plane, int64_t k, int64_t nrhs,
    OzakiConst C) {
    typedef I8Cfg<BM, BN, WM, WN> D;
    __shared__ __attribute__((aligned(1024))) char smem[2 * D::STAGE];
    const int l = blockIdx.y;
    const int p = C.p[l];
    const float invp = C.invp[l];
    const int64_t tiles_m = (k + BM - 1) / BM, tiles_n = (nrhs + BN - 1) / BN;
    // heaviest row tiles first, consecutive workgroups along a row
    const int64_t rr = (int64_t)blockIdx.x / tiles_n, tn = (int64_t)blockIdx.x % tiles_n;
    const int64_t tm = TRI == 1 ? tiles_m - 1 - rr : rr;
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int lane = threadIdx.x & 63, gq = lane >> 4, cc = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WM, wn = wave / WM;
    const signed char* A = mplanes + l * m_plane;
    const signed char* X = xplanes + l * x_plane;
    int oa[D::FM], ox[D::FN];
#pragma unroll
    for (int i = 0; i < D::FM; ++i) {
        const int m = wm * D::SM + 16 * i + cc;
        oa[i] = (4 * m + (gq ^ ((m >> 2) & 3))) * 16;
    }
#pragma unroll
    for (int j = 0; j < D::FN; ++j) {
        const int n = wn * D::SN + 16 * j + cc;
        ox[j] = D::A_BYTES + (4 * n + (gq ^ ((n >> 2) & 3))) * 16;
    }
    v4i acc[D::FM][D::FN];
#pragma unroll
    for (int i = 0; i < D::FM; ++i)
#pragma unroll
        for (int j = 0; j < D::FN; ++j) acc[i][j] = v4i{0, 0, 0, 0};
    int64_t kb = 0, ke = (k + kI8Bk - 1) / kI8Bk;
    if (TRI == 1) {
        const int64_t last = m0 + BM < k ? m0 + BM : k;
        ke = (last + kI8Bk - 1) / kI8Bk;
    } else {
        kb = m0 / kI8Bk;
    }
    const int64_t mlim = k - m0, nlim = nrhs - n0;
    auto stage = [&](int64_t kt, char* st) {
        const int64_t k0 = kt * kI8Bk;
        i8_stage<D>(A + k0 + m0 * ldm, ldm, mlim, X + k0 + n0 * ldxp, ldxp, nlim, k - k0, st, wave,
                    lane);
    };
    if (kb < ke) stage(kb, smem + (kb & 1) * D::STAGE);
    __syncthreads();
    for (int64_t kt = kb; kt < ke; ++kt) {
        const char* st = smem + (kt & 1) * D::STAGE;
        if (kt + 1 < ke) stage(kt + 1, smem + ((kt + 1) & 1) * D::STAGE);
        v4i fa[D::FM], fx[D::FN];
#pragma unroll
        for (int i = 0; i < D::FM; ++i) fa[i] = *(const v4i*)(st + oa[i]);
#pragma unroll
        for (int j = 0; j < D::FN; ++j) fx[j] = *(const v4i*)(st + ox[j]);
#pragma unroll
        for (int i = 0; i < D::FM; ++i)
#pragma unroll
            for (int j = 0; j < D::FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[i], fx[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // residues in [0, p): the float quotient of |sum| < 2^28 is off by at most one
    unsigned char* Q = qplanes + l * q_plane;
#pragma unroll
    for (int i = 0; i < D::FM; ++i)
#pragma unroll
        for (int j = 0; j < D::FN; ++j) {
            const int64_t gi = m0 + wm * D::SM + 16 * i + 4 * gq;
            const int64_t gj = n0 + wn * D::SN + 16 * j + cc;
            if (gj >= nrhs) continue;
            unsigned packed = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int v = acc[i][j][r];
                int t = (int)floorf((float)v * invp);
                int res = v - t * p;
                if (res < 0) res += p;
                if (res >= p) res -= p;
                packed |= (unsigned)res << (8 * r);
            }
            unsigned char* dst = Q + gi + gj * ldq;
            if (gi + 3 < k) {
                *(unsigned*)dst = packed;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (gi + r < k) dst[r] = (unsigned char)(packed >> (8 * r));
            }
        }
}

// ---------------------------------------------------------------- reconstruction

// R(i, j) := beta C0(i, j) + gamma 2^(-e_i - f_j) Y(i, j), where Y is the integer
// in (-P/2, P/2] congruent to the product residues: S = sum_l w_l q_l exactly
// in five 32-bit limbs, S - floor(S / P) P (the quotient from FP64, then
// corrected), symmetric representative, rounded to FP64.
__device__ __forceinline__ bool geq4(const uint32_t a[4], const uint32_t b[4]) {
    for (int q = 3; q >= 0; --q)
        if (a[q] != b[q]) return a[q] > b[q];
    return true;
}

__device__ __forceinline__ void sub4(uint32_t a[4], const uint32_t b[4]) {
    uint64_t borrow = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t d = (uint64_t)a[q] - b[q] - borrow;
        a[q] = (uint32_t)d;
        borrow = (d >> 63) & 1;
    }
}

__global__ __launch_bounds__(256) void crt_kernel(const unsigned char* __restrict__ qplanes,
                                                  int64_t ldq, int64_t q_plane,
                                                  const int* __restrict__ e,
                                                  const int* __restrict__ f, int64_t k,
                                                  int64_t nrhs, int rhs_trans, double beta,
                                                  double gamma, const double* b0, int64_t ldb0,
                                                  double* r, int64_t ldr, OzakiConst C) {
    const int64_t total = k * nrhs;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx % k, j = idx / k;
        uint64_t acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int l = 0; l < kOzN; ++l) {
            const uint64_t q = qplanes[l * q_plane + i + j * ldq];
#pragma unroll
            for (int w = 0; w < 4; ++w) acc[w] += (uint64_t)C.w[l][w] * q;
        }
        uint32_t s[5];
        uint64_t carry = 0;
#pragma unroll
        for (int w = 0; w < 5; ++w) {
            const uint64_t v = acc[w] + carry;
            s[w] = (uint32_t)v;
            carry = v >> 32;
        }
        // S < 16 * 256 * P < 2^138: subtract t P with t = floor(S / P) - 1 or so
        const double sd = ldexp((double)s[4], 128) + ldexp((double)s[3], 96) +
                          ldexp((double)s[2], 64) + ldexp((double)s[1], 32) + (double)s[0];
        double td = floor(sd / C.Pd) - 1.0;
        if (td < 0.0) td = 0.0;
        const uint64_t t = (uint64_t)td;  // below 2^13
        uint64_t borrow = 0, c2 = 0;
#pragma unroll
        for (int w = 0; w < 5; ++w) {
            const uint64_t tp = (w < 4 ? t * C.P[w] : 0) + c2;  // limb w of t P
            c2 = tp >> 32;
            const uint64_t d = (uint64_t)s[w] - (uint32_t)tp - borrow;
            s[w] = (uint32_t)d;
            borrow = (d >> 63) & 1;
        }
        // now 0 <= S < 3 P (t was at most one below the quotient, plus rounding)
        uint32_t m4[4] = {s[0], s[1], s[2], s[3]};
        if (s[4] != 0 || geq4(m4, C.P)) sub4(m4, C.P);
        if (geq4(m4, C.P)) sub4(m4, C.P);
        bool neg = false;
        if (!geq4(C.halfP, m4)) {  // m4 > P/2: the representative is m4 - P
            uint32_t pm[4] = {C.P[0], C.P[1], C.P[2], C.P[3]};
            sub4(pm, m4);
            m4[0] = pm[0];
            m4[1] = pm[1];
            m4[2] = pm[2];
            m4[3] = pm[3];
            neg = true;
        }
        const uint64_t hi = ((uint64_t)m4[3] << 32) | m4[2], lo = ((uint64_t)m4[1] << 32) | m4[0];
        double y = ldexp((double)hi, 64) + (double)lo;
        if (neg) y = -y;
        const int ei = e[i], fj = f[j];
        const double bv = beta == 0.0 ? 0.0 : beta * (rhs_trans ? b0[j + i * ldb0] : b0[i + j * ldb0]);
        double out;
        if (ei == kSentinel || fj == kSentinel) out = __builtin_nan("");
        else out = bv + gamma * ldexp(y, -(ei + fj));
        if (rhs_trans) r[j + i * ldr] = out;
        else r[i + j * ldr] = out;
    }
}

OzakiConst make_const() {
    OzakiConst c{};
    // pairwise coprime moduli <= 256, largest first
    int chosen = 0;
    for (int cand = 256; cand > 1 && chosen < kOzN; --cand) {
        bool ok = true;
        for (int q = 0; q < chosen && ok; ++q) {
            int a = cand, b = c.p[q];
            while (b) {
                const int t = a % b;
                a = b;
                b = t;
            }
            ok = a == 1;
        }
        if (ok) c.p[chosen++] = cand;
    }
    u128 P = 1;
    for (int l = 0; l < kOzN; ++l) P *= (u128)c.p[l];
    for (int l = 0; l < kOzN; ++l) {
        const u128 Ml = P / (u128)c.p[l];
        const int mr = (int)(Ml % (u128)c.p[l]);
        int inv = 0;
        for (int t = 1; t < c.p[l]; ++t)
            if ((mr * t) % c.p[l] == 1) { inv = t; break; }
        const u128 w = (Ml * (u128)inv) % P;  // Ml < 2^118, inv < 256: no overflow
        for (int q = 0; q < 4; ++q) c.w[l][q] = (uint32_t)(w >> (32 * q));
        c.invp[l] = 1.0f / (float)c.p[l];
        c.invpd[l] = 1.0 / (double)c.p[l];
    }
    for (int q = 0; q < 4; ++q) {
        c.P[q] = (uint32_t)(P >> (32 * q));
        c.halfP[q] = (uint32_t)((P >> 1) >> (32 * q));
    }
    c.Pd = std::ldexp((double)(uint64_t)(P >> 64), 64) + (double)(uint64_t)P;
    return c;
}

unsigned grid_of(int64_t total) {
    int64_t b = (total + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

const OzakiConst& ozaki_const() {
    static OzakiConst c = make_const();
    return c;
}

size_t ozaki_m_bytes(int64_t k) {
    return al256((size_t)k * 4) + kOzN * al256((size_t)k * ld_m(k));
}

size_t ozaki_x_bytes(int64_t k, int64_t nrhs) {
    return al256((size_t)nrhs * 4) + kOzN * al256((size_t)nrhs * ld_x(k)) +
           kOzN * al256((size_t)nrhs * ld_r(k));
}

hipError_t ozaki_split_m(const double* a, int64_t lda, int64_t k, int uplo, bool a_trans,
                         bool unit, void* ws, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    int* e = (int*)ws;
    signed char* planes = (signed char*)ws + al256((size_t)k * 4);
    const int64_t ldm = ld_m(k), pb = (int64_t)al256((size_t)k * ldm);
    if (!a_trans)
        hipLaunchKernelGGL(m_rowexp_kernel, dim3((unsigned)((k + 63) / 64)), dim3(512), 0, s, a,
                           lda, k, uplo, 0, unit ? 1 : 0, e);
    else
        hipLaunchKernelGGL(m_rowexp_kernel, dim3((unsigned)((k + 7) / 8)), dim3(512), 0, s, a, lda,
                           k, uplo, 1, unit ? 1 : 0, e);
    dim3 grid((unsigned)((ldm + 63) / 64), (unsigned)((k + 63) / 64));
    hipLaunchKernelGGL(m_split_kernel, grid, dim3(256), 0, s, a, lda, k, uplo, a_trans ? 1 : 0,
                       unit ? 1 : 0, e, planes, ldm, pb, ozaki_const());
    return hipGetLastError();
}

hipError_t ozaki_product(const void* mws, int tri, int64_t k, int64_t nrhs, bool rhs_trans,
                         double beta, double gamma, const double* x, int64_t ldx,
                         const double* b0, int64_t ldb0, double* r, int64_t ldr, void* xws,
                         hipStream_t s) {
    if (k <= 0 || nrhs <= 0) return hipSuccess;
    if (tri != 1 && tri != 2) return hipErrorInvalidValue;
    const OzakiConst& C = ozaki_const();
    const int* e = (const int*)mws;
    const signed char* mplanes = (const signed char*)mws + al256((size_t)k * 4);
    const int64_t ldm = ld_m(k), mpb = (int64_t)al256((size_t)k * ldm);
    int* f = (int*)xws;
    signed char* xplanes = (signed char*)xws + al256((size_t)nrhs * 4);
    const int64_t ldxp = ld_x(k), xpb = (int64_t)al256((size_t)nrhs * ldxp);
    unsigned char* qplanes = (unsigned char*)(xplanes + kOzN * xpb);
    const int64_t ldq = ld_r(k), qpb = (int64_t)al256((size_t)nrhs * ldq);
    hipLaunchKernelGGL(x_split_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, x, ldx, k,
                       rhs_trans ? 1 : 0, f, xplanes, ldxp, xpb, C);
    constexpr int BM = 256, BN = 128;
    const int64_t tiles = ((k + BM - 1) / BM) * ((nrhs + BN - 1) / BN);
    dim3 grid((unsigned)tiles, kOzN);
    if (tri == 1)
        hipLaunchKernelGGL((ozaki_gemm_kernel<BM, BN, 4, 2, 1>), grid, dim3(512), 0, s, mplanes,
                           ldm, mpb, xplanes, ldxp, xpb, qplanes, ldq, qpb, k, nrhs, C);
    else
        hipLaunchKernelGGL((ozaki_gemm_kernel<BM, BN, 4, 2, 2>), grid, dim3(512), 0, s, mplanes,
                           ldm, mpb, xplanes, ldxp, xpb, qplanes, ldq, qpb, k, nrhs, C);
    hipLaunchKernelGGL(crt_kernel, dim3(grid_of(k * nrhs)), dim3(256), 0, s, qplanes, ldq, qpb, e,
                       f, k, nrhs, rhs_trans ? 1 : 0, beta, gamma, b0, ldb0, r, ldr, C);
    return hipGetLastError();
}

}  // namespace redsea
