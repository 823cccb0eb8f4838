// Trailing-update product C -= A X on MFMA matrix cores, gfx950.
//
// This is the "gemm" task the paper offloads to the accelerator (Sec. V-A:
// with many right-hand sides the update of stage 2 of Sec. IV becomes a
// matrix-matrix product; the grey rectangles of Fig. 2-4).  A workgroup owns a
// BM x BN tile of C, split over WM x WN waves; each wave keeps its
// (BM/WM) x (BN/WN) sub-tile as 16 x 16 MFMA accumulators.  K advances in
// steps of BK through a double-buffered LDS stage: the next stage's global
// loads are in flight while the current stage feeds the matrix cores.  The
// tile configuration is a template parameter so the tuner can pick one per
// shape.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "tiles.h"

namespace redsea {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Per-type MFMA 16x16x4 operations.  For both types lane l supplies
// A[l % 16][l / 16] and X[l / 16][l % 16]; the 16 x 16 result lives in four
// registers per lane whose row index differs between the two instructions.
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row of register r for lane l (column is l % 16)
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Tile configuration: BM x BN tile, BK k-stage, WM x WN waves, MINB
// workgroups per CU requested from the register allocator.
template <int BM_, int BN_, int BK_, int WM_, int WN_, int MINB_>
struct Cfg {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, MINB = MINB_;
    static constexpr int NT = 64 * WM * WN;
    static constexpr int FM = BM / WM / 16, FN = BN / WN / 16;  // fragments per wave
    static constexpr int LA = BM * BK / NT, LX = BN * BK / NT;  // loads per thread
    static constexpr int PAD = 2;
    static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile");
    static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "loads");
    static_assert(BK % 4 == 0, "k");
};

template <typename T, typename C>
struct Smem {
    T a[2][C::BK][C::BM + C::PAD];
    T x[2][C::BK][C::BN + C::PAD];
};

template <typename T, typename C, bool AT, bool RT, int TRI = 0, bool UNIT = false>
__device__ __forceinline__ void load_stage(const GemmArgs& g, int64_t m0, int64_t n0, int64_t k0,
                                           int tid, T (&ra)[C::LA], T (&rx)[C::LX]) {
    const T* a = (const T*)g.a;
    const T* x = (const T*)g.x;
#pragma unroll
    for (int p = 0; p < C::LA; ++p) {
        const int idx = p * C::NT + tid;
        int kk, mm;
        if (!AT) { kk = idx / C::BM; mm = idx % C::BM; }  // column of A: BM contiguous rows
        else { mm = idx / C::BK; kk = idx % C::BK; }      // row of A^T storage: BK contiguous k
        const int64_t gi = m0 + mm, gk = k0 + kk;
        T v = T(0);
        const bool inside = TRI == 0 || TRI == 3 || (TRI == 1 ? gk <= gi : gk >= gi);
        if (gi < g.M && gk < g.K && inside) {
            if ((TRI == 1 || TRI == 2) && UNIT && gi == gk) v = T(1);
            else v = AT ? a[gk + gi * g.lda] : a[gi + gk * g.lda];
        }
        ra[p] = v;
    }
#pragma unroll
    for (int p = 0; p < C::LX; ++p) {
        const int idx = p * C::NT + tid;
        int kk, jj;
        if (!RT) { jj = idx / C::BK; kk = idx % C::BK; }  // column of X: BK contiguous k
        else { kk = idx / C::BN; jj = idx % C::BN; }      // row of X^T storage: BN contiguous j
        const int64_t gj = n0 + jj, gk = k0 + kk;
        T v = T(0);
        if (gj < g.N && gk < g.K) v = RT ? x[gj + gk * g.ldx] : x[gk + gj * g.ldx];
        rx[p] = v;
    }
}

template <typename T, typename C, bool AT, bool RT>
__device__ __forceinline__ void store_stage(Smem<T, C>& sm, int buf, int tid, const T (&ra)[C::LA],
                                            const T (&rx)[C::LX]) {
#pragma unroll
    for (int p = 0; p < C::LA; ++p) {
        const int idx = p * C::NT + tid;
        int kk, mm;
        if (!AT) { kk = idx / C::BM; mm = idx % C::BM; }
        else { mm = idx / C::BK; kk = idx % C::BK; }
        sm.a[buf][kk][mm] = ra[p];
    }
#pragma unroll
    for (int p = 0; p < C::LX; ++p) {
        const int idx = p * C::NT + tid;
        int kk, jj;
        if (!RT) { jj = idx / C::BK; kk = idx % C::BK; }
        else { kk = idx / C::BN; jj = idx % C::BN; }
        sm.x[buf][kk][jj] = rx[p];
    }
}

// TRI = 3: C -= A X on the entries with i <= j only (C square); the other
// modes as in gemm_dma_kernel below.
template <typename T, typename C, bool AT, bool RT, int TRI = 0, bool UNIT = false>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int64_t m0, int64_t n0,
                                          Smem<T, C>& sm, T beta = T(1), T gamma = T(-1)) {
    typedef typename Mfma<T>::acc_t acc_t;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % C::WM, wn = wave / C::WM;
    constexpr int SM = C::BM / C::WM, SN = C::BN / C::WN;  // wave sub-tile

    acc_t acc[C::FM][C::FN];
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    T ra[C::LA], rx[C::LX];
    // k range: all of K, or for a triangular M only the stages that meet the
    // triangle in rows [m0, m0 + BM)
    int64_t kb = 0, ke = (g.K + C::BK - 1) / C::BK;
    if (TRI == 1) {
        const int64_t last = m0 + C::BM < g.K ? m0 + C::BM : g.K;
        ke = (last + C::BK - 1) / C::BK;
    } else if (TRI == 2) {
        kb = m0 / C::BK;
    }
    load_stage<T, C, AT, RT, TRI, UNIT>(g, m0, n0, kb * C::BK, tid, ra, rx);
    store_stage<T, C, AT, RT>(sm, 0, tid, ra, rx);
    __syncthreads();
    for (int64_t kt = kb; kt < ke; ++kt) {
        const int buf = (int)((kt - kb) & 1);
        const bool more = kt + 1 < ke;
        if (more) load_stage<T, C, AT, RT, TRI, UNIT>(g, m0, n0, (kt + 1) * C::BK, tid, ra, rx);
#pragma unroll
        for (int ks = 0; ks < C::BK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            T fa[C::FM], fx[C::FN];
#pragma unroll
            for (int i = 0; i < C::FM; ++i) fa[i] = sm.a[buf][kr][wm * SM + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < C::FN; ++j) fx[j] = sm.x[buf][kr][wn * SN + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < C::FM; ++i)
#pragma unroll
                for (int j = 0; j < C::FN; ++j) acc[i][j] = Mfma<T>::mma(fa[i], fx[j], acc[i][j]);
        }
        if (more) store_stage<T, C, AT, RT>(sm, buf ^ 1, tid, ra, rx);
        __syncthreads();
    }

    T* c = (T*)g.c;
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = m0 + wm * SM + i * 16 + Mfma<T>::row(lane, r);
                const int64_t gj = n0 + wn * SN + j * 16 + (lane & 15);
                if (gi < g.M && gj < g.N && (TRI != 3 || gi <= gj)) {
                    T* p = RT ? c + gj + gi * g.ldc : c + gi + gj * g.ldc;
                    if (TRI == 0 || TRI == 3) *p = *p - acc[i][j][r];
                    else *p = (beta == T(0) ? T(0) : beta * *p) + gamma * acc[i][j][r];
                }
            }
}

// Tile (tm, tn) of launch index b over the tiles with tm <= tn, column by
// column: b = tn (tn + 1) / 2 + tm.  As in tile_coords, the launch index is
// first remapped so that each of the eight XCDs (launch indices are dealt to
// them round-robin) takes one contiguous run of b: a few consecutive tile
// columns, whose tiles share row and column panels in that XCD's L2.
__device__ __forceinline__ void upper_tile_coords(int64_t& tm, int64_t& tn) {
    constexpr int64_t kXcd = 8;
    const int64_t nwg = (int64_t)gridDim.x;
    int64_t b = blockIdx.x;
    if (nwg % kXcd == 0) b = (b % kXcd) * (nwg / kXcd) + b / kXcd;
    int64_t t = (int64_t)((__builtin_sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (t > 0 && t * (t + 1) / 2 > b) --t;
    while ((t + 1) * (t + 2) / 2 <= b) ++t;
    tn = t;
    tm = b - t * (t + 1) / 2;
}

template <typename T, typename C, bool AT, bool RT>
__global__ __launch_bounds__(C::NT, C::MINB) void gemm_kernel(GemmArgs g) {
    __shared__ Smem<T, C> sm;
    const int64_t tiles_m = (g.M + C::BM - 1) / C::BM, tiles_n = (g.N + C::BN - 1) / C::BN;
    int64_t tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    gemm_tile<T, C, AT, RT>(g, tm * C::BM, tn * C::BN, sm);
}

template <typename T, typename C, bool AT, bool RT>
__global__ __launch_bounds__(C::NT, C::MINB) void gemm_group_kernel(GemmGroup grp,
                                                                    int64_t tiles_m_max) {
    __shared__ Smem<T, C> sm;
    const GemmArgs& g = grp.g[blockIdx.y];
    const int64_t tm = blockIdx.x % tiles_m_max, tn = blockIdx.x / tiles_m_max;
    if (tm * C::BM >= g.M || tn * C::BN >= g.N) return;  // uniform over the workgroup
    gemm_tile<T, C, AT, RT>(g, tm * C::BM, tn * C::BN, sm);
}

// Short-K product (the small updates near the leaves of the recursion).  For
// K of a few hundred the double-buffered pipeline never reaches steady state
// and the read of C at the end adds a second memory latency.  This kernel
// reads its C tile first, stages K in chunks of KC through one LDS buffer and
// keeps two workgroups per CU so one computes while the other loads.
template <typename T, int BM, int BN, int KC, bool AT, bool RT>
__global__ __launch_bounds__(256, 2) void gemm_shortk_kernel(GemmArgs g) {
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr int WM = 2, WN = 2, SM = BM / WM, SN = BN / WN, FM = SM / 16, FN = SN / 16;
    constexpr int NT = 256, LA = BM * KC / NT, LX = BN * KC / NT, PAD = 2;
    __shared__ T As[KC][BM + PAD];
    __shared__ T Xs[KC][BN + PAD];
    const int64_t tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
    int64_t tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    T* c = (T*)g.c;
    const T* a = (const T*)g.a;
    const T* x = (const T*)g.x;

    T cv[FM][FN][4];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = m0 + wm * SM + i * 16 + Mfma<T>::row(lane, r);
                const int64_t gj = n0 + wn * SN + j * 16 + (lane & 15);
                cv[i][j][r] = (gi < g.M && gj < g.N) ? (RT ? c[gj + gi * g.ldc] : c[gi + gj * g.ldc])
                                                     : T(0);
            }
    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    for (int64_t k0 = 0; k0 < g.K; k0 += KC) {
        T ra[LA], rx[LX];
#pragma unroll
        for (int p = 0; p < LA; ++p) {
            const int idx = p * NT + tid;
            int kk, mm;
            if (!AT) { kk = idx / BM; mm = idx % BM; }
            else { mm = idx / KC; kk = idx % KC; }
            const int64_t gi = m0 + mm, gk = k0 + kk;
            ra[p] = (gi < g.M && gk < g.K) ? (AT ? a[gk + gi * g.lda] : a[gi + gk * g.lda]) : T(0);
        }
#pragma unroll
        for (int p = 0; p < LX; ++p) {
            const int idx = p * NT + tid;
            int kk, jj;
            if (!RT) { jj = idx / KC; kk = idx % KC; }
            else { kk = idx / BN; jj = idx % BN; }
            const int64_t gj = n0 + jj, gk = k0 + kk;
            rx[p] = (gj < g.N && gk < g.K) ? (RT ? x[gj + gk * g.ldx] : x[gk + gj * g.ldx]) : T(0);
        }
        if (k0 > 0) __syncthreads();  // the previous chunk has been consumed
#pragma unroll
        for (int p = 0; p < LA; ++p) {
            const int idx = p * NT + tid;
            int kk, mm;
            if (!AT) { kk = idx / BM; mm = idx % BM; }
            else { mm = idx / KC; kk = idx % KC; }
            As[kk][mm] = ra[p];
        }
#pragma unroll
        for (int p = 0; p < LX; ++p) {
            const int idx = p * NT + tid;
            int kk, jj;
            if (!RT) { jj = idx / KC; kk = idx % KC; }
            else { kk = idx / BN; jj = idx % BN; }
            Xs[kk][jj] = rx[p];
        }
        __syncthreads();
        const int64_t krem = g.K - k0;
        const int ksteps = krem >= KC ? KC / 4 : (int)((krem + 3) / 4);
        for (int ks = 0; ks < ksteps; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            T fa[FM], fx[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) fa[i] = As[kr][wm * SM + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < FN; ++j) fx[j] = Xs[kr][wn * SN + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = Mfma<T>::mma(fa[i], fx[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = m0 + wm * SM + i * 16 + Mfma<T>::row(lane, r);
                const int64_t gj = n0 + wn * SN + j * 16 + (lane & 15);
                if (gi < g.M && gj < g.N) {
                    T* p = RT ? c + gj + gi * g.ldc : c + gi + gj * g.ldc;
                    *p = cv[i][j][r] - acc[i][j][r];
                }
            }
}

template <typename T, int BM, int BN, int KC, bool AT, bool RT>
hipError_t gemm_shortk_launch(const GemmArgs& g, hipStream_t s) {
    const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_shortk_kernel<T, BM, BN, KC, AT, RT>), dim3((unsigned)tiles),
                       dim3(256), 0, s, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 product with operands brought straight from memory into LDS.
//
// buffer_load_dwordx4 ... lds writes 16 bytes per lane to LDS at M0 + 16 *
// lane, without passing through registers, and a lane whose byte offset lies
// past the buffer's record count receives zeros.  That removes the register
// staging, the LDS store phase and the bounds branches of gemm_tile: per
// k-stage a wave issues a handful of such loads for the NEXT stage right after
// the barrier and then runs the current stage's MFMAs, and one barrier per
// stage (whose wait for outstanding loads is what makes the next stage
// visible) is the only synchronisation.  The MFMAs of a stage's last k-step
// run after the barrier, on fragments read before it, so the matrix pipe is
// still busy while the waves meet.
//
// Each 16-byte lane load is a pair of consecutive elements, so an operand is
// staged in one of three layouts, chosen by which index is contiguous in
// memory and by the tile width BW:
//  * w-major, BW >= 128 (pairs along the m or j index): one row of BW
//    elements per k, rows padded by 16 elements so rows k and k+1 fall on
//    opposite halves of the 64 banks;
//  * w-major, BW = 64: a 1 KB load holds rows k and k+2 (k = 4a + b, b < 2),
//    loads are 1152 bytes apart, so rows 4s + b and 4s + b + 1 again sit on
//    opposite bank halves and a fragment's offsets stay affine in (s, f);
//  * k-major (pairs along k): 1 KB loads of 8 columns x 16 k; within a load
//    the pair slot of column wl is XOR-swizzled so that the 32 lanes of one
//    half-wave fragment read (16 columns, one k pair) hit every bank once.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void* lds_ptr_t;
constexpr unsigned kDmaOob = 0x7FFFFFF0u;  // byte offset at the record count: reads zero
constexpr int kDmaBk = 16;

template <int BW, bool KMAJOR>
struct DmaOp {
    static constexpr bool NARROW = !KMAJOR && BW == 64;
    static constexpr int ROW = BW + 16;                          // padded w-major row, elements
    static constexpr int CHUNKS = BW * kDmaBk / 128;             // 1 KB loads per stage
    static constexpr int PER_ROW = BW / 128;                     // wide w-major: loads per k row
    static constexpr int BYTES =
        KMAJOR ? BW * kDmaBk * 8 : (NARROW ? CHUNKS * 1152 : kDmaBk * ROW * 8);
    static_assert(KMAJOR ? BW % 8 == 0 : (BW == 64 || BW % 128 == 0), "operand width");
    // swizzled pair slot of column wl of chunk c (k-major)
    static __device__ __forceinline__ int swz(int wl, int c) { return ((wl >> 1) << 1) ^ (c & 1); }
    // Issue the loads of chunk q of a stage.  p points at element (k0, w0) of
    // the operand, whose (k, w) element is p[w + k*ld] (w-major) or
    // p[k + w*ld] (k-major); wlim and klim are the in-range extents from there.
    static __device__ __forceinline__ void load(const double* p, int64_t ld, int64_t wlim,
                                                int64_t klim, char* lds, int q, int lane) {
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc((void*)p, 0, (int)kDmaOob, 0x00020000);
        unsigned voff;
        char* dst;
        if (KMAJOR) {
            const int wl = lane >> 3, kp = (lane & 7) ^ swz(wl, q);
            const int w = 8 * q + wl;
            voff = (w < wlim && 2 * kp < klim) ? (unsigned)((2 * kp + w * ld) * 8) : kDmaOob;
            dst = lds + q * 1024;
        } else if (NARROW) {
            const int k = 4 * (q >> 1) + (q & 1) + 2 * (lane >> 5);
            const int w = 2 * (lane & 31);
            voff = (w < wlim && k < klim) ? (unsigned)((w + k * ld) * 8) : kDmaOob;
            dst = lds + q * 1152;
        } else {
            const int k = q / PER_ROW, h = q % PER_ROW;
            const int w = h * 128 + 2 * lane;
            voff = (w < wlim && k < klim) ? (unsigned)((w + k * ld) * 8) : kDmaOob;
            dst = lds + k * ROW * 8 + h * 1024;
        }
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr_t)dst, 16, voff, 0, 0, 0);
    }
    // The same chunk in four 4-byte loads per lane (quarter u covers bytes
    // [256u, 256u + 256) of the chunk; lanes 2i and 2i+1 carry the two halves
    // of one element).  Each element is checked on its own, so no index has
    // to be even, and every access is 4-byte aligned whatever ld is.
    static __device__ __forceinline__ void load_dw(const double* p, int64_t ld, int64_t wlim,
                                                   int64_t klim, char* lds, int q, int lane) {
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc((void*)p, 0, (int)kDmaOob, 0x00020000);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int d = u * 32 + (lane >> 1), half = lane & 1;  // element d of the chunk
            int k, w;
            char* dst;
            if (KMAJOR) {
                const int t = d >> 1, wl = t >> 3, kp = (t & 7) ^ swz(wl, q);
                k = 2 * kp + (d & 1);
                w = 8 * q + wl;
                dst = lds + q * 1024 + u * 256;
            } else if (NARROW) {
                k = 4 * (q >> 1) + (q & 1) + 2 * (d >> 6);
                w = d & 63;
                dst = lds + q * 1152 + u * 256;
            } else {
                k = q / PER_ROW;
                w = (q % PER_ROW) * 128 + d;
                dst = lds + k * ROW * 8 + (q % PER_ROW) * 1024 + u * 256;
            }
            const int64_t e = KMAJOR ? k + w * ld : w + k * ld;
            const unsigned voff = (w < wlim && k < klim) ? (unsigned)(e * 8 + 4 * half) : kDmaOob;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr_t)dst, 4, voff, 0, 0, 0);
        }
    }
    // Element offset (doubles) of (k = 4*ks + lane/16, w = wb + 16*f + lane%16)
    // without the f term: the fragment f adds fstride() elements.
    static __device__ __forceinline__ int frag_off(int ks, int wb, int lane) {
        const int g = lane >> 4, cc = lane & 15;
        if (NARROW) return ((g & 1) + 2 * ks) * 144 + (g >> 1) * 64 + wb + cc;
        if (!KMAJOR) return (4 * ks + g) * ROW + wb + cc;
        const int wl = cc & 7, c = (wb >> 3) + (cc >> 3);
        const int kp = 2 * ks + (g >> 1);
        return c * 128 + (wl * 8 + (kp ^ swz(wl, c))) * 2 + (g & 1);
    }
    static constexpr int fstride() { return KMAJOR ? 256 : 16; }
};

template <int BM, int BN, int WM, int WN, int MINB, bool AT, bool RT>
struct DmaCfg {
    static constexpr int NW = WM * WN, NT = 64 * NW, SM = BM / WM, SN = BN / WN;
    static constexpr int FM = SM / 16, FN = SN / 16;
    typedef DmaOp<BM, AT> OA;   // A's contiguous index is m unless transposed
    typedef DmaOp<BN, !RT> OX;  // X's contiguous index is k unless transposed
    static constexpr int STAGE = OA::BYTES + OX::BYTES;
    static_assert(OA::CHUNKS % NW == 0 && OX::CHUNKS % NW == 0, "chunks per wave");
    static_assert(SM % 16 == 0 && SN % 16 == 0, "wave tile");
};

template <typename D, bool AT, bool RT, bool DW>
__device__ __forceinline__ void dma_stage(const GemmArgs& g, int64_t m0, int64_t n0, int64_t k0,
                                          char* st, int wave, int lane) {
    const double* a = (const double*)g.a;
    const double* x = (const double*)g.x;
    const double* pa = AT ? a + k0 + m0 * g.lda : a + m0 + k0 * g.lda;
    const double* px = RT ? x + n0 + k0 * g.ldx : x + k0 + n0 * g.ldx;
    const int64_t mlim = g.M - m0, nlim = g.N - n0, klim = g.K - k0;
#pragma unroll
    for (int i = 0; i < D::OA::CHUNKS / D::NW; ++i) {
        if (DW) D::OA::load_dw(pa, g.lda, mlim, klim, st, i * D::NW + wave, lane);
        else D::OA::load(pa, g.lda, mlim, klim, st, i * D::NW + wave, lane);
    }
#pragma unroll
    for (int i = 0; i < D::OX::CHUNKS / D::NW; ++i) {
        if (DW) D::OX::load_dw(px, g.ldx, nlim, klim, st + D::OA::BYTES, i * D::NW + wave, lane);
        else D::OX::load(px, g.ldx, nlim, klim, st + D::OA::BYTES, i * D::NW + wave, lane);
    }
}

// TRI = 0: C -= A X.  TRI = 3: the same on the entries with i <= j only (C
// square, equal square tiles; the grid covers the tiles that meet that
// triangle): with X = A^T stored as A, the symmetric update of one triangle
// of a Cholesky factorisation's trailing matrix.  TRI = 1 / 2: A is the
// lower / upper triangle of its
// storage (the other triangle is never used, whatever it holds; with UNIT the
// diagonal is taken as 1) and C := beta C + gamma A X (C not read when beta
// is 0): the triangular product, and with gamma = -1 the residual of a
// triangular solve.  Only the k-stages that meet the triangle in rows
// [m0, m0 + BM) are run, and in the stages that cross the diagonal the A
// fragments are masked after they are read from LDS.
// DW: operands loaded with 4-byte lane accesses (any shape, any leading
// dimension) instead of 16-byte ones (even shapes and leading dimensions).
template <int BM, int BN, int WM, int WN, int MINB, bool AT, bool RT, int TRI = 0, bool UNIT = false,
          bool DW = false>
__global__ __launch_bounds__(64 * WM * WN, MINB) void gemm_dma_kernel(GemmArgs g, double beta,
                                                                      double gamma) {
    typedef DmaCfg<BM, BN, WM, WN, MINB, AT, RT> D;
    __shared__ __attribute__((aligned(1024))) char smem[2 * D::STAGE];
    static_assert(TRI != 3 || BM == BN, "square tiles for the triangular update");
    constexpr bool TRIA = TRI == 1 || TRI == 2;  // triangular A operand
    const int64_t tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
    int64_t tm, tn;
    if (TRI == 0) {
        tile_coords(tiles_m, tiles_n, tm, tn);
    } else if (TRI == 3) {
        upper_tile_coords(tm, tn);
    } else {
        // Triangle: a row tile's work grows with its distance into the
        // triangle.  Rows are taken heaviest first, and consecutive
        // workgroups walk along a row, so the round-robin dispatch over the
        // XCDs gives each XCD an equal share of every row (and a fixed set of
        // X column panels).
        const int64_t r = (int64_t)blockIdx.x / tiles_n;
        tn = (int64_t)blockIdx.x % tiles_n;
        tm = TRI == 1 ? tiles_m - 1 - r : r;
    }
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WM, wn = wave / WM;
    int oa[4], ox[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        oa[ks] = D::OA::frag_off(ks, wm * D::SM, lane);
        ox[ks] = D::OX::frag_off(ks, wn * D::SN, lane);
    }
    v4d acc[D::FM][D::FN];
#pragma unroll
    for (int i = 0; i < D::FM; ++i)
#pragma unroll
        for (int j = 0; j < D::FN; ++j) acc[i][j] = v4d{0, 0, 0, 0};

    // k-stages [kb, ke): all of K, or those meeting the triangle
    int64_t kb = 0, ke = (g.K + kDmaBk - 1) / kDmaBk;
    if (TRI == 1) {
        const int64_t last = m0 + BM < g.K ? m0 + BM : g.K;
        ke = (last + kDmaBk - 1) / kDmaBk;
    } else if (TRI == 2) {
        kb = m0 / kDmaBk;
    }
    // triangle mask of an A fragment element: row m0 + wm*SM + 16 i + lane%16,
    // column k0 + 4 ks + lane/16
    const int64_t mrow = m0 + wm * D::SM + (lane & 15);
    auto mask = [&](double v, int i, int64_t kcol) -> double {
        const int64_t m = mrow + 16 * i;
        const bool inside = TRI == 1 ? kcol <= m : kcol >= m;
        return inside ? ((UNIT && kcol == m) ? 1.0 : v) : 0.0;
    };
    if (kb < ke) dma_stage<D, AT, RT, DW>(g, m0, n0, kb * kDmaBk, smem + (kb & 1) * D::STAGE, wave, lane);
    __syncthreads();
    double la[D::FM], lx[D::FN];  // fragments of the last k-step, used after the barrier
    for (int64_t kt = kb; kt < ke; ++kt) {
        char* st = smem + (kt & 1) * D::STAGE;
        const double* sa = (const double*)st;
        const double* sx = (const double*)(st + D::OA::BYTES);
        const int64_t k0 = kt * kDmaBk;
        // a stage crossing the diagonal of this row tile (uniform)
        const bool diag = TRIA && k0 + kDmaBk > m0 && k0 < m0 + BM;
        if (kt + 1 < ke)
            dma_stage<D, AT, RT, DW>(g, m0, n0, (kt + 1) * kDmaBk, smem + ((kt + 1) & 1) * D::STAGE,
                                     wave, lane);
        if (kt > kb) {
#pragma unroll
            for (int i = 0; i < D::FM; ++i)
#pragma unroll
                for (int j = 0; j < D::FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(la[i], lx[j], acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int ks = 0; ks < 3; ++ks) {
            double fa[D::FM], fx[D::FN];
#pragma unroll
            for (int i = 0; i < D::FM; ++i) fa[i] = sa[oa[ks] + i * D::OA::fstride()];
            if (TRIA && diag) {
#pragma unroll
                for (int i = 0; i < D::FM; ++i) fa[i] = mask(fa[i], i, k0 + 4 * ks + (lane >> 4));
            }
#pragma unroll
            for (int j = 0; j < D::FN; ++j) fx[j] = sx[ox[ks] + j * D::OX::fstride()];
#pragma unroll
            for (int i = 0; i < D::FM; ++i)
#pragma unroll
                for (int j = 0; j < D::FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fx[j], acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < D::FM; ++i) la[i] = sa[oa[3] + i * D::OA::fstride()];
        if (TRIA && diag) {
#pragma unroll
            for (int i = 0; i < D::FM; ++i) la[i] = mask(la[i], i, k0 + 12 + (lane >> 4));
        }
#pragma unroll
        for (int j = 0; j < D::FN; ++j) lx[j] = sx[ox[3] + j * D::OX::fstride()];
        __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
    }
    if (kb < ke) {
#pragma unroll
        for (int i = 0; i < D::FM; ++i)
#pragma unroll
            for (int j = 0; j < D::FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(la[i], lx[j], acc[i][j], 0, 0, 0);
    }

    double* c = (double*)g.c;
#pragma unroll
    for (int i = 0; i < D::FM; ++i)
#pragma unroll
        for (int j = 0; j < D::FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = m0 + wm * D::SM + i * 16 + (lane >> 4) + 4 * r;
                const int64_t gj = n0 + wn * D::SN + j * 16 + (lane & 15);
                if (gi < g.M && gj < g.N && (TRI != 3 || gi <= gj)) {
                    double* p = RT ? c + gj + gi * g.ldc : c + gi + gj * g.ldc;
                    if (TRI == 0 || TRI == 3) *p = *p - acc[i][j][r];
                    else *p = (beta == 0.0 ? 0.0 : beta * *p) + gamma * acc[i][j][r];
                }
            }
}

// Shapes the direct-to-LDS kernel accepts.  16-byte loads: every index that
// is loaded in pairs is even, leading dimensions are even and operands
// 16-byte aligned (so a pair never straddles the end of a row or column).
// 4-byte loads: any shape.  Either way one stage of each operand must span
// less than the 1 GB byte-offset range used for a buffer load.
template <int BM, int BN, bool AT, bool RT>
bool dma_span_ok(const GemmArgs& g) {
    const int64_t lim = (int64_t)1 << 30;
    const int64_t sa = AT ? (kDmaBk + (BM - 1) * g.lda) * 8 : (BM + (kDmaBk - 1) * g.lda) * 8;
    const int64_t sx = RT ? (BN + (kDmaBk - 1) * g.ldx) * 8 : (kDmaBk + (BN - 1) * g.ldx) * 8;
    return sa < lim && sx < lim && (((uintptr_t)g.a | (uintptr_t)g.x) & 3) == 0;
}

template <int BM, int BN, bool AT, bool RT>
bool dma_ok(const GemmArgs& g) {
    if ((g.lda | g.ldx) & 1) return false;
    if (((uintptr_t)g.a | (uintptr_t)g.x) & 15) return false;
    if (g.K & 1) return false;                   // k pairs (A^T or X) and k tails
    if (!AT && (g.M & 1)) return false;          // m pairs
    if (RT && (g.N & 1)) return false;           // j pairs
    return dma_span_ok<BM, BN, AT, RT>(g);
}

template <int BM, int BN, int WM, int WN, int MINB, bool AT, bool RT, int TRI = 0, bool UNIT = false,
          bool DW = false>
hipError_t gemm_dma_launch_f64(const GemmArgs& g, hipStream_t s, double beta = 1.0,
                               double gamma = -1.0) {
    const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_dma_kernel<BM, BN, WM, WN, MINB, AT, RT, TRI, UNIT, DW>),
                       dim3((unsigned)tiles), dim3(64 * WM * WN), 0, s, g, beta, gamma);
    return hipGetLastError();
}

template <typename T, typename C, bool AT, bool RT, int TRI, bool UNIT>
__global__ __launch_bounds__(C::NT, C::MINB) void residual_kernel(GemmArgs g, T beta, T gamma) {
    __shared__ Smem<T, C> sm;
    const int64_t tiles_m = (g.M + C::BM - 1) / C::BM, tiles_n = (g.N + C::BN - 1) / C::BN;
    int64_t tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    gemm_tile<T, C, AT, RT, TRI, UNIT>(g, tm * C::BM, tn * C::BN, sm, beta, gamma);
}

template <typename T, typename C, bool AT, bool RT, int TRI, bool UNIT>
hipError_t residual_launch(const GemmArgs& g, double beta, double gamma, hipStream_t s) {
    const int64_t tiles = ((g.M + C::BM - 1) / C::BM) * ((g.N + C::BN - 1) / C::BN);
    hipLaunchKernelGGL((residual_kernel<T, C, AT, RT, TRI, UNIT>), dim3((unsigned)tiles),
                       dim3(C::NT), 0, s, g, (T)beta, (T)gamma);
    return hipGetLastError();
}

template <typename T, typename C, bool AT, bool RT>
__global__ __launch_bounds__(C::NT, C::MINB) void syrk_kernel(GemmArgs g) {
    static_assert(C::BM == C::BN, "square tiles");
    __shared__ Smem<T, C> sm;
    int64_t tm, tn;
    upper_tile_coords(tm, tn);
    gemm_tile<T, C, AT, RT, 3>(g, tm * C::BM, tn * C::BN, sm);
}

template <typename T, typename C, bool AT, bool RT>
hipError_t gemm_launch_t(const GemmArgs& g, hipStream_t s) {
    const int64_t tiles = ((g.M + C::BM - 1) / C::BM) * ((g.N + C::BN - 1) / C::BN);
    hipLaunchKernelGGL((gemm_kernel<T, C, AT, RT>), dim3((unsigned)tiles), dim3(C::NT), 0, s, g);
    return hipGetLastError();
}

template <typename T, typename C, bool AT, bool RT>
hipError_t gemm_group_launch_t(const GemmGroup& grp, hipStream_t s) {
    int64_t max_m = 0, max_n = 0;
    for (int i = 0; i < grp.count; ++i) {
        if (grp.g[i].M > max_m) max_m = grp.g[i].M;
        if (grp.g[i].N > max_n) max_n = grp.g[i].N;
    }
    if (max_m <= 0 || max_n <= 0) return hipSuccess;
    const int64_t tm = (max_m + C::BM - 1) / C::BM, tn = (max_n + C::BN - 1) / C::BN;
    hipLaunchKernelGGL((gemm_group_kernel<T, C, AT, RT>),
                       dim3((unsigned)(tm * tn), (unsigned)grp.count), dim3(C::NT), 0, s, grp, tm);
    return hipGetLastError();
}

// Tile configurations (index = tile argument).
typedef Cfg<128, 128, 16, 2, 2, 1> Tile0;  // 64x64 per wave
typedef Cfg<128, 128, 16, 2, 2, 2> Tile1;  // same, two workgroups per CU
typedef Cfg<128, 128, 32, 2, 2, 1> Tile2;  // deeper k-stage
typedef Cfg<64, 64, 16, 2, 2, 2> Tile3;    // small tiles for short M
typedef Cfg<64, 128, 16, 2, 2, 2> Tile4;   // short M, wide N
typedef Cfg<256, 128, 16, 4, 2, 1> Tile5;  // eight waves
typedef Cfg<64, 64, 16, 2, 2, 4> Tile6;    // small tiles, four workgroups per CU
typedef Cfg<64, 128, 32, 2, 2, 1> Tile7;   // short M, wide N, deeper k-stage
typedef Cfg<256, 128, 8, 4, 2, 2> Tile10;  // eight waves, short k-stage
// 8: short-K 64x64, 9: short-K 32x64; FP64 direct-to-LDS: 11: 256x128 on
// eight waves, 12: 128x128 on four waves (two workgroups per CU), 13:
// 128x128 on eight waves, 14: 64x64, 15: 128x64, 16: 64x128 (four waves each),
// 17: 64x32 (four waves of 32x16, for short products with many columns)
constexpr int kTiles = 18;

// Direct-to-LDS FP64 tiles where the shape allows them, else the register-
// staged tile of the same size.
// staging layouts exist for k-major operands of any width that is a multiple
// of 8 and for m/j-major ones 64 wide or a multiple of 128 wide
constexpr bool dma_width_ok(int bw, bool kmajor) { return kmajor ? bw % 8 == 0 : (bw == 64 || bw % 128 == 0); }

template <typename T, int BM, int BN, int WM, int WN, int MINB, bool AT, bool RT, typename Fallback>
hipError_t gemm_dma_or(const GemmArgs& g, hipStream_t s) {
    if constexpr (sizeof(T) == 8 && dma_width_ok(BM, AT) && dma_width_ok(BN, !RT)) {
        if (dma_ok<BM, BN, AT, RT>(g)) return gemm_dma_launch_f64<BM, BN, WM, WN, MINB, AT, RT>(g, s);
        if (dma_span_ok<BM, BN, AT, RT>(g))
            return gemm_dma_launch_f64<BM, BN, WM, WN, MINB, AT, RT, 0, false, true>(g, s);
    }
    return gemm_launch_t<T, Fallback, AT, RT>(g, s);
}

template <typename T, bool AT, bool RT>
hipError_t gemm_by_tile(int tile, const GemmArgs& g, hipStream_t s) {
    switch (tile) {
        case 0: return gemm_launch_t<T, Tile0, AT, RT>(g, s);
        case 1: return gemm_launch_t<T, Tile1, AT, RT>(g, s);
        case 2: return gemm_launch_t<T, Tile2, AT, RT>(g, s);
        case 3: return gemm_launch_t<T, Tile3, AT, RT>(g, s);
        case 4: return gemm_launch_t<T, Tile4, AT, RT>(g, s);
        case 5: return gemm_launch_t<T, Tile5, AT, RT>(g, s);
        case 6: return gemm_launch_t<T, Tile6, AT, RT>(g, s);
        case 7: return gemm_launch_t<T, Tile7, AT, RT>(g, s);
        case 8: return gemm_shortk_launch<T, 64, 64, 64, AT, RT>(g, s);
        case 9: return gemm_shortk_launch<T, 32, 64, 64, AT, RT>(g, s);
        case 10: return gemm_launch_t<T, Tile10, AT, RT>(g, s);
        case 11: return gemm_dma_or<T, 256, 128, 4, 2, 1, AT, RT, Tile5>(g, s);
        case 12: return gemm_dma_or<T, 128, 128, 2, 2, 2, AT, RT, Tile1>(g, s);
        case 13: return gemm_dma_or<T, 128, 128, 4, 2, 2, AT, RT, Tile1>(g, s);
        case 14: return gemm_dma_or<T, 64, 64, 2, 2, 4, AT, RT, Tile6>(g, s);
        case 15: return gemm_dma_or<T, 128, 64, 2, 2, 2, AT, RT, Tile3>(g, s);
        case 16: return gemm_dma_or<T, 64, 128, 2, 2, 2, AT, RT, Tile4>(g, s);
        case 17: return gemm_dma_or<T, 64, 32, 2, 2, 4, AT, RT, Tile6>(g, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, bool AT, bool RT>
hipError_t gemm_group_by_tile(int tile, const GemmGroup& grp, hipStream_t s) {
    switch (tile) {
        case 0: return gemm_group_launch_t<T, Tile0, AT, RT>(grp, s);
        case 1: return gemm_group_launch_t<T, Tile1, AT, RT>(grp, s);
        case 2: return gemm_group_launch_t<T, Tile2, AT, RT>(grp, s);
        case 3: return gemm_group_launch_t<T, Tile3, AT, RT>(grp, s);
        case 4: return gemm_group_launch_t<T, Tile4, AT, RT>(grp, s);
        case 5: return gemm_group_launch_t<T, Tile5, AT, RT>(grp, s);
        case 6: return gemm_group_launch_t<T, Tile6, AT, RT>(grp, s);
        case 7: return gemm_group_launch_t<T, Tile7, AT, RT>(grp, s);
        default: return gemm_group_launch_t<T, Tile3, AT, RT>(grp, s);
    }
}

template <typename T>
hipError_t gemm_any(int tile, bool at, bool rt, const GemmArgs& g, hipStream_t s) {
    if (!at && !rt) return gemm_by_tile<T, false, false>(tile, g, s);
    if (at && !rt) return gemm_by_tile<T, true, false>(tile, g, s);
    if (!at && rt) return gemm_by_tile<T, false, true>(tile, g, s);
    return gemm_by_tile<T, true, true>(tile, g, s);
}

template <typename T>
hipError_t gemm_group_any(int tile, bool at, bool rt, const GemmGroup& grp, hipStream_t s) {
    if (!at && !rt) return gemm_group_by_tile<T, false, false>(tile, grp, s);
    if (at && !rt) return gemm_group_by_tile<T, true, false>(tile, grp, s);
    if (!at && rt) return gemm_group_by_tile<T, false, true>(tile, grp, s);
    return gemm_group_by_tile<T, true, true>(tile, grp, s);
}

template <typename T, bool AT, bool RT, int TRI>
hipError_t residual_u(bool unit, const GemmArgs& g, double beta, double gamma, hipStream_t s) {
    // FP64: direct-to-LDS 128 x 128 tile on eight waves where the shape allows it
    if constexpr (sizeof(T) == 8) {
        if (dma_ok<128, 128, AT, RT>(g))
            return unit ? gemm_dma_launch_f64<128, 128, 4, 2, 2, AT, RT, TRI, true>(g, s, beta, gamma)
                        : gemm_dma_launch_f64<128, 128, 4, 2, 2, AT, RT, TRI, false>(g, s, beta, gamma);
        if (dma_span_ok<128, 128, AT, RT>(g))
            return unit ? gemm_dma_launch_f64<128, 128, 4, 2, 2, AT, RT, TRI, true, true>(g, s, beta, gamma)
                        : gemm_dma_launch_f64<128, 128, 4, 2, 2, AT, RT, TRI, false, true>(g, s, beta, gamma);
    }
    return unit ? residual_launch<T, Tile5, AT, RT, TRI, true>(g, beta, gamma, s)
                : residual_launch<T, Tile5, AT, RT, TRI, false>(g, beta, gamma, s);
}

template <typename T, int TRI>
hipError_t residual_t(bool at, bool rt, bool unit, const GemmArgs& g, double beta, double gamma,
                      hipStream_t s) {
    if (!at && !rt) return residual_u<T, false, false, TRI>(unit, g, beta, gamma, s);
    if (at && !rt) return residual_u<T, true, false, TRI>(unit, g, beta, gamma, s);
    if (!at && rt) return residual_u<T, false, true, TRI>(unit, g, beta, gamma, s);
    return residual_u<T, true, true, TRI>(unit, g, beta, gamma, s);
}

// Triangular update on square tiles of B: FP64 direct-to-LDS where the shape
// allows it, else the register-staged tile of the same size.
template <typename T, int B, int WM, int WN, int MINB, typename Fallback, bool AT, bool RT>
hipError_t syrk_tiles(const GemmArgs& g, hipStream_t s) {
    const int64_t t = (g.M + B - 1) / B, tiles = t * (t + 1) / 2;
    if constexpr (sizeof(T) == 8) {
        if (dma_ok<B, B, AT, RT>(g)) {
            hipLaunchKernelGGL((gemm_dma_kernel<B, B, WM, WN, MINB, AT, RT, 3>),
                               dim3((unsigned)tiles), dim3(64 * WM * WN), 0, s, g, 1.0, -1.0);
            return hipGetLastError();
        }
        if (dma_span_ok<B, B, AT, RT>(g)) {
            hipLaunchKernelGGL((gemm_dma_kernel<B, B, WM, WN, MINB, AT, RT, 3, false, true>),
                               dim3((unsigned)tiles), dim3(64 * WM * WN), 0, s, g, 1.0, -1.0);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((syrk_kernel<T, Fallback, AT, RT>), dim3((unsigned)tiles),
                       dim3(Fallback::NT), 0, s, g);
    return hipGetLastError();
}

// 128 x 128 tiles on eight waves once the triangle has enough of them to fill
// the GPU (order 4096: 528 tiles), 64 x 64 tiles below (order 2048: 528
// instead of 136).
template <typename T, bool AT, bool RT>
hipError_t syrk_t(const GemmArgs& g, hipStream_t s) {
    if (g.M >= 4096) return syrk_tiles<T, 128, 4, 2, 2, Tile1, AT, RT>(g, s);
    return syrk_tiles<T, 64, 2, 2, 4, Tile3, AT, RT>(g, s);
}

}  // namespace

hipError_t launch_syrk(int dtype, bool a_trans, bool rhs_trans, const GemmArgs& g, hipStream_t s) {
    if (g.M != g.N) return hipErrorInvalidValue;
    if (g.M <= 0 || g.K <= 0) return hipSuccess;
    if (a_trans == rhs_trans) return hipErrorInvalidValue;
    if (dtype == 0)
        return a_trans ? syrk_t<double, true, false>(g, s) : syrk_t<double, false, true>(g, s);
    return a_trans ? syrk_t<float, true, false>(g, s) : syrk_t<float, false, true>(g, s);
}

hipError_t launch_trmm(int dtype, bool a_trans, bool rhs_trans, int tri, bool unit, double beta,
                       double gamma, const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (tri != 1 && tri != 2) return hipErrorInvalidValue;
    if (dtype == 0)
        return tri == 1 ? residual_t<double, 1>(a_trans, rhs_trans, unit, g, beta, gamma, s)
                        : residual_t<double, 2>(a_trans, rhs_trans, unit, g, beta, gamma, s);
    return tri == 1 ? residual_t<float, 1>(a_trans, rhs_trans, unit, g, beta, gamma, s)
                    : residual_t<float, 2>(a_trans, rhs_trans, unit, g, beta, gamma, s);
}

int gemm_tile_count() { return kTiles; }

// Default tile for a product shape, from sweeps of the configurations on
// MI355X (N = 8192).  FP64: the direct-to-LDS 128 x 128 eight-wave tile once
// M and K reach 1024, the direct-to-LDS 64 x 64 tile below that and the
// 64 x 32 tile for M <= 256 (each falls back to a register-staged tile on
// shapes the direct path does not accept).
// FP32: the short-K kernel for small square updates, 64 x 64 tiles for short
// M or K, the eight-wave 256 x 128 tile otherwise.
int gemm_default_tile(int dtype, int64_t M, int64_t N, int64_t K) {
    (void)N;
    if (dtype == 0) return (M >= 1024 && K >= 1024) ? 13 : (M <= 256 ? 17 : 14);
    if (K <= 160 && M <= 160) return 9;
    if (M <= 768 || K <= 384) return 3;
    return 5;
}

hipError_t launch_gemm(int dtype, bool a_trans, bool rhs_trans, const GemmArgs& g, hipStream_t s,
                       int tile) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
    if (tile < 0) tile = gemm_default_tile(dtype, g.M, g.N, g.K);
    return dtype == 0 ? gemm_any<double>(tile, a_trans, rhs_trans, g, s)
                      : gemm_any<float>(tile, a_trans, rhs_trans, g, s);
}

hipError_t launch_gemm_group(int dtype, bool a_trans, bool rhs_trans, const GemmGroup& grp,
                             hipStream_t s, int tile) {
    if (grp.count <= 0) return hipSuccess;
    if (grp.count > kMaxGroup) return hipErrorInvalidValue;
    if (tile < 0) tile = gemm_default_tile(dtype, grp.g[0].M, grp.g[0].N, grp.g[0].K);
    return dtype == 0 ? gemm_group_any<double>(tile, a_trans, rhs_trans, grp, s)
                      : gemm_group_any<float>(tile, a_trans, rhs_trans, grp, s);
}

}  // namespace redsea
