// Solve entry point for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The only scratch memory of a native-precision solve is the
// packed copy of its diagonal blocks, or the flags of the one-launch thin
// solve; here it lives in a fixed file-scope device array instead of the
// library's per-stream workspace, so a call launches kernels and nothing else.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/redsea.h"
#include "exec.h"
#include "kernels.h"

namespace redsea {

namespace {

constexpr size_t kScratchBytes = REDSEA_NOALLOC_SCRATCH_BYTES;
constexpr size_t kFlagBytes = (size_t)64 << 10;  // the one-launch solve's flags (up to ~32000 right-hand sides)

// Each device that loads the library holds its own copy of this array until
// the process ends.  Host code never uses its name as an address: the device
// address comes from hipGetSymbolAddress, per device.
__device__ __attribute__((aligned(256))) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[64] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_ptr(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return REDSEA_ERR_HIP;
    if (dev < 0 || dev >= 64) return REDSEA_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return REDSEA_ERR_HIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return REDSEA_OK;
}

}  // namespace

}  // namespace redsea

using namespace redsea;

extern "C" {

int redsea_trsm_noalloc(int dtype, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                        double alpha, const void* A, int64_t lda, void* B, int64_t ldb,
                        const redsea_opts* opts, void* stream) {
    int rc = check_args(dtype, side, uplo, trans, diag, m, n, A, lda, B, ldb, alpha != 0.0);
    if (rc) return rc;
    int variant = opts ? opts->variant : 0;
    int nb = opts ? opts->nb : 0;
    int precision = opts ? opts->precision : 0;
    if (variant < 0 || variant > 3) return -13;
    if (!(nb == 0 || nb == 16 || nb == 32 || nb == 64 || nb == 128 || nb == 256 || nb == 512))
        return -13;
    if (precision < 0 || precision > 3) return -13;
    // refinement needs a workspace the size of the problem
    if (precision == REDSEA_PREC_FP32_IR || precision == REDSEA_PREC_BF16_IR)
        return REDSEA_ERR_UNSUPPORTED;
    // the array's address on this device (looked up on the first call, also
    // an empty one, so that a caller can do it before capturing a graph)
    void* ptr = nullptr;
    if ((rc = scratch_ptr(&ptr))) return rc;
    if (m == 0 || n == 0) return REDSEA_OK;
    if (variant == 0) variant = VAR_RECURSIVE;
    const Canon c = canonicalize(dtype, side, uplo, trans, diag, m, n, A, lda, B, ldb);
    const int64_t leaf = pick_nb(nb, c.k);
    // the array: the one-launch solve's flags first, then the packed blocks
    if (alpha != 0.0 && kFlagBytes + packed_bytes(c, leaf) > kScratchBytes)
        return REDSEA_ERR_TOO_LARGE;
    int* flags = (size_t)thin_flag_count(c.k, c.nrhs) * sizeof(int) <= kFlagBytes ? (int*)ptr : nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (alpha != 1.0) {
        if (launch_scale(dtype, B, m, n, ldb, alpha, s) != hipSuccess) return REDSEA_ERR_HIP;
        if (alpha == 0.0) return REDSEA_OK;
    }
    return execute(c, variant, leaf, s, (unsigned char*)ptr + kFlagBytes, flags);
}

}  // extern "C"
