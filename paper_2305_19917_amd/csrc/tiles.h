// Device-side tile ordering shared by the product kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace redsea {

// Workgroups are dispatched round-robin over the eight XCDs (each with its
// own L2).  The launch index is remapped so that every XCD receives one
// contiguous range of logical tiles, and logical tiles walk bands of GM
// row-tiles along N, so an XCD's resident workgroups share A row panels and
// X column panels in its L2.
__device__ __forceinline__ void tile_coords(int64_t tiles_m, int64_t tiles_n, int64_t& tm,
                                            int64_t& tn) {
    constexpr int64_t kXcd = 8, GM = 8;
    const int64_t nwg = (int64_t)gridDim.x;
    int64_t bid = blockIdx.x;
    if (nwg % kXcd == 0) bid = (bid % kXcd) * (nwg / kXcd) + bid / kXcd;
    const int64_t band = GM * tiles_n;
    const int64_t first = (bid / band) * GM;
    const int64_t gsz = tiles_m - first < GM ? tiles_m - first : GM;
    const int64_t r = bid % band;
    tm = first + r % gsz;
    tn = r / gsz;
}

}  // namespace redsea
