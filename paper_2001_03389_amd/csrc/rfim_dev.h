// Device helpers shared by the uint8 and float32 kernels.
#pragma once

#include "rfim_internal.h"

namespace rfim {

// last beam of a launch table whose first row (tile) is <= g
__device__ inline int find_beam_by_row(const DevBeam* beams, int nbeams, int64_t g) {
    int lo = 0, hi = nbeams - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (beams[mid].row0 <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline int find_beam_by_tile(const DevBeam* beams, int nbeams, int64_t g) {
    int lo = 0, hi = nbeams - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (beams[mid].tile0 <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// XCD-aware work-group order: the hardware deals work-groups round-robin to
// the 8 XCDs; give each XCD a contiguous range of tiles so that neighbouring
// tiles (which share L2 lines of a row) are handled by the same XCD's L2.
__device__ inline int64_t xcd_remap(int64_t i, int64_t n) {
    const int64_t X = 8;
    int64_t x = i % X, j = i / X;
    int64_t q = n / X, r = n % X;
    return x * q + (x < r ? x : r) + j;
}

}  // namespace rfim
