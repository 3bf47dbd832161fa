// Device helpers shared by the uint8 and float32 kernels.
#pragma once

#include "rfim_internal.h"

namespace rfim {

// Loads and stores through global-address-space pointers.  Beam pointers come
// from launch tables in memory, so the compiler would otherwise address them
// as flat, which may alias LDS and forces waits on LDS traffic around them.
// (uint4 goes through a native vector type: copying HIP's uint4 struct takes a
// generic reference and would turn the access back into a flat one.)
typedef unsigned int rfim_u32x4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ inline T ld_global(const void* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
template <>
__device__ inline uint4 ld_global<uint4>(const void* p) {
    const rfim_u32x4 v = *(const __attribute__((address_space(1))) rfim_u32x4*)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
template <typename T>
__device__ inline void st_global(void* p, const T& v) {
    *(__attribute__((address_space(1))) T*)p = v;
}
template <>
__device__ inline void st_global<uint4>(void* p, const uint4& v) {
    rfim_u32x4 w;
    w.x = v.x; w.y = v.y; w.z = v.z; w.w = v.w;
    *(__attribute__((address_space(1))) rfim_u32x4*)p = w;
}

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
