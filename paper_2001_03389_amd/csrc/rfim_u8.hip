// uint8 sigma-cut kernels for gfx950 (RFIm, arXiv:2001.03389, Section IV).
//
// Two kernels per run of [TD steps][FD steps]:
//  * k_td_rows_u8 -- one work-group per channel row.  Builds the row's exact
//    256-bin histogram (every TD statistic of a uint8 row is a function of it:
//    S1, S2, the lower median), then runs every TD step of the run on the
//    histogram alone: the cut interval of step j is computed exactly, the
//    counts outside it move to the replacement value's bin, and step j+1 sees
//    the modified row without another pass over the data.  The result is a
//    per-row record of the composite map (nested intervals plus the value and
//    flag byte a sample gets when it first falls outside them).
//  * k_fused_u8 -- one work-group per (beam, time tile).  Streams a
//    [C x Tt] tile from HBM, applies each row's TD map, stores it transposed in
//    LDS ([Tt][C], channels contiguous) and runs every FD step of the run on
//    the tile: per time sample, bin sums, the exact sum of squared mean-
//    corrected values, the exact cut and the replacement.  It then writes the
//    tile (and flag bits) back.
#include "rfim_exact.h"

namespace rfim {

namespace {

__device__ inline int find_beam_by_row(const DevBeam* beams, int nbeams, int64_t g) {
    int lo = 0, hi = nbeams - 1;  // last beam with row0 <= g
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

// block-wide sum of one u64 per thread (256 threads, 4 waves)
__device__ inline uint64_t block_sum_u64(uint64_t v, uint64_t* red) {
    v = wave_sum_u64(v);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// exclusive prefix sum over the 256 threads (u32 values)
__device__ inline uint32_t block_excl_scan_u32(uint32_t v, uint32_t* red) {
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    __syncthreads();
    if (lane == 63) red[wave] = incl;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; w++) base += red[w];
    return base + incl - v;
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

}  // namespace

__global__ __launch_bounds__(kBlock) void k_td_rows_u8(const DevBeam* __restrict__ beams,
                                                       int nbeams, Segment seg,
                                                       uint32_t* __restrict__ rec,
                                                       unsigned long long* __restrict__ counts,
                                                       int count_stride) {
    __shared__ uint32_t hist[4][256];
    __shared__ uint64_t red64[4];
    __shared__ uint32_t red32[4];
    __shared__ int s_lo[kMaxSteps], s_hi[kMaxSteps], s_r[kMaxSteps];
    __shared__ int s_med;

    const int tid = threadIdx.x, wave = tid >> 6;
    const int64_t g = blockIdx.x;
    const int b = find_beam_by_row(beams, nbeams, g);
    const DevBeam& bm = beams[b];
    const int64_t c = g - bm.row0;
    const int64_t T = bm.T;
    const uint8_t* row = (const uint8_t*)bm.in + c * bm.stride;

    for (int i = tid; i < 4 * 256; i += kBlock) (&hist[0][0])[i] = 0;
    __syncthreads();

    // histogram: unaligned head bytes, aligned dwords, tail bytes
    int64_t head = (int64_t)((4 - ((uintptr_t)row & 3)) & 3);
    if (head > T) head = T;
    for (int64_t i = tid; i < head; i += kBlock) atomicAdd(&hist[wave][row[i]], 1u);
    const int64_t nd = (T - head) >> 2;
    const uint32_t* rw = (const uint32_t*)(row + head);
    for (int64_t i = tid; i < nd; i += kBlock) {
        uint32_t v = __builtin_nontemporal_load(rw + i);
        atomicAdd(&hist[wave][v & 255u], 1u);
        atomicAdd(&hist[wave][(v >> 8) & 255u], 1u);
        atomicAdd(&hist[wave][(v >> 16) & 255u], 1u);
        atomicAdd(&hist[wave][v >> 24], 1u);
    }
    for (int64_t i = head + 4 * nd + tid; i < T; i += kBlock) atomicAdd(&hist[wave][row[i]], 1u);
    __syncthreads();

    // thread v owns histogram bin v from here on
    const uint32_t v = (uint32_t)tid;
    uint32_t hv = hist[0][v] + hist[1][v] + hist[2][v] + hist[3][v];
    const uint64_t n = (uint64_t)T;

    for (int j = 0; j < seg.n_td; j++) {
        const SegStep& st = seg.td[j];
        uint64_t S1 = block_sum_u64((uint64_t)hv * v, red64);
        uint64_t S2 = block_sum_u64((uint64_t)hv * v * v, red64);
        if (st.replace == RFIM_REPLACE_MEDIAN) {
            // lower median: the bin holding rank floor((n-1)/2)
            uint32_t before = block_excl_scan_u32(hv, red32);
            uint64_t q = (n - 1) / 2;
            if (hv > 0 && before <= q && q < (uint64_t)before + hv) s_med = (int)v;
        }
        __syncthreads();
        if (tid == 0) {
            int lo, hi;
            td_bounds_u8(n, S1, S2, st.kx, &lo, &hi);
            s_lo[j] = lo;
            s_hi[j] = hi;
            s_r[j] = st.replace == RFIM_REPLACE_MEDIAN ? s_med : (int)rn_div_u64(S1, n);
        }
        __syncthreads();
        const int lo = s_lo[j], hi = s_hi[j], r = s_r[j];
        const bool out = (int)v < lo || (int)v > hi;
        uint64_t moved = block_sum_u64(out ? hv : 0u, red64);
        if (out) hv = 0;
        if ((int)v == r) hv += (uint32_t)moved;
        if (tid == 0 && counts && st.bit >= 0 && moved)
            atomicAdd(&counts[(int64_t)bm.cidx * count_stride + st.bit], (unsigned long long)moved);
    }

    // composite record of the run, one u32 per step:
    //   [7:0] L_j, [15:8] H_j  -- nested interval: a sample stays untouched
    //                             through step j iff L_j <= x <= H_j
    //   [23:16] value a sample first flagged at step j ends with
    //   [31:24] flag bits it collects (step j and any later step that cuts
    //           the replacement value)
    if (tid < seg.n_td) {
        const int j = tid;
        int L = 0, H = 255;
        for (int i = 0; i <= j; i++) {
            L = max(L, s_lo[i]);
            H = min(H, s_hi[i]);
        }
        int val = s_r[j];
        uint32_t f = seg.td[j].bit >= 0 ? (1u << seg.td[j].bit) : 0u;
        for (int i = j + 1; i < seg.n_td; i++) {
            if (val < s_lo[i] || val > s_hi[i]) {
                val = s_r[i];
                if (seg.td[i].bit >= 0) f |= 1u << seg.td[i].bit;
            }
        }
        // an empty interval is encoded as L = 1, H = 0
        if (L > H) {
            L = 1;
            H = 0;
        }
        rec[g * seg.n_td + j] = (uint32_t)L | ((uint32_t)H << 8) | ((uint32_t)val << 16) | (f << 24);
    }
}

namespace {

// group of G consecutive lanes (G a power of two <= 64): sum of a u128
__device__ inline u128 group_sum_u128(u128 v, int G) {
    uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
    for (int o = 1; o < G; o <<= 1) {
        uint64_t olo = __shfl_xor(lo, o, 64);
        uint64_t ohi = __shfl_xor(hi, o, 64);
        uint64_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1 : 0);
        lo = nlo;
    }
    return ((u128)hi << 64) | lo;
}

// lower median (rank floor((n-1)/2)) of n bytes spaced `step` apart in LDS:
// the largest value v with #{x < v} <= rank, found bit by bit
__device__ inline int lds_lower_median_u8(const uint8_t* p, int64_t n, int64_t step) {
    const int64_t rank = (n - 1) / 2;
    int prefix = 0;
    for (int bit = 7; bit >= 0; bit--) {
        int cand = prefix | (1 << bit);
        int64_t below = 0;
        for (int64_t i = 0; i < n; i++) below += p[i * step] < cand;
        if (below <= rank) prefix = cand;
    }
    return prefix;
}

__device__ inline uint8_t td_map(uint8_t x, const uint32_t* r, int m, uint8_t* fl) {
    uint8_t out = x, f = 0;
    for (int j = m - 1; j >= 0; j--) {
        uint32_t e = r[j];
        int L = e & 255, H = (e >> 8) & 255;
        if ((int)x < L || (int)x > H) {
            out = (uint8_t)(e >> 16);
            f = (uint8_t)(e >> 24);
        }
    }
    *fl |= f;
    return out;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_fused_u8(const DevBeam* __restrict__ beams, int nbeams,
                                                     int64_t total_tiles, Segment seg,
                                                     const uint32_t* __restrict__ rec,
                                                     unsigned long long* __restrict__ counts,
                                                     int count_stride) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ unsigned long long s_cnt[kMaxSteps];

    const int tid = threadIdx.x;
    const int64_t g = xcd_remap(blockIdx.x, total_tiles);
    const int b = find_beam_by_tile(beams, nbeams, g);
    const DevBeam& bm = beams[b];
    const int64_t C = bm.C, T = bm.T, stride = bm.stride;
    const int Tt = bm.Tt, Cp = bm.Cp;
    const int64_t t0 = (g - bm.tile0) * Tt;
    const int tw = Tt >> 2;
    const bool want_flags = seg.flags_mode != 0 && bm.flags != nullptr;
    uint8_t* tile = lds;
    uint8_t* ftile = lds + (size_t)Tt * Cp;
    const uint8_t* in = (const uint8_t*)bm.in;
    uint8_t* out = (uint8_t*)bm.out;

    if (tid < kMaxSteps) s_cnt[tid] = 0;

    // ---- phase 1: load rows, apply the TD maps, store transposed into LDS
    for (int64_t idx = tid; idx < C * tw; idx += kBlock) {
        const int64_t c = idx / tw;
        const int w = (int)(idx - c * tw);
        const int64_t t = t0 + 4 * w;
        const uint8_t* src = in + c * stride + t;
        uint8_t x[4], f[4] = {0, 0, 0, 0};
        if (t + 3 < T && (((uintptr_t)src) & 3) == 0) {
            uint32_t d = *(const uint32_t*)src;
            x[0] = d & 255; x[1] = (d >> 8) & 255; x[2] = (d >> 16) & 255; x[3] = d >> 24;
        } else {
#pragma unroll
            for (int j = 0; j < 4; j++) x[j] = (t + j < T) ? src[j] : 0;
        }
        if (seg.flags_mode == 2 && want_flags) {
            const uint8_t* fs = bm.flags + c * stride + t;
#pragma unroll
            for (int j = 0; j < 4; j++) f[j] = (t + j < T) ? fs[j] : 0;
        }
        if (seg.n_td > 0) {
            uint32_t r[kMaxSteps];
            const uint32_t* rp = rec + (bm.row0 + c) * seg.n_td;
            for (int j = 0; j < seg.n_td; j++) r[j] = rp[j];
#pragma unroll
            for (int j = 0; j < 4; j++) x[j] = td_map(x[j], r, seg.n_td, &f[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            tile[(size_t)(4 * w + j) * Cp + c] = x[j];
            if (want_flags) ftile[(size_t)(4 * w + j) * Cp + c] = f[j];
        }
    }
    __syncthreads();

    // ---- phase 2: FD steps; G consecutive lanes own one time sample
    if (seg.n_fd > 0) {
        const int G = kBlock / Tt;
        const int tl = tid / G, q = tid % G;
        const bool valid = t0 + tl < T;
        uint8_t* colp = tile + (size_t)tl * Cp;
        uint8_t* fcol = ftile + (size_t)tl * Cp;
        for (int s = 0; s < seg.n_fd; s++) {
            const SegStep& st = seg.fd[s];
            const int64_t B = st.bin == 0 ? C : st.bin;
            const int64_t nb = C / B;
            // sum over bins of B * (B * Q_b - S_b^2) = sum over channels of Z_c^2
            u128 sz2 = 0;
            for (int64_t bb = q; bb < nb; bb += G) {
                uint64_t S = 0, Q = 0;
                const uint8_t* p = colp + bb * B;
                for (int64_t i = 0; i < B; i++) {
                    uint32_t x = p[i];
                    S += x;
                    Q += x * x;
                }
                sz2 += (u128)B * ((u128)B * Q - (u128)S * S);
            }
            sz2 = group_sum_u128(sz2, G);
            const uint64_t z = fd_zthr(sz2, C, st.kx, (uint64_t)B * 255u);
            uint64_t nflag = 0;
            for (int64_t bb = q; bb < nb; bb += G) {
                uint8_t* p = colp + bb * B;
                uint64_t S = 0;
                for (int64_t i = 0; i < B; i++) S += p[i];
                int64_t lo = ceil_div((int64_t)S - (int64_t)z, B);
                int64_t hi = floor_div((int64_t)S + (int64_t)z, B);
                int64_t cnt = 0;
                for (int64_t i = 0; i < B; i++) cnt += ((int64_t)p[i] < lo) || ((int64_t)p[i] > hi);
                if (cnt == 0) continue;
                const int r = st.replace == RFIM_REPLACE_MEDIAN ? lds_lower_median_u8(p, B, 1)
                                                               : (int)rn_div_u64(S, (uint64_t)B);
                for (int64_t i = 0; i < B; i++) {
                    if (((int64_t)p[i] < lo) || ((int64_t)p[i] > hi)) {
                        p[i] = (uint8_t)r;
                        if (want_flags && st.bit >= 0) fcol[bb * B + i] |= (uint8_t)(1u << st.bit);
                    }
                }
                nflag += (uint64_t)cnt;
            }
            if (valid && nflag && counts && st.bit >= 0) atomicAdd(&s_cnt[s], (unsigned long long)nflag);
        }
    }
    __syncthreads();

    // ---- phase 3: write the tile back in row order
    for (int64_t idx = tid; idx < C * tw; idx += kBlock) {
        const int64_t c = idx / tw;
        const int w = (int)(idx - c * tw);
        const int64_t t = t0 + 4 * w;
        uint8_t* dst = out + c * stride + t;
        uint8_t x[4], f[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            x[j] = tile[(size_t)(4 * w + j) * Cp + c];
            f[j] = want_flags ? ftile[(size_t)(4 * w + j) * Cp + c] : 0;
        }
        if (t + 3 < T && (((uintptr_t)dst) & 3) == 0) {
            *(uint32_t*)dst = (uint32_t)x[0] | ((uint32_t)x[1] << 8) | ((uint32_t)x[2] << 16) |
                              ((uint32_t)x[3] << 24);
        } else {
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (t + j < T) dst[j] = x[j];
        }
        if (want_flags) {
            uint8_t* fd = bm.flags + c * stride + t;
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (t + j < T) fd[j] = f[j];
        }
    }
    if (counts && seg.n_fd > 0) {
        __syncthreads();
        if (tid < seg.n_fd && s_cnt[tid] && seg.fd[tid].bit >= 0)
            atomicAdd(&counts[(int64_t)bm.cidx * count_stride + seg.fd[tid].bit], s_cnt[tid]);
    }
}

hipError_t launch_td_rows_u8(const DevBeam* d_beams, int nbeams, int64_t total_rows,
                             const Segment& seg, uint32_t* d_rec, unsigned long long* d_counts,
                             int count_stride, hipStream_t s) {
    if (total_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_td_rows_u8, dim3((unsigned)total_rows), dim3(kBlock), 0, s, d_beams,
                       nbeams, seg, d_rec, d_counts, count_stride);
    return hipGetLastError();
}

hipError_t launch_fused_u8(const DevBeam* d_beams, int nbeams, int64_t total_tiles,
                           const Segment& seg, const uint32_t* d_rec, size_t lds_bytes,
                           unsigned long long* d_counts, int count_stride, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fused_u8, dim3((unsigned)total_tiles), dim3(kBlock), lds_bytes, s,
                       d_beams, nbeams, total_tiles, seg, d_rec, d_counts, count_stride);
    return hipGetLastError();
}

}  // namespace rfim
