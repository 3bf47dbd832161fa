// uint8 sigma-cut kernels for gfx950 (RFIm, arXiv:2001.03389, Section IV).
//
// Two kernels per run of [TD steps][FD steps]:
//  * k_td_rows_u8 -- one wave per channel row (four rows per work-group), the
//    row read in 16 KB chunks of loads.  Builds the row's exact
//    256-bin histogram (every TD statistic of a uint8 row is a function of it:
//    S1, S2, the lower median), then runs every TD step of the run on the
//    histogram alone: the step's exact cut gives the interval of byte values
//    kept, the counts of the values cut move to the replacement value's bin,
//    and step j+1 sees the modified row without another pass over the data.  The
//    result is a per-row record of the composite map: nested intervals, plus the
//    value and flag byte a sample gets when it first falls outside them.
//  * k_fused_u8 -- one work-group per (beam, time tile).  Streams a [C x Tt]
//    tile from HBM four rows at a time, transposes 4x4 byte blocks in registers
//    and stores the tile in LDS as [Tt][C] (channels contiguous).  Samples a TD
//    step cuts are rare: a byte-parallel mask finds them and an LDS worklist
//    applies their TD maps.  Every FD step then runs on the LDS tile: per time
//    sample, dot4 bin sums and sums of squares, the exact sum of squared mean-
//    corrected values, the exact cut and a byte-select replacement.  The tile is
//    transposed back and written out.
#include <algorithm>

#include "rfim_dev.h"
#include "rfim_exact.h"

namespace rfim {

namespace {

// Bytes of x outside [lo, hi] (0 <= lo, hi <= 255; lo > hi means empty) as
// 0xFF, the others as 0x00.  Works on the even and odd bytes as 16-bit lanes:
// lane + (0x8000 - lo) has bit 15 set iff lane >= lo, lane + (0x7FFF - hi) has
// it set iff lane > hi; v_perm replicates each lane's bit 15 into a byte.
__device__ inline uint32_t outside_mask(uint32_t x, uint32_t klo, uint32_t khi) {
    const uint32_t e = x & 0x00FF00FFu;
    const uint32_t o = (x >> 8) & 0x00FF00FFu;
    const uint32_t oe = ~(e + klo) | (e + khi);
    const uint32_t oo = ~(o + klo) | (o + khi);
    return __builtin_amdgcn_perm(oo, oe, 0x0B090A08u);
}

__device__ inline uint32_t klo_of(uint32_t lo) { return (0x8000u - lo) * 0x00010001u; }
__device__ inline uint32_t khi_of(uint32_t hi) { return (0x7FFFu - hi) * 0x00010001u; }

// 4x4 byte transpose: y[j] byte i = x[i] byte j (its own inverse)
__device__ inline void transpose4(const uint32_t x[4], uint32_t y[4]) {
    const uint32_t t0 = __builtin_amdgcn_perm(x[1], x[0], 0x06020400u);
    const uint32_t t1 = __builtin_amdgcn_perm(x[1], x[0], 0x07030501u);
    const uint32_t t2 = __builtin_amdgcn_perm(x[3], x[2], 0x06020400u);
    const uint32_t t3 = __builtin_amdgcn_perm(x[3], x[2], 0x07030501u);
    y[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
    y[1] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    y[2] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    y[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// load 4 bytes of a row starting at sample t (bytes at or past T read as 0)
__device__ inline uint32_t load4(const uint8_t* p, int64_t t, int64_t T) {
    if (t + 3 < T && (((uintptr_t)p) & 3) == 0) return *(const uint32_t*)p;
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < 4; j++)
        if (t + j < T) v |= (uint32_t)p[j] << (8 * j);
    return v;
}

__device__ inline void store4(uint8_t* p, uint32_t v, int64_t t, int64_t T) {
    if (t + 3 < T && (((uintptr_t)p) & 3) == 0) {
        *(uint32_t*)p = v;
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; j++)
        if (t + j < T) p[j] = (uint8_t)(v >> (8 * j));
}

}  // namespace

// ---------------------------------------------------------------------------
// TD statistics and decisions, one wave per row (4 rows per work-group)
// ---------------------------------------------------------------------------
namespace {

constexpr int kHistCopies = 4;     // per wave, lane & 3 picks the copy
constexpr int kHistPitch = 272;    // words per histogram copy (copies 16 banks apart)
constexpr int kRowsPerWG = kBlock / 64;

// Sum over the 64 lanes with DPP row rotations (every lane of a 16-lane row
// ends with the row sum) and four lane reads; the result is wave-uniform.
__device__ inline uint32_t wave_sum_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false);  // row_ror:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false);  // row_ror:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xf, 0xf, false);  // row_ror:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xf, 0xf, false);  // row_ror:1
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

// wave sum of u64 values whose total is known to fit
__device__ inline uint64_t wave_sum_u64_split(uint64_t v) {
    // 3 x 22-bit slices: each slice sum stays below 2^28 for 64 lanes
    const uint32_t a = wave_sum_u32((uint32_t)(v & 0x3FFFFFu));
    const uint32_t b = wave_sum_u32((uint32_t)((v >> 22) & 0x3FFFFFu));
    const uint32_t c = wave_sum_u32((uint32_t)(v >> 44));
    return (uint64_t)a + ((uint64_t)b << 22) + ((uint64_t)c << 44);
}

// num / den rounded to nearest, ties to even, for num < 2^53 and den < 2^32:
// FP64 quotient, then an exact integer correction
__device__ inline uint64_t rn_div_small(uint64_t num, uint64_t den) {
    uint64_t q = (uint64_t)((double)num / (double)den);
    while (q * den > num) q--;
    while ((q + 1) * den <= num) q++;
    const uint64_t r = num - q * den;
    if (2 * r > den || (2 * r == den && (q & 1))) q++;
    return q;
}

__device__ inline void hist4(uint32_t* h, uint32_t v) {
    atomicAdd(&h[v & 255u], 1u);
    atomicAdd(&h[(v >> 8) & 255u], 1u);
    atomicAdd(&h[(v >> 16) & 255u], 1u);
    atomicAdd(&h[v >> 24], 1u);
}

}  // namespace

// One pass over a row by one wave: dword-aligned 16-byte loads for the bulk,
// single bytes for the unaligned head and the tail.  The bulk goes in chunks
// of kRowChunk 16-byte loads per lane, all issued before any is consumed, so
// a wave waits for memory once per chunk (16 KB of row) rather than once per
// load.
constexpr int kRowChunk = 16;
template <typename FD, typename FB>
__device__ inline void row_pass(const uint8_t* row, int64_t T, int lane, FD&& on_dword, FB&& on_byte) {
    int64_t head = (int64_t)((4 - ((uintptr_t)row & 3)) & 3);
    if (head > T) head = T;
    if (lane < head) on_byte((uint32_t)row[lane]);
    const int64_t n16 = (T - head) >> 4;
    const uint8_t* body = row + head;
    for (int64_t base = 0; base < n16; base += 64 * kRowChunk) {
        uint4 v[kRowChunk];
#pragma unroll
        for (int u = 0; u < kRowChunk; u++) {
            const int64_t i = base + lane + 64 * u;
            v[u] = i < n16 ? ld_global<uint4>(body + 16 * i) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < kRowChunk; u++) {
            if (base + lane + 64 * u < n16) {
                on_dword(v[u].x); on_dword(v[u].y); on_dword(v[u].z); on_dword(v[u].w);
            }
        }
    }
    for (int64_t k = head + 16 * n16 + lane; k < T; k += 64) on_byte((uint32_t)row[k]);
}

// Kept interval of a TD step over the byte values: v is kept exactly when
// |n*v - S1| <= z, z being the largest integer with z^2 <= k^2 * D (the exact
// test of the row's mean and population deviation); *lo > *hi when no value
// is kept.  Wave-uniform.
// floor(a / n) for |a| < 2^53 and 0 < n < 2^31: FP64 quotient, exact correction
__device__ inline int64_t floor_div_fp(int64_t a, int64_t n) {
    int64_t q = (int64_t)floor((double)a / (double)n);
    while (q * n > a) q--;
    while ((q + 1) * n <= a) q++;
    return q;
}

__device__ inline void td_interval(uint64_t n, uint64_t S1, u128 D, const KExact& kx, int* lo, int* hi) {
    const int64_t z = (int64_t)fd_zthr(D, 1, kx, 255 * n);
    const int64_t l = -floor_div_fp(z - (int64_t)S1, (int64_t)n), h = floor_div_fp((int64_t)S1 + z, (int64_t)n);
    *lo = (int)(l < 0 ? 0 : (l > 256 ? 256 : l));
    *hi = (int)(h > 255 ? 255 : (h < -1 ? -1 : h));
}

// Runs every TD step of the run for one row (one wave).  The row is described
// by hv[u] = number of samples with byte value 4*lane+u among the tracked
// values, plus an aggregate (nJ samples, sums S1J, S2J) of untracked values
// that all lie in [jlo, jhi].  Untracked values are never cut as long as every
// step keeps [jlo, jhi]; if a step does not, returns false and writes nothing
// (the caller retries with every value tracked).  Median steps need nJ == 0.
__device__ bool td_decide(const Segment& seg, uint64_t n, uint32_t hv[4], uint64_t nJ, uint64_t S1J,
                          uint64_t S2J, int jlo, int jhi, int lane, int* s_lo, int* s_hi, int* s_r,
                          unsigned long long* s_mv) {
    for (int j = 0; j < seg.n_td; j++) {
        const SegStep& st = seg.td[j];
        uint64_t S1 = 0, S2 = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint64_t v = 4 * lane + u;
            S1 += (uint64_t)hv[u] * v;
            S2 += (uint64_t)hv[u] * v * v;
        }
        S1 = wave_sum_u64_split(S1) + S1J;   // below 2^39 / 2^47 for n < 2^31
        S2 = wave_sum_u64_split(S2) + S2J;
        if (n == 0) {   // masked run: every sample of the row is set aside
            if (lane == 0) {
                s_lo[j] = 0;
                s_hi[j] = 255;
                s_r[j] = 0;
                s_mv[j] = 0;
            }
            continue;
        }
        int r;
        if (st.replace == RFIM_REPLACE_MEDIAN) {
            // lower median: the byte value holding rank floor((n-1)/2)
            const uint32_t mine = hv[0] + hv[1] + hv[2] + hv[3];
            uint32_t incl = mine;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(incl, o, 64);
                if (lane >= o) incl += t;
            }
            const uint64_t q = (n - 1) / 2;
            uint32_t before = incl - mine;
            int med = -1;
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (hv[u] > 0 && before <= q && q < (uint64_t)before + hv[u]) med = 4 * lane + u;
                before += hv[u];
            }
            const uint64_t mb = __ballot(med >= 0);
            r = __shfl(med, __ffsll((unsigned long long)mb) - 1, 64);
        } else {
            r = (int)rn_div_small(S1, n);
        }
        const u128 D = (u128)n * S2 - (u128)S1 * S1;
        int lo, hi;
        td_interval(n, S1, D, st.kx, &lo, &hi);
        uint32_t keepbits = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) keepbits |= (4 * lane + u >= lo && 4 * lane + u <= hi) ? 1u << u : 0u;
        if (nJ > 0 && (lo > jlo || hi < jhi)) return false;   // an untracked value may be cut
        uint32_t moved32 = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) moved32 += ((keepbits >> u) & 1) ? 0u : hv[u];
        const uint64_t moved = wave_sum_u32(moved32);   // at most n < 2^31
#pragma unroll
        for (int u = 0; u < 4; u++) if (!((keepbits >> u) & 1)) hv[u] = 0;
        if (seg.td_masked) {
            n -= moved;   // the cut samples leave the statistics of the run
        } else if (nJ > 0 && r >= jlo && r <= jhi) {
            nJ += moved;
            S1J += moved * (uint64_t)r;
            S2J += moved * (uint64_t)r * (uint64_t)r;
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++) if (4 * lane + u == r) hv[u] += (uint32_t)moved;
        }
        if (lane == 0) {
            s_lo[j] = lo <= hi ? lo : 1;   // kept values form [lo, hi]; empty as [1, 0]
            s_hi[j] = lo <= hi ? hi : 0;
            s_r[j] = r;
            s_mv[j] = moved;
        }
    }
    return true;
}

// LDS of one TD row group (one row per wave)
template <int R>
struct TdSharedR {
    uint32_t hist[R][kHistCopies * kHistPitch];
    int lo[R][kMaxSteps], hi[R][kMaxSteps], r[R][kMaxSteps];
    unsigned long long mv[R][kMaxSteps];
    int beam[R];
};
using TdShared = TdSharedR<kRowsPerWG>;

// Rows g0 .. g0 + R - 1 of a launch's row space (R waves), wave w on row
// g0 + w; rows at or past `row_end` are skipped.  Called by every thread of
// the work-group.
template <int R>
__device__ __attribute__((always_inline)) inline void td_row_group(const DevBeam* __restrict__ beams, int nbeams, int64_t g0, int64_t row_end,
                                    const Segment& seg, uint32_t* __restrict__ rec,
                                    unsigned long long* __restrict__ counts, int count_stride,
                                    TdSharedR<R>& sh) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t g = g0 + wave;
    // waves past the last row skip the row work but still reach the
    // work-group barrier of the flag counts below
    if (g < row_end) {
        unsigned long long* s_mv = sh.mv[wave];
        uint32_t* hist = sh.hist[wave];
        int* s_lo = sh.lo[wave];
        int* s_hi = sh.hi[wave];
        int* s_r = sh.r[wave];
        const int b = find_beam_by_row(beams, nbeams, g);
        const DevBeam& bm = beams[b];
        const int64_t c = g - bm.row0;
        const int64_t T = bm.T;
        const uint64_t n = (uint64_t)T;
        const uint8_t* row = (const uint8_t*)bm.in + c * bm.stride;
        uint32_t* h = hist + (lane & (kHistCopies - 1)) * kHistPitch;

        auto clear_hist = [&] {
            for (int i = lane; i < kHistCopies * kHistPitch; i += 64) hist[i] = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        };
        // lane l owns the byte values 4l .. 4l+3
        auto read_hist = [&](uint32_t hv[4]) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int u = 0; u < 4; u++) {
                uint32_t t = 0;
#pragma unroll
                for (int cp = 0; cp < kHistCopies; cp++) t += hist[cp * kHistPitch + 4 * lane + u];
                hv[u] = t;
            }
        };

        // Measured alternatives, all slower than one pass with a full histogram:
        // exact S1, S2 by dot4 with a histogram of only the bytes outside a band
        // around the row's bulk (a band from the row's first 2 KB; a band from the
        // first cut in a second pass; or the row held in VGPRs with the dwords
        // holding out-of-band bytes compacted into an LDS queue first).  The
        // first two leave some out-of-band byte in nearly every wave-wide dword;
        // the last costs more occupancy than the atomics it saves.
        {
            // every value tracked: the row's full histogram
            clear_hist();
            row_pass(row, T, lane, [&](uint32_t x) { hist4(h, x); }, [&](uint32_t x) { atomicAdd(&h[x], 1u); });
            uint32_t hv[4];
            read_hist(hv);
            td_decide(seg, n, hv, 0, 0, 0, 1, 0, lane, s_lo, s_hi, s_r, s_mv);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();

        // composite record of the run, one u32 per step:
        //   [7:0] L_j, [15:8] H_j  -- nested interval: a sample stays untouched
        //                             through step j iff L_j <= x <= H_j
        //   [23:16] value a sample first cut at step j ends with
        //   [31:24] flag bits it collects (step j and any later step that cuts
        //           the replacement value; step j alone in a masked run)
        if (lane < seg.n_td) {
            const int j = lane;
            int L = 0, H = 255;
            for (int k = 0; k <= j; k++) {
                L = max(L, s_lo[k]);
                H = min(H, s_hi[k]);
            }
            int val = s_r[j];
            uint32_t f = seg.td[j].bit >= 0 ? (1u << seg.td[j].bit) : 0u;
            // a masked run never tests a sample again once it is cut
            for (int k = j + 1; k < seg.n_td && !seg.td_masked; k++) {
                if (val < s_lo[k] || val > s_hi[k]) {
                    val = s_r[k];
                    if (seg.td[k].bit >= 0) f |= 1u << seg.td[k].bit;
                }
            }
            if (L > H) {  // empty interval: every value is cut
                L = 1;
                H = 0;
            }
            rec[g * seg.n_td + j] = (uint32_t)L | ((uint32_t)H << 8) | ((uint32_t)val << 16) | (f << 24);
        }
        if (lane == 0) sh.beam[wave] = bm.cidx;
    }   // g < row_end

    // Flag counts.  Every row of a beam adds to the same few counters, and
    // one atomic per row and step left the kernel waiting on those atomics
    // for most of its time; so the work-group's rows are summed in LDS first
    // and each step's sum goes out with one atomic per beam.
    if (counts) {
        __syncthreads();
        const int j = threadIdx.x;
        if (j < seg.n_td) {
            const int nw = (int)min((int64_t)R, row_end - g0);
            int cb = sh.beam[0];
            unsigned long long sum = 0;
            for (int w = 0; w < nw; w++) {
                if (sh.beam[w] != cb) {
                    if (sum) atomicAdd(&counts[(int64_t)cb * count_stride + seg.td[j].ci], sum);
                    cb = sh.beam[w];
                    sum = 0;
                }
                sum += sh.mv[w][j];
            }
            if (sum) atomicAdd(&counts[(int64_t)cb * count_stride + seg.td[j].ci], sum);
        }
    }
}


// R rows (waves) per work-group, a tuning parameter
template <int R>
__global__ __launch_bounds__(64 * R) void k_td_rows_u8(const DevBeam* __restrict__ beams,
                                                       int nbeams, int64_t total_rows, Segment seg,
                                                       uint32_t* __restrict__ rec,
                                                       unsigned long long* __restrict__ counts,
                                                       int count_stride) {
    __shared__ TdSharedR<R> sh;
    td_row_group<R>(beams, nbeams, (int64_t)blockIdx.x * R, total_rows, seg, rec, counts, count_stride, sh);
}

namespace {

// group of G consecutive lanes (G a power of two <= 64): sum of u64 values
__device__ inline uint64_t group_sum_u64(uint64_t v, int G) {
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

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

// Full TD composite map of one byte (records r[0..m) of its row)
__device__ inline uint32_t td_map_byte(uint32_t x, const uint32_t* __restrict__ r, int m,
                                       uint32_t* fl) {
    uint32_t out = x, f = 0;
    for (int j = m - 1; j >= 0; j--) {
        const uint32_t e = r[j];
        const uint32_t L = e & 255u, H = (e >> 8) & 255u;
        if (x < L || x > H) {
            out = (e >> 16) & 255u;
            f = e >> 24;
        }
    }
    *fl = f;
    return out;
}

// lower median (rank floor((n-1)/2)) of the n bytes at p: the largest value v
// with #{x < v} <= rank, found bit by bit
__device__ inline uint32_t lds_lower_median_u8(const uint8_t* p, int64_t n) {
    const int64_t rank = (n - 1) / 2;
    uint32_t prefix = 0;
    for (int bit = 7; bit >= 0; bit--) {
        const uint32_t cand = prefix | (1u << bit);
        int64_t below = 0;
        if ((n & 3) == 0 && (((uintptr_t)p) & 3) == 0) {
            const uint32_t kc = klo_of(cand);
            for (int64_t i = 0; i < n; i += 4) {
                const uint32_t x = *(const uint32_t*)(p + i);
                // bytes >= cand have bit 15 of their lane set after adding kc
                const uint32_t e = (x & 0x00FF00FFu) + kc, o = ((x >> 8) & 0x00FF00FFu) + kc;
                below += 4 - (int64_t)__popc((e & 0x80008000u) | ((o & 0x80008000u) >> 1));
            }
        } else {
            for (int64_t i = 0; i < n; i++) below += p[i] < cand;
        }
        if (below <= rank) prefix = cand;
    }
    return prefix;
}

constexpr int kExcCap = 768;  // TD exception worklist entries per work-group

}  // namespace

// ---------------------------------------------------------------------------
// TD apply + FD steps on an LDS tile, one work-group per (beam, time tile)
// ---------------------------------------------------------------------------
namespace {

struct TileCtx {
    const uint8_t* in;
    uint8_t* out;
    uint8_t* flags;
    const uint32_t* rec;   // this beam's TD records, [row][n_td]
    int64_t C, T, stride, t0;
    int Tt, Cp, tw, tw_log, n_td;
    int64_t nq4;
};

// the 4 rows c0..c0+3 of dword w of the tile; rows past C read as 0
template <bool INTERIOR>
__device__ inline void load_quad(const TileCtx& k, const uint8_t* base, int64_t c0, int w, uint32_t x[4]) {
    const int64_t t = k.t0 + 4 * w;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (INTERIOR) {
            const int64_t c = c0 + i < k.C ? c0 + i : k.C - 1;
            const uint32_t v = *(const uint32_t*)(base + c * k.stride + t);
            x[i] = c0 + i < k.C ? v : 0u;
        } else {
            x[i] = (c0 + i < k.C) ? load4(base + (c0 + i) * k.stride + t, t, k.T) : 0u;
        }
    }
}

template <bool INTERIOR>
__device__ inline void store_quad(const TileCtx& k, uint8_t* base, int64_t c0, int w, const uint32_t x[4]) {
    const int64_t t = k.t0 + 4 * w;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (c0 + i >= k.C) continue;
        if (INTERIOR)
            *(uint32_t*)(base + (c0 + i) * k.stride + t) = x[i];
        else
            store4(base + (c0 + i) * k.stride + t, x[i], t, k.T);
    }
}

// bytes of the dword at sample t that lie inside the batch
__device__ inline uint32_t valid_bytes(int64_t t, int64_t T) {
    return t + 3 < T ? 0xFFFFFFFFu : (t >= T ? 0u : (0xFFFFFFFFu >> (8 * (4 - (T - t)))));
}

// TD composite map of one dword of row c (4 samples); *fv gets the flag bytes
__device__ inline uint32_t td_map_dword(const TileCtx& k, int64_t c, uint32_t xv, uint32_t* fv) {
    const uint32_t* rp = k.rec + c * k.n_td;
    uint32_t nv = 0, f4 = 0;
    for (int j = 0; j < 4; j++) {
        uint32_t f;
        nv |= td_map_byte((xv >> (8 * j)) & 255u, rp, k.n_td, &f) << (8 * j);
        f4 |= f << (8 * j);
    }
    *fv = f4;
    return nv;
}

// Phase 1 body for one row-quad task: 4 rows in, TD fast check (exceptions
// to the worklist), 4x4 transpose, LDS tile [Tt][Cp]
template <bool INTERIOR>
__device__ inline void tile_load_task(const TileCtx& k, int64_t idx, uint8_t* tile, uint8_t* ftile,
                                      bool want_flags, bool or_flags, uint32_t* exc_pos,
                                      uint32_t* exc_n) {
    const int64_t q4 = idx >> k.tw_log;
    const int w = (int)(idx & (k.tw - 1));
    const int64_t c0 = 4 * q4;
    uint32_t x[4], y[4], tf[4] = {0u, 0u, 0u, 0u};
    load_quad<INTERIOR>(k, k.in, c0, w, x);
    if (k.n_td > 0) {
        const uint32_t valid = INTERIOR ? 0xFFFFFFFFu : valid_bytes(k.t0 + 4 * w, k.T);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int64_t c = c0 + i < k.C ? c0 + i : k.C - 1;
            const uint32_t e = k.rec[c * k.n_td + (k.n_td - 1)];
            uint32_t m = outside_mask(x[i], klo_of(e & 255u), khi_of((e >> 8) & 255u)) & valid;
            if (c0 + i >= k.C) m = 0;
            if (m) {
                const uint32_t slot = atomicAdd(exc_n, 1u);
                if (slot < (uint32_t)kExcCap) {
                    exc_pos[slot] = ((uint32_t)(c0 + i) << 8) | (uint32_t)w;
                } else {   // worklist full: map here
                    x[i] = td_map_dword(k, c, x[i], &tf[i]);
                    tf[i] &= valid;
                }
            }
        }
    }
    transpose4(x, y);
#pragma unroll
    for (int j = 0; j < 4; j++) *(uint32_t*)(tile + (size_t)(4 * w + j) * k.Cp + c0) = y[j];
    if (want_flags) {
        uint32_t fx[4] = {0u, 0u, 0u, 0u}, fy[4];
        if (or_flags) load_quad<INTERIOR>(k, k.flags, c0, w, fx);
#pragma unroll
        for (int i = 0; i < 4; i++) fx[i] |= tf[i];
        transpose4(fx, fy);
#pragma unroll
        for (int j = 0; j < 4; j++) *(uint32_t*)(ftile + (size_t)(4 * w + j) * k.Cp + c0) = fy[j];
    }
}

// Phase 1 for a 4-row x 16-sample task of an interior tile whose rows are
// dword aligned, in two halves so that a thread can issue the loads of all
// its tasks before it waits for any: fetch16 loads the 4 rows (one 16-byte
// load each) and their last TD records, load_task16 does the rest.
// The loads of NB tasks (idx = b0 + u * kBlock): every offset is computed
// first, then every load is issued, unconditionally -- a task past n (the
// caller ignores it) reads task n-1, and with no TD step the record read is
// entry 0 -- so no branch splits the batch and it is in flight at once.
// Offsets are 32-bit (the wide path is taken for beams below 4 GB only).
// Rows past C read row C-1 here; load_task16 zeroes them.
template <int NB>
__device__ inline void fetch16_batch(const TileCtx& k, int64_t b0, int64_t n, uint4 (&x)[NB][4],
                                     uint32_t (&e)[NB][4]) {
    const int tq_log = k.tw_log - 2;              // 16-sample chunks per tile row
    const uint32_t cmax = (uint32_t)k.C - 1u;
    const bool td = k.n_td > 0;
    uint32_t xo[NB][4], eo[NB][4];
#pragma unroll
    for (int u = 0; u < NB; u++) {
        const int64_t idx = min(b0 + (int64_t)u * kBlock, n - 1);
        const uint32_t c0 = 4u * (uint32_t)(idx >> tq_log);
        const uint32_t col = (uint32_t)k.t0 + 16u * ((uint32_t)idx & ((1u << tq_log) - 1u));
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t c = min(c0 + (uint32_t)i, cmax);
            xo[u][i] = c * (uint32_t)k.stride + col;
            eo[u][i] = td ? c * (uint32_t)k.n_td + (uint32_t)(k.n_td - 1) : 0u;
        }
    }
#pragma unroll
    for (int u = 0; u < NB; u++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            x[u][i] = ld_global<uint4>(k.in + xo[u][i]);
            e[u][i] = ld_global<uint32_t>(k.rec + eo[u][i]);
        }
}

// Bit 4*i + j set when dword j of row i of the task holds a byte that a TD
// step of the run cuts (outside the row's final nested interval).
__device__ inline uint32_t exc_bits16(const TileCtx& k, int64_t idx, const uint4 x[4], const uint32_t e[4]) {
    if (k.n_td <= 0) return 0u;
    const int tq_log = k.tw_log - 2;
    const int64_t c0 = 4 * (idx >> tq_log);
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (c0 + i >= k.C) continue;
        const uint32_t klo = klo_of(e[i] & 255u), khi = khi_of((e[i] >> 8) & 255u);
        const uint32_t* xi = &x[i].x;
#pragma unroll
        for (int j = 0; j < 4; j++) bits |= (outside_mask(xi[j], klo, khi) != 0u ? 1u : 0u) << (4 * i + j);
    }
    return bits;
}

// The rest of a task: its exception dwords go to the worklist from *slot on
// (mapped here once the worklist is full), then the 4x4 transposes into LDS.
__device__ inline void load_task16(const TileCtx& k, int64_t idx, uint4 x[4], uint32_t bits, uint32_t* slot,
                                   uint8_t* tile, uint8_t* ftile, bool want_flags, bool or_flags,
                                   uint32_t* exc_pos) {
    const int tq_log = k.tw_log - 2;
    const int64_t q4 = idx >> tq_log;
    const int w16 = (int)(idx & ((1 << tq_log) - 1));
    const int64_t c0 = 4 * q4;
#pragma unroll
    for (int i = 0; i < 4; i++)
        if (c0 + i >= k.C) x[i] = make_uint4(0u, 0u, 0u, 0u);   // rows past C
    uint32_t tf[4][4] = {};   // TD flag bytes of dwords mapped here (worklist full)
    uint32_t ovf = 0;         // exception dwords past the worklist's end
    while (bits) {
        const int b = __ffs(bits) - 1;
        bits &= bits - 1;
        const uint32_t sl = (*slot)++;
        if (sl < (uint32_t)kExcCap)
            exc_pos[sl] = ((uint32_t)(c0 + (b >> 2)) << 8) | (uint32_t)(4 * w16 + (b & 3));
        else
            ovf |= 1u << b;
    }
    if (ovf) {   // worklist full: map those here (constant indices keep x in VGPRs)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            uint32_t* xi = &x[i].x;
#pragma unroll
            for (int j = 0; j < 4; j++)
                if ((ovf >> (4 * i + j)) & 1u) xi[j] = td_map_dword(k, c0 + i, xi[j], &tf[i][j]);
        }
    }
    uint32_t a[4], y[4];
#define RFIM_T16(F, J)                                                                      \
    a[0] = x[0].F; a[1] = x[1].F; a[2] = x[2].F; a[3] = x[3].F;                             \
    transpose4(a, y);                                                                       \
    for (int jj = 0; jj < 4; jj++)                                                          \
        *(uint32_t*)(tile + (size_t)(16 * w16 + 4 * (J) + jj) * k.Cp + c0) = y[jj];
    RFIM_T16(x, 0) RFIM_T16(y, 1) RFIM_T16(z, 2) RFIM_T16(w, 3)
#undef RFIM_T16
    if (want_flags) {
        for (int j = 0; j < 4; j++) {
            uint32_t fx[4] = {0u, 0u, 0u, 0u}, fy[4];
            if (or_flags) load_quad<true>(k, k.flags, c0, 4 * w16 + j, fx);
            for (int i = 0; i < 4; i++) fx[i] |= tf[i][j];
            transpose4(fx, fy);
            for (int jj = 0; jj < 4; jj++)
                *(uint32_t*)(ftile + (size_t)(16 * w16 + 4 * j + jj) * k.Cp + c0) = fy[jj];
        }
    }
}

// Phase 3 body for a 4-row x 16-sample task of an interior tile
__device__ inline void tile_store_task16(const TileCtx& k, int64_t idx, const uint8_t* tile,
                                         const uint8_t* ftile, bool want_flags) {
    const int tq_log = k.tw_log - 2;
    const int64_t q4 = idx >> tq_log;
    const int w16 = (int)(idx & ((1 << tq_log) - 1));
    const int64_t c0 = 4 * q4;
    uint4 x[4];
    uint32_t a[4], y[4];
#define RFIM_S16(F, J)                                                                      \
    for (int jj = 0; jj < 4; jj++)                                                          \
        y[jj] = *(const uint32_t*)(tile + (size_t)(16 * w16 + 4 * (J) + jj) * k.Cp + c0);   \
    transpose4(y, a);                                                                       \
    x[0].F = a[0]; x[1].F = a[1]; x[2].F = a[2]; x[3].F = a[3];
    RFIM_S16(x, 0) RFIM_S16(y, 1) RFIM_S16(z, 2) RFIM_S16(w, 3)
#undef RFIM_S16
    const uint32_t col = (uint32_t)k.t0 + 16u * (uint32_t)w16;   // 32-bit offsets: beams below 4 GB
#pragma unroll
    for (int i = 0; i < 4; i++)
        if (c0 + i < k.C) st_global<uint4>(k.out + ((uint32_t)(c0 + i) * (uint32_t)k.stride + col), x[i]);
    if (want_flags) {
        for (int j = 0; j < 4; j++) {
            uint32_t fy[4], fx[4];
            for (int jj = 0; jj < 4; jj++)
                fy[jj] = *(const uint32_t*)(ftile + (size_t)(16 * w16 + 4 * j + jj) * k.Cp + c0);
            transpose4(fy, fx);
            store_quad<true>(k, k.flags, c0, 4 * w16 + j, fx);
        }
    }
}

// Phase 3 body: transpose back and write 4 rows (and flags)
template <bool INTERIOR>
__device__ inline void tile_store_task(const TileCtx& k, int64_t idx, const uint8_t* tile,
                                       const uint8_t* ftile, bool want_flags) {
    const int64_t q4 = idx >> k.tw_log;
    const int w = (int)(idx & (k.tw - 1));
    const int64_t c0 = 4 * q4;
    uint32_t y[4], x[4];
#pragma unroll
    for (int j = 0; j < 4; j++) y[j] = *(const uint32_t*)(tile + (size_t)(4 * w + j) * k.Cp + c0);
    transpose4(y, x);
    store_quad<INTERIOR>(k, k.out, c0, w, x);
    if (want_flags) {
#pragma unroll
        for (int j = 0; j < 4; j++) y[j] = *(const uint32_t*)(ftile + (size_t)(4 * w + j) * k.Cp + c0);
        transpose4(y, x);
        store_quad<INTERIOR>(k, k.flags, c0, w, x);
    }
}


__device__ inline void put_dword_transposed(uint8_t* tile, const TileCtx& k, int64_t c, int w, uint32_t v) {
#pragma unroll
    for (int j = 0; j < 4; j++) tile[(size_t)(4 * w + j) * k.Cp + c] = (uint8_t)(v >> (8 * j));
}

__device__ inline void or_dword_transposed(uint8_t* tile, const TileCtx& k, int64_t c, int w, uint32_t v) {
#pragma unroll
    for (int j = 0; j < 4; j++) tile[(size_t)(4 * w + j) * k.Cp + c] |= (uint8_t)(v >> (8 * j));
}

}  // namespace

// Phase 2: every FD step of the run on the LDS tile; G = 256/Tt consecutive
// lanes own one time sample (column).  VEC: every lane's share of a bin is a
// multiple of 16 bytes at a 16-byte boundary (the host checks), so bins are
// read with 16-byte LDS loads and summed with dot4; otherwise bytes.
template <bool VEC>
__device__ inline void fd_steps(const TileCtx& k, const Segment& seg, uint8_t* tile, uint8_t* ftile,
                                bool want_flags, bool count, unsigned long long* s_cnt) {
    const int tid = threadIdx.x;
    const int Tt = k.Tt;
    const int G = kBlock / Tt;
    const int tl = tid / G, q = tid % G;
    const bool valid = k.t0 + tl < k.T;
    const int64_t C = k.C;
    uint8_t* colp = tile + (size_t)tl * k.Cp;
    uint8_t* fcol = ftile + (size_t)tl * k.Cp;
    for (int s = 0; s < seg.n_fd; s++) {
        const SegStep& st = seg.fd[s];
        const int64_t B = st.bin == 0 ? C : st.bin;
        const int nb = (int)(C / B);
        const int bshift = (B & (B - 1)) == 0 ? __ffsll((unsigned long long)B) - 1 : -1;
        // lanes per bin: bins split over lanes when there are fewer bins than
        // lanes (and, for VEC, the split stays 16-byte aligned)
        int lpb = 1;
        if (nb < G && (G % nb) == 0 && (B % ((VEC ? 16 : 1) * (G / nb))) == 0) lpb = G / nb;
        const int64_t chunk = B / lpb;
        const int first = lpb > 1 ? q / lpb : q;
        const int bstep = lpb > 1 ? nb : G;     // lpb > 1: one bin per lane
        const int64_t coff = lpb > 1 ? (int64_t)(q % lpb) * chunk : 0;
        // statistics: sum over bins of B*(B*Q_b - S_b^2) = sum of Z_c^2
        u128 sz2 = 0;
        for (int bb = first; bb < nb; bb += bstep) {
            const uint8_t* p = colp + (int64_t)bb * B + coff;
            uint64_t S = 0, Q = 0;
            if (VEC) {
                for (int64_t i0 = 0; i0 < chunk; i0 += 65536) {
                    uint32_t s32 = 0, q32 = 0;
                    const int64_t i1 = min(chunk, i0 + 65536);
                    for (int64_t i = i0; i < i1; i += 16) {
                        const uint4 x = *(const uint4*)(p + i);
                        s32 = __builtin_amdgcn_udot4(x.x, 0x01010101u, s32, false);
                        s32 = __builtin_amdgcn_udot4(x.y, 0x01010101u, s32, false);
                        s32 = __builtin_amdgcn_udot4(x.z, 0x01010101u, s32, false);
                        s32 = __builtin_amdgcn_udot4(x.w, 0x01010101u, s32, false);
                        q32 = __builtin_amdgcn_udot4(x.x, x.x, q32, false);
                        q32 = __builtin_amdgcn_udot4(x.y, x.y, q32, false);
                        q32 = __builtin_amdgcn_udot4(x.z, x.z, q32, false);
                        q32 = __builtin_amdgcn_udot4(x.w, x.w, q32, false);
                    }
                    S += s32;
                    Q += q32;
                }
            } else {
                for (int64_t i = 0; i < chunk; i++) {
                    const uint32_t x = p[i];
                    S += x;
                    Q += x * x;
                }
            }
            if (lpb > 1) {
                S = group_sum_u64(S, lpb);   // lanes of one bin are adjacent
                Q = group_sum_u64(Q, lpb);
                if (q % lpb) continue;       // count each bin once
            }
            sz2 += (u128)B * ((u128)B * Q - (u128)S * S);
        }
        sz2 = group_sum_u128(sz2, G);
        const uint64_t z = fd_zthr(sz2, C, st.kx, (uint64_t)B * 255u);
        const uint32_t fbit = st.bit >= 0 ? (1u << st.bit) * 0x01010101u : 0u;
        uint64_t nflag = 0;
        for (int bb = first; bb < nb; bb += bstep) {
            uint8_t* p = colp + (int64_t)bb * B + coff;
            uint8_t* fp = fcol + (int64_t)bb * B + coff;
            // bin sum again (cheap) for the cut and the replacement
            uint64_t S = 0;
            if (VEC) {
                uint32_t s32 = 0;
                for (int64_t i = 0; i < chunk; i += 16) {
                    const uint4 x = *(const uint4*)(p + i);
                    s32 = __builtin_amdgcn_udot4(x.x, 0x01010101u, s32, false);
                    s32 = __builtin_amdgcn_udot4(x.y, 0x01010101u, s32, false);
                    s32 = __builtin_amdgcn_udot4(x.z, 0x01010101u, s32, false);
                    s32 = __builtin_amdgcn_udot4(x.w, 0x01010101u, s32, false);
                }
                S = s32;
            } else {
                for (int64_t i = 0; i < chunk; i++) S += p[i];
            }
            if (lpb > 1) S = group_sum_u64(S, lpb);
            // kept: |B*x - S| <= z  <=>  ceil((S - z)/B) <= x <= floor((S + z)/B)
            int64_t lo, hi;
            if (bshift >= 0) {
                lo = -((int64_t)(z - S) >> bshift);          // ceil((S - z) / 2^bshift)
                hi = (int64_t)(S + z) >> bshift;
            } else {
                lo = ceil_div((int64_t)S - (int64_t)z, B);
                hi = floor_div((int64_t)S + (int64_t)z, B);
            }
            lo = lo < 0 ? 0 : lo;
            hi = hi > 255 ? 255 : hi;
            uint32_t klo = klo_of(1), khi = khi_of(0);   // empty interval
            if (lo <= hi) {
                klo = klo_of((uint32_t)lo);
                khi = khi_of((uint32_t)hi);
            }
            uint32_t r;
            if (st.replace == RFIM_REPLACE_MEDIAN) {
                // needed only when the bin has an outlier in this column
                uint32_t any = 0;
                if (VEC) {
                    for (int64_t i = 0; i < chunk; i += 4) any |= outside_mask(*(const uint32_t*)(p + i), klo, khi);
                } else {
                    for (int64_t i = 0; i < chunk; i++) any |= ((int64_t)p[i] < lo || (int64_t)p[i] > hi);
                }
                if (lpb > 1) any = (uint32_t)group_sum_u64(any ? 1u : 0u, lpb);
                if (!any) continue;
                // every lane of a split bin computes the same median
                r = lds_lower_median_u8(colp + (int64_t)bb * B, B);
            } else if (bshift >= 0) {
                const uint64_t qv = S >> bshift, rem = S & (B - 1);
                r = (uint32_t)(qv + ((2 * rem > (uint64_t)B || (2 * rem == (uint64_t)B && (qv & 1))) ? 1 : 0));
            } else {
                r = (uint32_t)rn_div_u64(S, (uint64_t)B);
            }
            const uint32_t rrep = r * 0x01010101u;
            if (VEC) {
                for (int64_t i = 0; i < chunk; i += 16) {
                    uint4 x = *(const uint4*)(p + i);
                    const uint32_t m0 = outside_mask(x.x, klo, khi), m1 = outside_mask(x.y, klo, khi);
                    const uint32_t m2 = outside_mask(x.z, klo, khi), m3 = outside_mask(x.w, klo, khi);
                    if (m0 | m1 | m2 | m3) {
                        x.x = (x.x & ~m0) | (rrep & m0);
                        x.y = (x.y & ~m1) | (rrep & m1);
                        x.z = (x.z & ~m2) | (rrep & m2);
                        x.w = (x.w & ~m3) | (rrep & m3);
                        *(uint4*)(p + i) = x;
                        if (want_flags) {
                            uint4 f = *(const uint4*)(fp + i);
                            f.x |= m0 & fbit;
                            f.y |= m1 & fbit;
                            f.z |= m2 & fbit;
                            f.w |= m3 & fbit;
                            *(uint4*)(fp + i) = f;
                        }
                        nflag += (__popc(m0) + __popc(m1) + __popc(m2) + __popc(m3)) >> 3;
                    }
                }
            } else {
                for (int64_t i = 0; i < chunk; i++) {
                    if ((int64_t)p[i] < lo || (int64_t)p[i] > hi) {
                        p[i] = (uint8_t)r;
                        if (want_flags && st.bit >= 0) fp[i] |= (uint8_t)(1u << st.bit);
                        nflag++;
                    }
                }
            }
        }
        if (count) {   // one LDS add per wave (all lanes are here)
            const uint64_t tot = wave_sum_u64_split(valid ? nflag : 0u);
            if ((tid & 63) == 0 && tot) atomicAdd(&s_cnt[s], (unsigned long long)tot);
        }
    }
}

// Sum over groups of G consecutive lanes (G = 4, 8 or 16) with DPP: quad
// swaps, then the half-row and row mirrors; every lane gets its group's sum.
template <int G>
__device__ inline uint32_t group_sum_dpp(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);    // quad_perm 1,0,3,2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);    // quad_perm 2,3,0,1
    if (G >= 8) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false);  // row_half_mirror
    if (G >= 16) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false); // row_mirror
    return v;
}


// kept byte values of a 32-channel bin with sum S under the cut |32 x - S| <= z:
// ceil((S - z)/32) <= x <= floor((S + z)/32), as outside_mask constants
__device__ inline void bin32_bounds(uint32_t S, uint32_t z, uint32_t* klo, uint32_t* khi) {
    const int lo = -(((int)z - (int)S) >> 5);
    const int hi = (int)((S + z) >> 5);
    const int lc = lo < 0 ? 0 : lo, hc = hi > 255 ? 255 : hi;
    *klo = klo_of(1);   // empty interval
    *khi = khi_of(0);
    if (lc <= hc) {
        *klo = klo_of((uint32_t)lc);
        *khi = khi_of((uint32_t)hc);
    }
}

// lower median (rank 15) of the 32 bytes of a bin held in registers, by a
// bitwise search: per candidate, the bytes >= it are counted 16 bits at a time
__device__ inline uint32_t lower_median32(const uint4& a, const uint4& b) {
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t e[8], o[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        e[i] = w[i] & 0x00FF00FFu;
        o[i] = (w[i] >> 8) & 0x00FF00FFu;
    }
    uint32_t prefix = 0;
#pragma unroll
    for (int bit = 7; bit >= 0; bit--) {
        const uint32_t cand = prefix | (1u << bit);
        const uint32_t kc = klo_of(cand);   // a lane >= cand gets bit 15 set
        uint32_t ge = 0;
#pragma unroll
        for (int i = 0; i < 8; i++)
            ge += (uint32_t)__popc(((e[i] + kc) & 0x80008000u) | (((o[i] + kc) & 0x80008000u) >> 1));
        if (32u - ge <= 15u) prefix = cand;   // at most 15 bytes below cand
    }
    return prefix;
}

// replaces the bytes of the bin at `off` that the masks select by r (flags
// too); returns how many were replaced
__device__ inline uint32_t bin32_replace(uint8_t* tile, uint8_t* ftile, uint32_t off, uint4 a, uint4 b,
                                         const uint32_t m[8], uint32_t r, uint32_t fbit, bool want_flags) {
    const uint32_t rr = r * 0x01010101u;
    a.x = (a.x & ~m[0]) | (rr & m[0]);
    a.y = (a.y & ~m[1]) | (rr & m[1]);
    a.z = (a.z & ~m[2]) | (rr & m[2]);
    a.w = (a.w & ~m[3]) | (rr & m[3]);
    b.x = (b.x & ~m[4]) | (rr & m[4]);
    b.y = (b.y & ~m[5]) | (rr & m[5]);
    b.z = (b.z & ~m[6]) | (rr & m[6]);
    b.w = (b.w & ~m[7]) | (rr & m[7]);
    *(uint4*)(tile + off) = a;
    *(uint4*)(tile + off + 16) = b;
    if (want_flags) {
        uint4 fa = *(const uint4*)(ftile + off);
        uint4 fb = *(const uint4*)(ftile + off + 16);
        fa.x |= m[0] & fbit; fa.y |= m[1] & fbit; fa.z |= m[2] & fbit; fa.w |= m[3] & fbit;
        fb.x |= m[4] & fbit; fb.y |= m[5] & fbit; fb.z |= m[6] & fbit; fb.w |= m[7] & fbit;
        *(uint4*)(ftile + off) = fa;
        *(uint4*)(ftile + off + 16) = fb;
    }
    uint32_t n = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) n += (uint32_t)__popc(m[i]);
    return n >> 3;
}

__device__ inline void bin32_masks(const uint4& a, const uint4& b, uint32_t klo, uint32_t khi, uint32_t m[8]) {
    m[0] = outside_mask(a.x, klo, khi);
    m[1] = outside_mask(a.y, klo, khi);
    m[2] = outside_mask(a.z, klo, khi);
    m[3] = outside_mask(a.w, klo, khi);
    m[4] = outside_mask(b.x, klo, khi);
    m[5] = outside_mask(b.y, klo, khi);
    m[6] = outside_mask(b.z, klo, khi);
    m[7] = outside_mask(b.w, klo, khi);
}

// FD steps for bins of 32 channels: G lanes per time sample, lane q owns bins
// q, q+G, ... (at most kB32MaxBins).  Per bin: S = sum x <= 8160 and
// Q = sum x^2 <= 2.1e6, and sum over the bin of Z^2 = 32*(32*Q - S^2) < 2^30,
// so everything is 32-bit until the column total.  Median steps: bins with a
// cut are listed (list, *list_n, at most cap entries) and their medians are
// then taken by all lanes together, since a lane with such a bin would
// otherwise hold its whole wave; s_z keeps each time sample's threshold.
// Every thread of the work-group calls this (it has barriers).
template <int G>
__device__ inline void fd_steps_b32(const TileCtx& k, const Segment& seg, uint8_t* tile, uint8_t* ftile,
                                    bool want_flags, bool count, unsigned long long* s_cnt, uint32_t* list,
                                    uint32_t* list_n, uint32_t cap, uint32_t* s_z) {
    const int tid = threadIdx.x;
    const int tl = tid / G, q = tid % G;
    const bool valid = k.t0 + tl < k.T;
    const uint32_t C = (uint32_t)k.C;
    const int nb = (int)(C >> 5);
    const uint32_t col = (uint32_t)tl * (uint32_t)k.Cp;
    for (int s = 0; s < seg.n_fd; s++) {
        const SegStep& st = seg.fd[s];
        const bool med = st.replace == RFIM_REPLACE_MEDIAN;
        if (med) {
            if (tid == 0) *list_n = 0;
            __syncthreads();
        }
        uint32_t Sb[kB32MaxBins];
        uint32_t zlo = 0, zhi = 0;   // per-lane sum of Z^2 as 24-bit slices
#pragma unroll
        for (int i = 0; i < kB32MaxBins; i++) {
            const int bb = q + i * G;
            Sb[i] = 0;
            if (bb < nb) {
                const uint32_t off = col + (uint32_t)bb * 32u;
                const uint4 a = *(const uint4*)(tile + off);
                const uint4 b = *(const uint4*)(tile + off + 16);
                uint32_t S = __builtin_amdgcn_udot4(a.x, 0x01010101u, 0u, false);
                S = __builtin_amdgcn_udot4(a.y, 0x01010101u, S, false);
                S = __builtin_amdgcn_udot4(a.z, 0x01010101u, S, false);
                S = __builtin_amdgcn_udot4(a.w, 0x01010101u, S, false);
                S = __builtin_amdgcn_udot4(b.x, 0x01010101u, S, false);
                S = __builtin_amdgcn_udot4(b.y, 0x01010101u, S, false);
                S = __builtin_amdgcn_udot4(b.z, 0x01010101u, S, false);
                S = __builtin_amdgcn_udot4(b.w, 0x01010101u, S, false);
                uint32_t Q = __builtin_amdgcn_udot4(a.x, a.x, 0u, false);
                Q = __builtin_amdgcn_udot4(a.y, a.y, Q, false);
                Q = __builtin_amdgcn_udot4(a.z, a.z, Q, false);
                Q = __builtin_amdgcn_udot4(a.w, a.w, Q, false);
                Q = __builtin_amdgcn_udot4(b.x, b.x, Q, false);
                Q = __builtin_amdgcn_udot4(b.y, b.y, Q, false);
                Q = __builtin_amdgcn_udot4(b.z, b.z, Q, false);
                Q = __builtin_amdgcn_udot4(b.w, b.w, Q, false);
                Sb[i] = S;
                const uint32_t zb = 32u * (32u * Q - S * S);
                zlo += zb & 0xFFFFFFu;
                zhi += zb >> 24;
            }
        }
        zlo = group_sum_dpp<G>(zlo);
        zhi = group_sum_dpp<G>(zhi);
        const uint64_t sz2 = (uint64_t)zlo + ((uint64_t)zhi << 24);
        const uint32_t z = fd_zthr_small(sz2, C, st.kx, 32u * 255u);
        if (med && q == 0) s_z[tl] = z;
        const uint32_t fbit = st.bit >= 0 ? (1u << st.bit) * 0x01010101u : 0u;
        uint32_t nflag = 0;
        const int lane = tid & 63;
        if (!med) {
#pragma unroll
            for (int i = 0; i < kB32MaxBins; i++) {
                const int bb = q + i * G;
                if (bb >= nb) continue;
                const uint32_t S = Sb[i];
                uint32_t klo, khi;
                bin32_bounds(S, z, &klo, &khi);
                const uint32_t off = col + (uint32_t)bb * 32u;
                const uint4 a = *(const uint4*)(tile + off);
                const uint4 b = *(const uint4*)(tile + off + 16);
                uint32_t m[8];
                bin32_masks(a, b, klo, khi, m);
                if (m[0] | m[1] | m[2] | m[3] | m[4] | m[5] | m[6] | m[7]) {
                    const uint32_t qv = S >> 5, rem = S & 31u;
                    const uint32_t r = qv + ((rem > 16u || (rem == 16u && (qv & 1u))) ? 1u : 0u);
                    nflag += bin32_replace(tile, ftile, off, a, b, m, r, fbit, want_flags);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < kB32MaxBins; i++) {
                const int bb = q + i * G;
                const uint32_t off = col + (uint32_t)bb * 32u;
                uint4 a = make_uint4(0u, 0u, 0u, 0u), b = a;
                uint32_t m[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
                if (bb < nb) {
                    uint32_t klo, khi;
                    bin32_bounds(Sb[i], z, &klo, &khi);
                    a = *(const uint4*)(tile + off);
                    b = *(const uint4*)(tile + off + 16);
                    bin32_masks(a, b, klo, khi, m);
                }
                const bool cut = (m[0] | m[1] | m[2] | m[3] | m[4] | m[5] | m[6] | m[7]) != 0u;
                // list slots for this round's cut bins: one LDS add per wave
                const uint64_t bal = __ballot(cut);
                uint32_t base = 0;
                if (bal) {
                    const int leader = __ffsll((unsigned long long)bal) - 1;
                    if (lane == leader) base = atomicAdd(list_n, (uint32_t)__popcll(bal));
                    base = (uint32_t)__shfl((int)base, leader, 64);
                }
                const uint32_t sl =
                    base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                if (!cut) continue;
                if (sl < cap) {   // taken later by all lanes together
                    list[sl] = ((uint32_t)tl << 8) | (uint32_t)bb;
                    continue;
                }
                nflag += bin32_replace(tile, ftile, off, a, b, m, lower_median32(a, b), fbit, want_flags);
            }
        }
        if (count) {   // one LDS add per wave (all lanes are here)
            const uint32_t tot = wave_sum_u32(valid ? nflag : 0u);
            if ((tid & 63) == 0 && tot) atomicAdd(&s_cnt[s], (unsigned long long)tot);
        }
        if (med) {
            __syncthreads();
            const uint32_t nl = min(*list_n, cap);
            uint32_t nlist = 0;
            for (uint32_t e = tid; e < nl; e += kBlock) {
                const uint32_t ent = list[e];
                const uint32_t tl2 = ent >> 8, bb2 = ent & 255u;
                const uint32_t off = tl2 * (uint32_t)k.Cp + bb2 * 32u;
                const uint4 a = *(const uint4*)(tile + off);
                const uint4 b = *(const uint4*)(tile + off + 16);
                uint32_t S = 0;
                const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
                for (int i = 0; i < 8; i++) S = __builtin_amdgcn_udot4(w[i], 0x01010101u, S, false);
                uint32_t klo, khi;
                bin32_bounds(S, s_z[tl2], &klo, &khi);
                uint32_t m[8];
                bin32_masks(a, b, klo, khi, m);
                const uint32_t n = bin32_replace(tile, ftile, off, a, b, m, lower_median32(a, b), fbit, want_flags);
                if (k.t0 + (int64_t)tl2 < k.T) nlist += n;
            }
            if (count) {   // one LDS add per wave
                const uint32_t tot = wave_sum_u32(nlist);
                if (lane == 0 && tot) atomicAdd(&s_cnt[s], (unsigned long long)tot);
            }
            __syncthreads();
        }
    }
}

// Static LDS of one fused tile besides the tile itself
struct FusedShared {
    uint32_t exc_pos[kExcCap];   // (row << 8) | dword index in the tile
    uint32_t exc_n;
    unsigned long long s_cnt[kMaxSteps];
    uint32_t s_z[64];            // FD threshold per time sample of the tile
};

// Tile g of a launch's tile space, by the whole work-group; lds holds the
// [Tt][Cp] tile (and its flag tile).
template <bool VEC>
__device__ __attribute__((always_inline)) inline void fused_tile(const DevBeam* __restrict__ beams, int nbeams, int64_t g, const Segment& seg,
                                  const uint32_t* __restrict__ rec, unsigned long long* __restrict__ counts,
                                  int count_stride, uint8_t* lds, FusedShared& fs) {
    uint32_t* exc_pos = fs.exc_pos;
    uint32_t& exc_n = fs.exc_n;
    unsigned long long* s_cnt = fs.s_cnt;
    uint32_t* s_z = fs.s_z;
    const int tid = threadIdx.x;
    const int b = find_beam_by_tile(beams, nbeams, g);
    const DevBeam& bm = beams[b];
    TileCtx k;
    k.in = (const uint8_t*)bm.in;
    k.out = (uint8_t*)bm.out;
    k.flags = bm.flags;
    k.C = bm.C;
    k.T = bm.T;
    k.stride = bm.stride;
    k.Tt = bm.Tt;
    k.Cp = bm.Cp;
    k.t0 = (g - bm.tile0) * k.Tt;
    k.tw = k.Tt >> 2;
    k.tw_log = __ffs(k.tw) - 1;
    k.n_td = seg.n_td;
    k.rec = rec + bm.row0 * seg.n_td;
    k.nq4 = (k.C + 3) >> 2;
    const bool want_flags = seg.flags_mode != 0 && bm.flags != nullptr;
    const bool or_flags = seg.flags_mode == 2;
    const bool interior = k.t0 + k.Tt <= k.T && (k.stride & 3) == 0 &&
                          (((uintptr_t)k.in | (uintptr_t)k.out |
                            (want_flags ? (uintptr_t)k.flags : 0)) & 3) == 0;
    uint8_t* tile = lds;
    uint8_t* ftile = lds + (size_t)k.Tt * k.Cp;
    const int64_t ntask = k.nq4 * k.tw;

    if (tid < kMaxSteps) s_cnt[tid] = 0;
    if (tid == 0) exc_n = 0;
    __syncthreads();

    // ---- phase 1: rows in, TD fast check, transposed into LDS
    const bool wide = interior && (k.Tt & 15) == 0 && (uint64_t)k.C * (uint64_t)k.stride <= 0xFFFFFFFFull;
    if (wide) {
        constexpr int kPre = 3;   // tasks per thread whose loads are in flight together
        const int64_t n = ntask / 4;
        const int lane = tid & 63;
        // wave-uniform loop (the exception slots are reserved per wave)
        for (int64_t w0 = tid - lane; w0 < n; w0 += kPre * kBlock) {
            const int64_t b0 = w0 + lane;
            uint4 xs[kPre][4];
            uint32_t es[kPre][4];
            fetch16_batch<kPre>(k, b0, n, xs, es);
            uint32_t eb[kPre], cnt = 0;
#pragma unroll
            for (int u = 0; u < kPre; u++) {
                eb[u] = b0 + u * kBlock < n ? exc_bits16(k, b0 + u * kBlock, xs[u], es[u]) : 0u;
                cnt += (uint32_t)__popc(eb[u]);
            }
            // one worklist reservation for the wave: exclusive prefix of cnt
            uint32_t incl = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = (uint32_t)__shfl_up((int)incl, o, 64);
                if (lane >= o) incl += t;
            }
            const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
            uint32_t base = 0;
            if (total) {
                if (lane == 0) base = atomicAdd(&exc_n, total);
                base = (uint32_t)__shfl((int)base, 0, 64);
            }
            uint32_t slot = base + incl - cnt;
#pragma unroll
            for (int u = 0; u < kPre; u++)
                if (b0 + u * kBlock < n)
                    load_task16(k, b0 + u * kBlock, xs[u], eb[u], &slot, tile, ftile, want_flags, or_flags,
                                exc_pos);
        }
    } else if (interior) {
        for (int64_t idx = tid; idx < ntask; idx += kBlock)
            tile_load_task<true>(k, idx, tile, ftile, want_flags, or_flags, exc_pos, &exc_n);
    } else {
        for (int64_t idx = tid; idx < ntask; idx += kBlock)
            tile_load_task<false>(k, idx, tile, ftile, want_flags, or_flags, exc_pos, &exc_n);
    }
    __syncthreads();

    // ---- TD exceptions: full composite map for the dwords that need it
    if (k.n_td > 0 && k.n_td <= 4) {
        // a thread's (at most kExcCap / kBlock) exceptions: every record they
        // need is requested before any is used
        constexpr int kPer = (kExcCap + kBlock - 1) / kBlock;
        const uint32_t ne = min(exc_n, (uint32_t)kExcCap);   // the rest were mapped in phase 1
        uint32_t r[kPer][4];
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const uint32_t e = tid + u * kBlock;
            const uint32_t* rp = k.rec + (int64_t)(e < ne ? exc_pos[e] >> 8 : 0u) * k.n_td;
#pragma unroll
            for (int j = 0; j < 4; j++) r[u][j] = (e < ne && j < k.n_td) ? ld_global<uint32_t>(rp + j) : 0u;
        }
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const uint32_t e = tid + u * kBlock;
            if (e >= ne) continue;
            const uint32_t pos = exc_pos[e];
            const int64_t c = pos >> 8;
            const int w = pos & 255;
            uint32_t xv = 0;   // the tile still holds this dword's raw bytes
            for (int j = 0; j < 4; j++) xv |= (uint32_t)tile[(size_t)(4 * w + j) * k.Cp + c] << (8 * j);
            uint32_t nv = 0, f4 = 0;
#pragma unroll
            for (int b8 = 0; b8 < 4; b8++) {
                const uint32_t x = (xv >> (8 * b8)) & 255u;
                uint32_t out = x, f = 0;
                // the first step whose interval excludes x decides (intervals nest)
#pragma unroll
                for (int j = 3; j >= 0; j--) {
                    if (j >= k.n_td) continue;
                    const uint32_t rj = r[u][j];
                    if (x < (rj & 255u) || x > ((rj >> 8) & 255u)) {
                        out = (rj >> 16) & 255u;
                        f = rj >> 24;
                    }
                }
                nv |= out << (8 * b8);
                f4 |= f << (8 * b8);
            }
            put_dword_transposed(tile, k, c, w, nv);
            if (want_flags) or_dword_transposed(ftile, k, c, w, f4);
        }
    } else if (k.n_td > 0) {
        const uint32_t ne = min(exc_n, (uint32_t)kExcCap);   // the rest were mapped in phase 1
        for (uint32_t e = tid; e < ne; e += kBlock) {
            const uint32_t pos = exc_pos[e];
            const int64_t c = pos >> 8;
            const int w = pos & 255;
            // the tile still holds this dword's raw bytes
            uint32_t xv = 0;
            for (int j = 0; j < 4; j++) xv |= (uint32_t)tile[(size_t)(4 * w + j) * k.Cp + c] << (8 * j);
            uint32_t f;
            put_dword_transposed(tile, k, c, w, td_map_dword(k, c, xv, &f));
            if (want_flags) or_dword_transposed(ftile, k, c, w, f);
        }
    }
    __syncthreads();

    // ---- phase 2: FD steps
    if (seg.n_fd > 0) {
        // the host chose the path for this beam's shape, tile and bins
        const bool cnt = counts != nullptr;
        if (VEC && bm.path == RFIM_FD_PATH_U8_BIN32_G8)
            fd_steps_b32<8>(k, seg, tile, ftile, want_flags, cnt, s_cnt, exc_pos, &exc_n, kExcCap, s_z);
        else if (VEC && bm.path == RFIM_FD_PATH_U8_BIN32_G16)
            fd_steps_b32<16>(k, seg, tile, ftile, want_flags, cnt, s_cnt, exc_pos, &exc_n, kExcCap, s_z);
        else if (VEC && bm.path == RFIM_FD_PATH_U8_BIN32_G4)
            fd_steps_b32<4>(k, seg, tile, ftile, want_flags, cnt, s_cnt, exc_pos, &exc_n, kExcCap, s_z);
        else
            fd_steps<VEC>(k, seg, tile, ftile, want_flags, cnt, s_cnt);
    }
    __syncthreads();

    // ---- phase 3: transposed back, rows out
    if (wide) {
        for (int64_t idx = tid; idx < ntask / 4; idx += kBlock) tile_store_task16(k, idx, tile, ftile, want_flags);
    } else if (interior) {
        for (int64_t idx = tid; idx < ntask; idx += kBlock) tile_store_task<true>(k, idx, tile, ftile, want_flags);
    } else {
        for (int64_t idx = tid; idx < ntask; idx += kBlock) tile_store_task<false>(k, idx, tile, ftile, want_flags);
    }
    if (counts && seg.n_fd > 0 && tid < seg.n_fd && s_cnt[tid])
        atomicAdd(&counts[(int64_t)bm.cidx * count_stride + seg.fd[tid].ci], s_cnt[tid]);
}

// One work-group per (beam, time tile); work-groups are handed out so that
// each XCD gets a contiguous range of tiles.
template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_fused_u8(const DevBeam* __restrict__ beams, int nbeams,
                                                     int64_t total_tiles, Segment seg,
                                                     const uint32_t* __restrict__ rec,
                                                     unsigned long long* __restrict__ counts,
                                                     int count_stride) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ FusedShared fs;
    fused_tile<VEC>(beams, nbeams, xcd_remap(blockIdx.x, total_tiles), seg, rec, counts, count_stride, lds, fs);
}

// ---------------------------------------------------------------------------
// Persistent beam-major schedule: the TD pass and the fused pass of a run in
// one launch.  Work items are ordered by beam and, within a beam, its TD row
// groups come before its tiles, so a beam's second read follows its first
// closely enough to be served from the Infinity Cache.  The beams are dealt to
// kPersistQueues queues (balanced by item count on the host); work-group i
// takes items from queue i mod kPersistQueues, the XCD the hardware deals it
// to, so a beam's records stay in one XCD's L2, and moves on to the other
// queues when its own is empty, so every item is taken whatever the mapping.
// A tile waits until every row group of its beam is done (a per-beam counter,
// released after the group's records are written and acquired before they are
// read, once per beam and work-group).  The wait always ends: those row groups
// were all taken earlier, by running work-groups that never wait.  It is
// bounded anyway: past spin_limit polls the work-group sets the error word
// and stops taking items, and the host reports it.  wait_extra (0 in use) is
// added to the count a tile waits for: a test sets it to make every wait
// run out on purpose.  Both bodies inlined into one kernel need more
// registers than either alone; the fused pass's LDS already caps a CU at three
// work-groups (three waves per SIMD), which the register budget keeps.
template <bool VEC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_persist_u8(
    const DevBeam* __restrict__ beams, int nbeams, PersistQueues qs, Segment seg, uint32_t* __restrict__ rec,
    unsigned long long* __restrict__ counts, int count_stride, unsigned* __restrict__ ctl, uint32_t spin_limit,
    uint32_t wait_extra) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ FusedShared fs;
    __shared__ int64_t s_item;
    __shared__ int s_go;
    TdShared& tsh = *reinterpret_cast<TdShared*>(lds);   // the tile's LDS, reused by row groups
    unsigned* next = ctl;                                 // [kPersistQueues]
    unsigned* err = ctl + kPersistQueues;
    unsigned* done = ctl + kPersistQueues + 1;            // [nbeams]
    const int q0 = (int)(blockIdx.x % kPersistQueues);
    int acquired = -1;   // beam whose row groups this work-group has seen completed
    for (int qi = 0; qi < kPersistQueues;) {
        const int q = (q0 + qi) % kPersistQueues;
        __syncthreads();   // the previous item is done with the LDS
        if (threadIdx.x == 0) {
            const int64_t n = qs.base[q + 1] - qs.base[q];
            const int64_t k = n > 0 ? (int64_t)atomicAdd(&next[q], 1u) : n;
            s_item = k < n ? qs.base[q] + k : -1;
        }
        __syncthreads();
        const int64_t it = s_item;
        if (it < 0) {   // this queue is empty: the next one
            qi++;
            continue;
        }
        int lo = 0, hi = nbeams - 1;   // the beam: last with item0 <= it
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (beams[mid].item0 <= it) lo = mid; else hi = mid - 1;
        }
        const DevBeam& bm = beams[lo];
        const int64_t local = it - bm.item0;
        const int64_t ntd = seg.n_td > 0 ? (bm.C + kRowsPerWG - 1) / kRowsPerWG : 0;
        if (local < ntd) {
            td_row_group<kRowsPerWG>(beams, nbeams, bm.row0 + local * kRowsPerWG, bm.row0 + bm.C, seg, rec, counts,
                                     count_stride, tsh);
            __syncthreads();   // every wave's records are written (work-group scope)
            if (threadIdx.x == 0) __hip_atomic_fetch_add(&done[lo], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        if (ntd > 0 && acquired != lo) {
            if (threadIdx.x == 0) {
                int ok = 0;
                for (uint32_t n = 0;; n++) {
                    if (__hip_atomic_load(&done[lo], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >=
                        (unsigned)ntd + wait_extra) {
                        ok = 1;
                        break;
                    }
                    if (n >= spin_limit) break;
                    __builtin_amdgcn_s_sleep(4);
                }
                if (!ok) atomicOr(err, 1u);
                s_go = ok;
            }
            __syncthreads();
            if (!s_go) break;
            acquired = lo;
        }
        fused_tile<VEC>(beams, nbeams, bm.tile0 + (local - ntd), seg, rec, counts, count_stride, lds, fs);
    }
}

size_t td_group_lds_bytes() { return sizeof(TdShared); }

int persist_u8_grid(size_t lds_bytes, bool vec) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const hipError_t e = vec ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist_u8<true>, kBlock, lds_bytes)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist_u8<false>, kBlock, lds_bytes);
    if (e != hipSuccess || per <= 0) per = 1;
    return cus * per;
}

hipError_t launch_persist_u8(const DevBeam* d_beams, int nbeams, const PersistQueues& qs, const Segment& seg,
                             uint32_t* d_rec, size_t lds_bytes, bool vec, unsigned long long* d_counts,
                             int count_stride, unsigned* ctl, uint32_t spin_limit, uint32_t wait_extra, int grid,
                             hipStream_t s) {
    const int64_t total_items = qs.base[kPersistQueues];
    if (total_items <= 0) return hipSuccess;
    grid = (int)std::min<int64_t>(grid, total_items);
    if (vec)
        hipLaunchKernelGGL(k_persist_u8<true>, dim3(grid), dim3(kBlock), lds_bytes, s, d_beams, nbeams, qs, seg,
                           d_rec, d_counts, count_stride, ctl, spin_limit, wait_extra);
    else
        hipLaunchKernelGGL(k_persist_u8<false>, dim3(grid), dim3(kBlock), lds_bytes, s, d_beams, nbeams, qs, seg,
                           d_rec, d_counts, count_stride, ctl, spin_limit, wait_extra);
    return hipGetLastError();
}

hipError_t launch_td_rows_u8(const DevBeam* d_beams, int nbeams, int64_t total_rows, int rows_per_wg,
                             const Segment& seg, uint32_t* d_rec, unsigned long long* d_counts,
                             int count_stride, hipStream_t s) {
    if (total_rows <= 0) return hipSuccess;
    auto go = [&](auto kern, int R) {
        const int64_t wgs = (total_rows + R - 1) / R;
        hipLaunchKernelGGL(kern, dim3((unsigned)wgs), dim3(64 * R), 0, s, d_beams, nbeams, total_rows, seg, d_rec,
                           d_counts, count_stride);
    };
    switch (rows_per_wg) {
        case 2: go(k_td_rows_u8<2>, 2); break;
        case 8: go(k_td_rows_u8<8>, 8); break;
        default: go(k_td_rows_u8<4>, 4); break;
    }
    return hipGetLastError();
}

hipError_t launch_fused_u8(const DevBeam* d_beams, int nbeams, int64_t total_tiles,
                           const Segment& seg, const uint32_t* d_rec, size_t lds_bytes, bool vec,
                           unsigned long long* d_counts, int count_stride, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    if (vec)
        hipLaunchKernelGGL(k_fused_u8<true>, dim3((unsigned)total_tiles), dim3(kBlock), lds_bytes, s,
                           d_beams, nbeams, total_tiles, seg, d_rec, d_counts, count_stride);
    else
        hipLaunchKernelGGL(k_fused_u8<false>, dim3((unsigned)total_tiles), dim3(kBlock), lds_bytes, s,
                           d_beams, nbeams, total_tiles, seg, d_rec, d_counts, count_stride);
    return hipGetLastError();
}

}  // namespace rfim
