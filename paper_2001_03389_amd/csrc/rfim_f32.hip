// float32 sigma-cut kernels for gfx950 (RFIm, arXiv:2001.03389, Section IV).
//
// Same two-kernel shape as the uint8 path, per run of [TD steps][FD steps]:
//  * k_td_rows_f32 -- one work-group per channel row, the whole row resident in
//    VGPRs (up to 64 values per lane of a 1024-lane work-group).  Exact window
//    statistics (see rfim_f32_exact.h), every TD step of the run decided and
//    applied in registers, one record (Lo, H, r) per step: a sample x is kept
//    by step j iff Lo_j <= x <= H_j, else it becomes r_j.
//  * k_fused_f32 -- one work-group per (beam, time tile).  Rows in (16-byte
//    loads), the TD records applied on the way, tile stored in LDS as [Tt][Cp]
//    with channels contiguous and every B-channel bin padded by 4 floats so that
//    the lanes' 16-byte bin reads hit distinct banks.  One time sample per group
//    of lanes, one bin per lane: exact bin sums and sums of squares, the exact
//    cut of the time sample, per-bin float32 thresholds, replacement in
//    registers.  The tile is written back to rows.
// Rows and time samples that leave the window (values more than 2^-24 below
// the largest one, or a replacement value that is) go to lists that the wide
// kernels k_td_wide_f32 / k_fd_wide_f32 finish with big integers.
#include <algorithm>

#include "rfim_big.h"
#include "rfim_dev.h"

namespace rfim {

namespace {

constexpr u128 kZcap = (u128)1 << 70;   // beyond every |n*a - S| of a window row

// ---- wave / group reductions --------------------------------------------

__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
// The value of this lane's partner at distance o (1, 2, 4, ... 32) in a
// whole-wave reduction whose levels go in ascending order: DPP within 16-lane
// rows (quad swaps, then the half-row and row mirrors, whose partners lie in
// the other half once each half holds one value), LDS permutes across rows.
template <int O>
__device__ inline uint32_t lane_partner(uint32_t v) {
    if constexpr (O == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);
    else if constexpr (O == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);
    else if constexpr (O == 4) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false);
    else if constexpr (O == 8) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false);
    else return (uint32_t)__shfl_xor((int)v, O, 64);
}
template <int O>
__device__ inline uint64_t lane_partner64(uint64_t v) {
    return (uint64_t)lane_partner<O>((uint32_t)v) | ((uint64_t)lane_partner<O>((uint32_t)(v >> 32)) << 32);
}
__device__ inline uint32_t wave_min_u32(uint32_t v) {
    v = min(v, lane_partner<1>(v));
    v = min(v, lane_partner<2>(v));
    v = min(v, lane_partner<4>(v));
    v = min(v, lane_partner<8>(v));
    v = min(v, lane_partner<16>(v));
    return min(v, lane_partner<32>(v));
}
__device__ inline uint32_t wave_add_u32(uint32_t v) {
    v += lane_partner<1>(v);
    v += lane_partner<2>(v);
    v += lane_partner<4>(v);
    v += lane_partner<8>(v);
    v += lane_partner<16>(v);
    return v + lane_partner<32>(v);
}
__device__ inline int64_t wave_add_i64(int64_t v) {
    uint64_t u = (uint64_t)v;
    u += lane_partner64<1>(u);
    u += lane_partner64<2>(u);
    u += lane_partner64<4>(u);
    u += lane_partner64<8>(u);
    u += lane_partner64<16>(u);
    return (int64_t)(u + lane_partner64<32>(u));
}
template <int O>
__device__ inline u128 u128_partner(u128 v) {
    return (u128)lane_partner64<O>((uint64_t)v) | ((u128)lane_partner64<O>((uint64_t)(v >> 64)) << 64);
}
__device__ inline uint32_t wave_max_dpp(uint32_t v) {
    v = max(v, lane_partner<1>(v));
    v = max(v, lane_partner<2>(v));
    v = max(v, lane_partner<4>(v));
    v = max(v, lane_partner<8>(v));
    v = max(v, lane_partner<16>(v));
    return max(v, lane_partner<32>(v));
}
__device__ inline uint32_t wave_or_dpp(uint32_t v) {
    v |= lane_partner<1>(v);
    v |= lane_partner<2>(v);
    v |= lane_partner<4>(v);
    v |= lane_partner<8>(v);
    v |= lane_partner<16>(v);
    return v | lane_partner<32>(v);
}
// sum of u128 over the whole wave
__device__ inline u128 wave_add_u128(u128 v) {
    v += u128_partner<1>(v);
    v += u128_partner<2>(v);
    v += u128_partner<4>(v);
    v += u128_partner<8>(v);
    v += u128_partner<16>(v);
    return v + u128_partner<32>(v);
}
// sum of u128 over lanes xor-partnered within groups of G (power of two)
__device__ inline u128 group_add_u128(u128 v, int G) {
    uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
    for (int o = 1; o < G; o <<= 1) {
        const uint64_t olo = __shfl_xor(lo, o, 64);
        const uint64_t ohi = __shfl_xor(hi, o, 64);
        const uint64_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1 : 0);
        lo = nlo;
    }
    return ((u128)hi << 64) | lo;
}
__device__ inline uint32_t group_max_u32(uint32_t v, int G) {
    for (int o = 1; o < G; o <<= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ inline uint32_t group_min_u32(uint32_t v, int G) {
    for (int o = 1; o < G; o <<= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ inline uint32_t group_or_u32(uint32_t v, int G) {
    for (int o = 1; o < G; o <<= 1) v |= (uint32_t)__shfl_xor((int)v, o, 64);
    return v;
}

// smallest power of two >= v (v <= 64)
__device__ inline int pow2_ceil(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// tiny test: a non-zero value below the window of a row/column whose window
// threshold (bits of the smallest in-window magnitude) is thr
__device__ inline bool below_window(uint32_t bits, uint32_t thr) {
    const uint32_t m = bits & 0x7FFFFFFFu;
    return m != 0 && m < thr;
}

__device__ inline uint32_t window_thr(int EM) { return EM - 24 >= 1 ? (uint32_t)(EM - 24) << 23 : 0u; }
// bits of the smallest magnitude inside the second window (24 exponents lower)
__device__ inline uint32_t window_thr2(int EM) { return EM - 48 >= 1 ? (uint32_t)(EM - 48) << 23 : 0u; }

constexpr u128 kZcap2 = (u128)1 << 94;   // beyond every |n*a - S| in second-window units

// ---- work-group radix select (TD median) ---------------------------------

// Key of rank `rank` (ascending totalOrder) among the keys the callback adds,
// by four 8-bit digit rounds over per-wave LDS histograms.  All NT threads call.
template <int NT, typename AddKeys>
__device__ inline uint32_t wg_select_key(uint64_t rank, uint32_t* s_hist, uint32_t* s_tot, uint32_t* s_sel,
                                         AddKeys&& add_keys) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    uint32_t prefix = 0, mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int i = tid; i < NW * 256; i += NT) s_hist[i] = 0;
        __syncthreads();
        uint32_t* h = s_hist + wave * 256;
        add_keys([&](uint32_t k) {
            if (((k ^ prefix) & mask) == 0) atomicAdd(&h[(k >> shift) & 255u], 1u);
        });
        __syncthreads();
        uint32_t cnt = 0, incl = 0;
        if (tid < 256) {
            for (int w = 0; w < NW; w++) cnt += s_hist[w * 256 + tid];
            incl = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(incl, o, 64);
                if (lane >= o) incl += t;
            }
            if (lane == 63) s_tot[wave] = incl;
        }
        __syncthreads();
        if (tid < 256) {
            uint32_t off = 0;
            for (int w = 0; w < wave; w++) off += s_tot[w];
            const uint64_t excl = (uint64_t)off + incl - cnt;
            if (cnt && excl <= rank && rank < excl + cnt) {
                s_sel[0] = (uint32_t)tid;
                s_sel[1] = (uint32_t)excl;
            }
        }
        __syncthreads();
        rank -= s_sel[1];
        prefix |= s_sel[0] << shift;
        mask |= 255u << shift;
        __syncthreads();
    }
    return prefix;
}

// Key of rank `rank` among the values the callback visits, by value bins: a
// value x in [lo, hi) (by IEEE totalOrder) goes to bin (x - lo) * NB / (hi - lo)
// rounded down, a map that never decreases as x grows, so the bins keep the
// values' order; a prefix sum over the bins finds the one that holds the rank,
// and that bin's values, at most CAP of them, are ranked exactly by key.
// Returns false, the same on every thread, when the rank lies outside the
// range or its bin holds more than CAP values (the caller then runs
// wg_select_key).  The caller zeroes s_bins[0, NB) and s_m[0, 8) and
// synchronises first.  All NT threads call.
template <int NT, int NB, int CAP, typename Visit>
__device__ inline bool wg_select_bins(uint32_t rank, float lo, float hi, uint32_t* s_bins, uint32_t* s_cand,
                                      uint32_t* s_tot, uint32_t* s_m, Visit&& visit, uint32_t* key) {
    constexpr int NW = NT / 64;
    constexpr int BPT = NB / NT;
    static_assert(BPT * NT == NB, "bins per thread");
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t klo = f32_key(__float_as_uint(lo)), khi = f32_key(__float_as_uint(hi));
    const float inv = (float)NB / (hi - lo);   // finite and positive (the caller checks)
    auto bin_of = [&](float x) {
        const int b = (int)((x - lo) * inv);
        return b < NB ? b : NB - 1;
    };
    uint32_t below = 0;
    visit([&](float x) {
        const uint32_t k = f32_key(__float_as_uint(x));
        if (k < klo) below++;
        else if (k < khi) atomicAdd(&s_bins[bin_of(x)], 1u);
    });
    below = wave_add_u32(below);
    if (lane == 0 && below) atomicAdd(&s_m[0], below);
    __syncthreads();
    below = s_m[0];
    uint32_t c[BPT], sum = 0;
#pragma unroll
    for (int j = 0; j < BPT; j++) {
        c[j] = s_bins[tid * BPT + j];
        sum += c[j];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) s_tot[wave] = incl;
    __syncthreads();
    if (rank >= below) {
        const uint32_t r2 = rank - below;
        uint32_t acc = incl - sum;
        for (int w = 0; w < wave; w++) acc += s_tot[w];
        if (acc <= r2 && r2 < acc + sum) {
#pragma unroll
            for (int j = 0; j < BPT; j++) {
                if (r2 < acc + c[j]) {
                    s_m[1] = (uint32_t)(tid * BPT + j);
                    s_m[2] = r2 - acc;   // rank inside the bin
                    s_m[3] = c[j];
                    s_m[5] = 1;
                    break;
                }
                acc += c[j];
            }
        }
    }
    __syncthreads();
    const uint32_t m = s_m[3];
    if (!s_m[5] || m > (uint32_t)CAP) return false;
    const int jb = (int)s_m[1];
    visit([&](float x) {
        const uint32_t k = f32_key(__float_as_uint(x));
        if (k >= klo && k < khi && bin_of(x) == jb) s_cand[atomicAdd(&s_m[4], 1u)] = k;
    });
    __syncthreads();
    const uint32_t rr = s_m[2];
    for (uint32_t i = tid; i < m; i += NT) {
        const uint32_t my = s_cand[i];
        uint32_t pos = 0;
        for (uint32_t q = 0; q < m; q++) {
            const uint32_t o = s_cand[q];
            pos += (o < my || (o == my && q < i)) ? 1u : 0u;
        }
        if (pos == rr) s_m[6] = my;
    }
    __syncthreads();
    *key = s_m[6];
    return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// TD: one work-group per row, row resident in registers
// ---------------------------------------------------------------------------
// All TD steps of the run for row c of beam bm, by the whole work-group.
// VL of each lane's VPT values live in LDS (rows too long for the register
// file alone), the other VR = VPT - VL in registers.  TWO = false: the first
// window only; a row with values below it goes to the two-window list
// (tiny_*), whose kernel runs this body with TWO = true; a row with values
// below the second window goes to the wide list.
template <int NT, int VPT, int VL, bool TWO>
__device__ inline void td_row_f32(const DevBeam& bm, int64_t c, const Segment& seg, float4* __restrict__ rec,
                                  unsigned* __restrict__ tiny_n, int2* __restrict__ tiny_items,
                                  unsigned* __restrict__ wide_n, int2* __restrict__ wide_items,
                                  unsigned long long* __restrict__ counts, int count_stride) {
    constexpr int NW = NT / 64;
    constexpr int VR = VPT - VL;
    __shared__ uint32_t s_hist[NW * 256];
    __shared__ float s_row[VL > 0 ? VL * NT : 1];
    __shared__ uint32_t s_tot[NW], s_sel[2], s_msel[8];
    __shared__ double s_mom[NW][2];
    __shared__ int64_t s_S[NW], s_S1[NW];
    __shared__ uint64_t s_Q[NW][2], s_Q1[NW][2];
    __shared__ uint32_t s_u[NW][2];
    __shared__ float s_dec[3];
    __shared__ int s_bad;
    __shared__ uint32_t s_cnt[kMaxSteps];
    // wave 0 parks its row values here while it decides a step, so that the
    // decision's wide-integer temporaries reuse their registers
    __shared__ float s_park[64 * VR];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t T = bm.T;
    const float* row = (const float*)bm.in + c * bm.stride;
    const bool vec = (VPT % 4 == 0) && ((((uintptr_t)row) & 15) == 0);

    // values of this lane: index i*NT + tid (scalar) or 4*((i/4)*NT + tid) + i%4
    // (16-byte loads); both increase with i, so the valid ones are a prefix
    float v[VR];
    // value i of this lane (i a compile-time constant after unrolling)
    auto get = [&](int i) -> float { return i < VR ? v[i < VR ? i : 0] : s_row[(i - VR) * NT + tid]; };
    auto set = [&](int i, float x) {
        if (i < VR) v[i < VR ? i : 0] = x;
        else s_row[(i - VR) * NT + tid] = x;
    };
    // A full row (no padding) takes loops without per-value validity tests:
    // the compiler keeps those tests as one lane mask per value, more than the
    // scalar registers hold.
    const bool full = T == (int64_t)NT * VPT;
    int nv = 0;
    if (vec && full) {
#pragma unroll
        for (int i4 = 0; i4 < VPT / 4; i4++) {
            const float4 q = *(const float4*)(row + ((int64_t)i4 * NT + tid) * 4);
            set(4 * i4, q.x);
            set(4 * i4 + 1, q.y);
            set(4 * i4 + 2, q.z);
            set(4 * i4 + 3, q.w);
        }
        nv = VPT;
    } else if (vec) {
#pragma unroll
        for (int i4 = 0; i4 < VPT / 4; i4++) {
            const int64_t i0 = ((int64_t)i4 * NT + tid) * 4;
            if (i0 + 3 < T) {
                const float4 q = *(const float4*)(row + i0);
                set(4 * i4, q.x);
                set(4 * i4 + 1, q.y);
                set(4 * i4 + 2, q.z);
                set(4 * i4 + 3, q.w);
            } else {
#pragma unroll
                for (int j = 0; j < 4; j++) set(4 * i4 + j, i0 + j < T ? row[i0 + j] : 0.0f);
            }
            const int64_t rem = T - i0;
            nv += rem >= 4 ? 4 : (rem > 0 ? (int)rem : 0);
        }
    } else {
#pragma unroll
        for (int i = 0; i < VPT; i++) {
            const int64_t idx = (int64_t)i * NT + tid;
            set(i, idx < T ? row[idx] : 0.0f);
            nv += idx < T ? 1 : 0;
        }
    }

    // window of the row: largest magnitude, smallest non-zero magnitude
    uint32_t emax = 0, tmin = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < VPT; i++) {
        const uint32_t bb = __float_as_uint(get(i)) & 0x7FFFFFFFu;   // padding is +0
        emax = max(emax, bb);
        tmin = min(tmin, bb - 1u);                                  // 0 wraps: ignored
    }
    emax = wave_max_u32(emax);
    tmin = wave_min_u32(tmin);
    if (lane == 0) {
        s_u[wave][0] = emax;
        s_u[wave][1] = tmin;
    }
    if (tid < kMaxSteps) s_cnt[tid] = 0;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    emax = 0;
    tmin = 0xFFFFFFFFu;
    for (int w = 0; w < NW; w++) {
        emax = max(emax, s_u[w][0]);
        tmin = min(tmin, s_u[w][1]);
    }
    const int EM = f32_E(emax);
    const uint32_t thr = window_thr(EM), thr2 = window_thr2(EM);
    // values below the first window use the second; below that, the wide path
    const bool has_tiny = tmin != 0xFFFFFFFFu && tmin + 1u < thr;
    bool bad = tmin != 0xFFFFFFFFu && tmin + 1u < thr2;
    bool to_two = !TWO && has_tiny && !bad;   // hand over to the two-window kernel
    const bool tiny = TWO;
    const double sc = ldexp(1.0, 174 - EM), sc2 = ldexp(1.0, 198 - EM);
    const int e = EM - 174, e2 = EM - 198;
    const uint32_t n = (uint32_t)T;

    // The row's lower median m stays the lower median after a step that replaces
    // its cut samples by m while keeping m itself (cut samples lie strictly below
    // Lo <= m or above H >= m, and the counts on either side of m then keep m at
    // rank floor((n-1)/2)); known_med says m is current.
    bool known_med = false;
    float cur_med = 0.0f;
    // After the first step the exact sums change only by the replaced
    // samples, so each lane accumulates (r - x) and (r^2 - x^2) of the samples
    // it replaces (integers in units of each window, a value and its
    // replacement each in the window that holds it) and the next step adds
    // those deltas to the running totals wave 0 keeps.
    int64_t dS = 0, dS1 = 0;
    u128 dQ = 0, dQ1 = 0;           // two's complement: the deltas may be negative
    i128 St_run = 0, St1_run = 0;   // wave 0: running exact sums of both windows
    u128 Qt_run = 0, Qt1_run = 0;
    for (int j = 0; j < seg.n_td && !bad && !to_two; j++) {
        const SegStep& st = seg.td[j];
        // exact window sums (both windows when the row has values below the first)
        int64_t S = 0, S1 = 0;
        u128 Q = 0, Q1 = 0;
        if (j > 0) {
            S = dS;
            Q = dQ;
            S1 = dS1;
            Q1 = dQ1;
        } else if (!tiny) {
#pragma unroll
            for (int i0 = 0; i0 < VPT; i0 += 32) {
                WinAcc w{0.0, 0.0, 0.0};
#pragma unroll
                for (int i = i0; i < (i0 + 32 < VPT ? i0 + 32 : VPT); i++) winacc_add(w, (double)get(i) * sc);
                S += (int64_t)w.s;
                Q += winacc_q(w);
            }
        } else {
#pragma unroll
            for (int i0 = 0; i0 < VPT; i0 += 32) {
                WinAcc w{0.0, 0.0, 0.0}, w1{0.0, 0.0, 0.0};
#pragma unroll
                for (int i = i0; i < (i0 + 32 < VPT ? i0 + 32 : VPT); i++) {
                    const float x = get(i);
                    const bool lo = below_window(__float_as_uint(x), thr);
                    winacc_add(w, lo ? 0.0 : (double)x * sc);
                    winacc_add(w1, lo ? (double)x * sc2 : 0.0);
                }
                S += (int64_t)w.s;
                Q += winacc_q(w);
                S1 += (int64_t)w1.s;
                Q1 += winacc_q(w1);
            }
        }
        if (tiny) {
            S1 = wave_add_i64(S1);
            Q1 = wave_add_u128(Q1);
        }
        S = wave_add_i64(S);
        Q = wave_add_u128(Q);
        if (lane == 0) {
            s_S[wave] = S;
            s_Q[wave][0] = (uint64_t)Q;
            s_Q[wave][1] = (uint64_t)(Q >> 64);
            s_S1[wave] = S1;
            s_Q1[wave][0] = (uint64_t)Q1;
            s_Q1[wave][1] = (uint64_t)(Q1 >> 64);
        }
        __syncthreads();
        float med = cur_med;
        if (st.replace == RFIM_REPLACE_MEDIAN && !known_med) {
            // The lower median lies within one (population) standard deviation
            // of the mean, so value bins over mean -+ 1.0625 sd hold it; the
            // radix select is the fallback for rows the bins do not settle.
            constexpr int NB = NW * 128, CAP = NW * 128;   // both halves of s_hist
            const uint32_t rank = (n - 1) / 2;
            if (j == 0 && !tiny) {
                // mean and deviation from the step's exact window sums (one thread)
                if (tid == 0) {
                    double S = 0.0, Q = 0.0;
                    for (int w = 0; w < NW; w++) {
                        S += (double)s_S[w];
                        Q += u128_to_double(((u128)s_Q[w][1] << 64) | s_Q[w][0]);
                    }
                    const double m = S / n;
                    s_mom[0][0] = ldexp(m, e);
                    s_mom[0][1] = ldexp(sqrt(fmax(Q / n - m * m, 0.0)), e);
                }
            } else {
                double sx = 0.0, sxx = 0.0;   // padding is +0 until the row is written
#pragma unroll
                for (int i = 0; i < VPT; i++) {
                    const double x = (double)get(i);
                    sx += x;
                    sxx += x * x;
                }
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    sx += __shfl_xor(sx, o, 64);
                    sxx += __shfl_xor(sxx, o, 64);
                }
                if (lane == 0) {
                    s_mom[wave][0] = sx;
                    s_mom[wave][1] = sxx;
                }
                __syncthreads();
                if (tid == 0) {
                    sx = sxx = 0.0;
                    for (int w = 0; w < NW; w++) {
                        sx += s_mom[w][0];
                        sxx += s_mom[w][1];
                    }
                    const double m = sx / n;
                    s_mom[0][0] = m;
                    s_mom[0][1] = sqrt(fmax(sxx / n - m * m, 0.0));
                }
            }
            for (int i = tid; i < NB; i += NT) s_hist[i] = 0;
            if (tid < 8) s_msel[tid] = 0;
            __syncthreads();
            const double mu = s_mom[0][0], sd = s_mom[0][1];
            uint32_t key = 0;
            bool ok = false;
            const double rad = 1.0625 * sd + fabs(mu) * 0x1p-20;
            const float lo = (float)(mu - rad), hi = (float)(mu + rad);
            const float wdt = hi - lo;
            if (!ok)
                ok = isfinite(lo) && isfinite(hi) && wdt >= 0x1p-100f && isfinite((float)NB / wdt) &&
                     wg_select_bins<NT, NB, CAP>(rank, lo, hi, s_hist, s_hist + NB, s_tot, s_msel,
                                                 [&](auto&& add) {
                                                     if (full) {
#pragma unroll
                                                         for (int i = 0; i < VPT; i++) add(get(i));
                                                     } else {
#pragma unroll
                                                         for (int i = 0; i < VPT; i++)
                                                             if (i < nv) add(get(i));
                                                     }
                                                 }, &key);
            if (!ok)
                key = wg_select_key<NT>((uint64_t)(n - 1) / 2, s_hist, s_tot, s_sel, [&](auto&& add) {
                    if (full) {
#pragma unroll
                        for (int i = 0; i < VPT; i++) add(f32_key(__float_as_uint(get(i))));
                    } else {
#pragma unroll
                        for (int i = 0; i < VPT; i++)
                            if (i < nv) add(f32_key(__float_as_uint(get(i))));
                    }
                });
            med = __uint_as_float(key_f32(key));
        }
        if (wave == 0) {
#pragma unroll
            for (int i = 0; i < VR; i++) s_park[i * 64 + lane] = v[i];
            i128 St = 0, St1 = 0;
            u128 Qt = 0, Qt1 = 0;
            for (int w = 0; w < NW; w++) {
                St += s_S[w];
                Qt += ((u128)s_Q[w][1] << 64) | s_Q[w][0];
                St1 += s_S1[w];
                Qt1 += ((u128)s_Q1[w][1] << 64) | s_Q1[w][0];
            }
            if (j > 0) {   // the sums of step j > 0 are the deltas of step j - 1's replacements
                St += St_run;
                Qt += Qt_run;
                St1 += St1_run;
                Qt1 += Qt1_run;
            }
            St_run = St;
            Qt_run = Qt;
            St1_run = St1;
            Qt1_run = Qt1;
            float H, Lo, rm;
            if (!TWO) {
                const u128 Sa = St < 0 ? (u128)(-St) : (u128)St;
                const u128 D = (u128)n * Qt - Sa * Sa;
                // certified FP64 evaluation of the cut and the mean, else exact
                bool cert = false;
                if (st.kx.mode == 0) {
                    const double Sd = i128_to_double(St);
                    const double zr = st.kx.k * sqrt(u128_to_double(D));
                    cert = f32_cut_fast(Sd, zr, (double)n, e, &H, &Lo) && f32_mean_fast(Sd, (double)n, e, &rm);
                }
                if (!cert) {
                    const u128 z = zmax_k2(1, D, st.kx, kZcap);
                    H = f32_round_ratio(St + (i128)z, n, e, kRD);
                    Lo = f32_round_ratio(St - (i128)z, n, e, kRU);
                    rm = f32_round_ratio(St, n, e, kRN);
                }
            } else {
                // units of the second window: S = S0 * 2^24 + S1, Q = Q0 * 2^48 + Q1
                const i128 Sc = St * ((i128)1 << 24) + St1;
                const U512 D = d_combine(n, q_combine(Qt, Qt1), Sc);
                bool cert = false;   // certified FP64 evaluation, else exact
                if (st.kx.mode == 0) {
                    const double Sd = i128_to_double(Sc);
                    const double zr = st.kx.k * sqrt(u512_to_double(D));
                    cert = f32_cut_fast(Sd, zr, (double)n, e2, &H, &Lo) && f32_mean_fast(Sd, (double)n, e2, &rm);
                }
                if (!cert) {
                    const u128 z = zmax_k2w(1, D, st.kx, kZcap2);
                    H = f32_round_ratio(Sc + (i128)z, n, e2, kRD);
                    Lo = f32_round_ratio(Sc - (i128)z, n, e2, kRU);
                    rm = f32_round_ratio(Sc, n, e2, kRN);
                }
            }
            const float r = st.replace == RFIM_REPLACE_MEDIAN ? med : rm;
            if (lane == 0) {
                s_dec[0] = Lo;
                s_dec[1] = H;
                s_dec[2] = r;
                if (below_window(__float_as_uint(r), thr2)) s_bad = 1;
                else if (!TWO && below_window(__float_as_uint(r), thr)) s_bad = 2;
                rec[(bm.rec0 + c) * seg.n_td + j] = make_float4(Lo, H, r, 0.0f);
            }
#pragma unroll
            for (int i = 0; i < VR; i++) v[i] = s_park[i * 64 + lane];
        }
        __syncthreads();
        const float Lo = s_dec[0], H = s_dec[1], r = s_dec[2];
        bad = s_bad == 1;
        to_two = s_bad == 2;   // a replacement below the first window joins the data
        known_med = st.replace == RFIM_REPLACE_MEDIAN && !(med < Lo) && !(med > H);
        cur_med = med;
        uint32_t cnt = 0;
        // r lies in the first window (else the row left this kernel), or with
        // two windows in either
        const bool rlo = tiny && below_window(__float_as_uint(r), thr);
        const int64_t ra = rlo ? 0 : (int64_t)((double)r * sc);
        const int64_t ra1 = rlo ? (int64_t)((double)r * sc2) : 0;
        dS = 0;
        dQ = 0;
        dS1 = 0;
        dQ1 = 0;
        auto apply_one = [&](int i) {
            const float x = get(i);
            const bool f = x < Lo || x > H;
            if (f) {
                set(i, r);
                if (!tiny) {
                    const int64_t a = (int64_t)((double)x * sc);
                    dS += ra - a;
                    dQ += (u128)((i128)ra * ra) - (u128)((i128)a * a);
                } else {
                    const bool xlo = below_window(__float_as_uint(x), thr);
                    const int64_t a = xlo ? 0 : (int64_t)((double)x * sc);
                    const int64_t a1 = xlo ? (int64_t)((double)x * sc2) : 0;
                    dS += ra - a;
                    dQ += (u128)((i128)ra * ra) - (u128)((i128)a * a);
                    dS1 += ra1 - a1;
                    dQ1 += (u128)((i128)ra1 * ra1) - (u128)((i128)a1 * a1);
                }
            }
            cnt += f ? 1u : 0u;
        };
        if (full) {
#pragma unroll
            for (int i = 0; i < VPT; i++) apply_one(i);
        } else {
#pragma unroll
            for (int i = 0; i < VPT; i++)
                if (i < nv) apply_one(i);
        }
        cnt = wave_add_u32(cnt);
        if (lane == 0 && cnt) atomicAdd(&s_cnt[j], cnt);
    }
    __syncthreads();
    if (bad || to_two) {
        if (tid == 0) {
            const unsigned slot = atomicAdd(bad ? wide_n : tiny_n, 1u);
            (bad ? wide_items : tiny_items)[slot] = make_int2(bm.pad, (int)c);
        }
    } else if (counts && tid < seg.n_td && s_cnt[tid]) {
        atomicAdd(&counts[(int64_t)bm.cidx * count_stride + seg.td[tid].ci], (unsigned long long)s_cnt[tid]);
    }
    __syncthreads();   // the work-group's LDS is reused by the next row
}

template <int NT, int VPT, int VL>
__global__ __launch_bounds__(NT) void k_td_rows_f32(const DevBeam* __restrict__ beams, int nbeams, Segment seg,
                                                    float4* __restrict__ rec, unsigned* __restrict__ tiny_n,
                                                    int2* __restrict__ tiny_items, unsigned* __restrict__ wide_n,
                                                    int2* __restrict__ wide_items,
                                                    unsigned long long* __restrict__ counts, int count_stride) {
    const int64_t g = blockIdx.x;
    const int b = find_beam_by_row(beams, nbeams, g);
    const DevBeam& bm = beams[b];
    td_row_f32<NT, VPT, VL, false>(bm, g - bm.row0, seg, rec, tiny_n, tiny_items, wide_n, wide_items, counts,
                                   count_stride);
}

// Rows the fast kernel listed (values below its window): both windows, any
// row length the largest shape holds; a persistent grid walks the list.
__global__ __launch_bounds__(1024) void k_td_two_f32(const DevBeam* __restrict__ all, Segment seg,
                                                     float4* __restrict__ rec, const unsigned* __restrict__ tiny_n,
                                                     const int2* __restrict__ tiny_items,
                                                     unsigned* __restrict__ wide_n, int2* __restrict__ wide_items,
                                                     unsigned long long* __restrict__ counts, int count_stride) {
    const unsigned n = *tiny_n;
    for (unsigned it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 item = tiny_items[it];
        td_row_f32<1024, 64, 32, true>(all[item.x], item.y, seg, rec, nullptr, nullptr, wide_n, wide_items, counts,
                                       count_stride);
    }
}

// ---------------------------------------------------------------------------
// TD apply + FD steps on an LDS tile, one work-group per (beam, time tile)
// ---------------------------------------------------------------------------
namespace {

constexpr int kF32Block = 256;
constexpr int kF32Exc = 1024;   // TD exceptions listed per fused tile (4 KB: two 78 KB tiles fit a CU)

struct F32Tile {
    const float* in;
    float* out;
    uint8_t* flags;
    const float4* rec;   // this beam's composite TD records, [row][n_td]
    const float2* fast;  // this beam's innermost kept interval per row
    int64_t C, T, stride, t0;
    int Tt, Cp, nt, n_td;
};

// lower median (rank (B-1)/2 in totalOrder) of B register values
template <int B>
__device__ inline float bin_median(const float (&x)[B]) {
    uint32_t k[B];
#pragma unroll
    for (int i = 0; i < B; i++) k[i] = f32_key(__float_as_uint(x[i]));
#pragma unroll
    for (int size = 2; size <= B; size <<= 1) {
#pragma unroll
        for (int stride = size / 2; stride > 0; stride >>= 1) {
#pragma unroll
            for (int i = 0; i < B; i++) {
                const int j = i ^ stride;
                if (j > i) {
                    const uint32_t a = k[i], bb = k[j];
                    const bool up = (i & size) == 0;
                    k[i] = up ? min(a, bb) : max(a, bb);
                    k[j] = up ? max(a, bb) : min(a, bb);
                }
            }
        }
    }
    return __uint_as_float(key_f32(k[(B - 1) / 2]));
}

// Sum over G lanes (xor groups) of the low four 64-bit limbs of a U512.
__device__ inline U512 group_add_u256(U512 v, int G) {
    for (int o = 1; o < G; o <<= 1) {
        uint64_t w[4];
#pragma unroll
        for (int i = 0; i < 4; i++) w[i] = __shfl_xor(v.w[i], o, 64);
        u128 c = 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            c += (u128)v.w[i] + w[i];
            v.w[i] = (uint64_t)c;
            c >>= 64;
        }
    }
    return v;
}

// Every FD step of the run on one time sample held by a group of G2 lanes:
// lane's bins are x[kk] (B values each, act[kk] when the bin exists), flag
// bytes collect in fw, per-step counts in lc (16 bits per step).  TWO:
// statistics in both windows.  Returns 0 when done, 1 when the time sample
// needs the wide path (values below the last window), 2 (TWO = false only)
// when it needs the two-window kernel; x is then not final.
template <int B, int BPL, bool TWO, bool WAVE = false>
__device__ inline int fd_column_f32(float (&x)[BPL][B], uint32_t (&fw)[BPL][B / 4], const bool (&act)[BPL], int G2,
                                    uint32_t C, const Segment& seg, uint64_t lc[4]) {
    uint32_t emax = 0, tmin = 0xFFFFFFFFu;
#pragma unroll
    for (int kk = 0; kk < BPL; kk++)
#pragma unroll
        for (int j = 0; j < B; j++) {
            const uint32_t bb = __float_as_uint(x[kk][j]) & 0x7FFFFFFFu;
            emax = max(emax, bb);
            tmin = min(tmin, bb - 1u);
        }
    if constexpr (WAVE) {   // one time sample per wave (G2 == 64)
        emax = wave_max_dpp(emax);
        tmin = wave_min_u32(tmin);
    } else {
        emax = group_max_u32(emax, G2);
        tmin = group_min_u32(tmin, G2);
    }
    const int EM = f32_E(emax);
    const uint32_t thr = window_thr(EM), thr2 = window_thr2(EM);
    if (tmin != 0xFFFFFFFFu && tmin + 1u < thr2) return 1;
    if (!TWO && tmin != 0xFFFFFFFFu && tmin + 1u < thr) return 2;
    const double sc = ldexp(1.0, 174 - EM), sc2 = ldexp(1.0, 198 - EM);
    const int e = TWO ? EM - 198 : EM - 174;
    lc[0] = lc[1] = lc[2] = lc[3] = 0;
    // Bin medians, kept across median steps: replacing a bin's cut samples by
    // its lower median leaves that value the lower median (the counts on
    // either side only shrink), so once taken it stays valid until a mean step
    // changes the bin.  When any lane of the wave first needs one, every lane
    // takes all of its bins' medians at once (the sorting network runs once
    // per wave instead of once per step).
    float medc[BPL];
    bool medv = false;   // wave-uniform
    for (int s = 0; s < seg.n_fd; s++) {
        const SegStep& st = seg.fd[s];
        i128 S[BPL];
        u128 z = 0, Rv = 0;
        U512 Vw = u512_from(0);   // two windows: the sum of Z^2 (in second-window units)
        double zr = 0.0;
        if (!TWO) {
            u128 V = 0;
#pragma unroll
            for (int kk = 0; kk < BPL; kk++) {
                // recomputed every step: replacements reach most waves, and an
                // update by the replaced samples costs more (128-bit squares
                // under divergence) than one exact pass over the bin
                int64_t Sb = 0;
                u128 Qb = 0;
#pragma unroll
                for (int j0 = 0; j0 < B; j0 += 32) {
                    WinAcc w{0.0, 0.0, 0.0};
#pragma unroll
                    for (int j = j0; j < (j0 + 32 < B ? j0 + 32 : B); j++) winacc_add(w, (double)x[kk][j] * sc);
                    Sb += (int64_t)w.s;
                    Qb += winacc_q(w);
                }
                S[kk] = Sb;
                const u128 Sa = Sb < 0 ? (u128)(-(i128)Sb) : (u128)Sb;
                if (act[kk]) V += (u128)B * Qb - Sa * Sa;
            }
            if constexpr (WAVE) V = wave_add_u128(V);
            else V = group_add_u128(V, G2);
            // sum over the time sample of Z_c^2 = B * sum_b (B*Q_b - S_b^2);
            // the integer radius z is only needed where the FP64 cut is not
            // certified (below)
            Rv = (u128)B * V;
            zr = st.kx.mode == 0 ? st.kx.k * sqrt(u128_to_double(Rv) / (double)C) : 0.0;
        } else {
            U512 V = u512_from(0);
#pragma unroll
            for (int kk = 0; kk < BPL; kk++) {
                int64_t S0 = 0, S1 = 0;
                u128 Q0 = 0, Q1 = 0;
#pragma unroll
                for (int j0 = 0; j0 < B; j0 += 32) {
                    WinAcc w{0.0, 0.0, 0.0}, w1{0.0, 0.0, 0.0};
#pragma unroll
                    for (int j = j0; j < (j0 + 32 < B ? j0 + 32 : B); j++) {
                        const bool lo = below_window(__float_as_uint(x[kk][j]), thr);
                        winacc_add(w, lo ? 0.0 : (double)x[kk][j] * sc);
                        winacc_add(w1, lo ? (double)x[kk][j] * sc2 : 0.0);
                    }
                    S0 += (int64_t)w.s;
                    Q0 += winacc_q(w);
                    S1 += (int64_t)w1.s;
                    Q1 += winacc_q(w1);
                }
                // units of the second window: S = S0 * 2^24 + S1, Q = Q0 * 2^48 + Q1
                S[kk] = (i128)S0 * ((i128)1 << 24) + S1;
                if (act[kk]) V = u512_add(V, d_combine(B, q_combine(Q0, Q1), S[kk]));
            }
            V = group_add_u256(V, G2);
            Vw = u512_mul_u128(V, (u128)B);
            zr = st.kx.mode == 0 ? st.kx.k * sqrt(u512_to_double(Vw) / (double)C) : 0.0;
        }
        const int bit = st.bit;
        uint32_t bad = 0;
        // cut interval per bin: certified FP64 evaluation, else exact
        float Hs[BPL], Los[BPL];
        bool cert[BPL];
        bool need = false;
#pragma unroll
        for (int kk = 0; kk < BPL; kk++) {
            cert[kk] = false;
            Hs[kk] = Los[kk] = 0.0f;
            if (st.kx.mode == 0 && act[kk])
                cert[kk] = f32_cut_fast(TWO ? i128_to_double(S[kk]) : (double)(int64_t)S[kk], zr, (double)B, e,
                                        &Hs[kk], &Los[kk]);
            need |= act[kk] && !cert[kk];
        }
        if (need) {
            z = TWO ? zmax_k2w(C, Vw, st.kx, kZcap2) : zmax_k2(C, Rv, st.kx, kZcap);
#pragma unroll
            for (int kk = 0; kk < BPL; kk++) {
                if (!act[kk] || cert[kk]) continue;
                Hs[kk] = f32_round_ratio(S[kk] + (i128)z, B, e, kRD);
                Los[kk] = f32_round_ratio(S[kk] - (i128)z, B, e, kRU);
            }
        }
        uint64_t fms[BPL];
        bool anyf = false;
#pragma unroll
        for (int kk = 0; kk < BPL; kk++) {
            uint64_t fm = 0;
            const float H = Hs[kk], Lo = Los[kk];
#pragma unroll
            for (int j = 0; j < B; j++) fm |= (uint64_t)(x[kk][j] < Lo || x[kk][j] > H) << j;
            fms[kk] = act[kk] ? fm : 0;
            anyf |= fms[kk] != 0;
        }
        const bool wave_cut = __ballot(anyf) != 0;
        if (st.replace == RFIM_REPLACE_MEDIAN && wave_cut && !medv) {
#pragma unroll
            for (int kk = 0; kk < BPL; kk++) medc[kk] = bin_median<B>(x[kk]);
            medv = true;
        }
        if (st.replace != RFIM_REPLACE_MEDIAN && wave_cut) medv = false;
#pragma unroll
        for (int kk = 0; kk < BPL; kk++) {
            if (!act[kk]) continue;
            const uint64_t fm = fms[kk];
            if (!fm) continue;
            float r;
            if (st.replace == RFIM_REPLACE_MEDIAN) r = medc[kk];
            else if (!f32_mean_fast(TWO ? i128_to_double(S[kk]) : (double)(int64_t)S[kk], (double)B, e, &r))
                r = f32_round_ratio(S[kk], B, e, kRN);
            if (below_window(__float_as_uint(r), thr2)) bad |= 1u;
            else if (!TWO && below_window(__float_as_uint(r), thr)) bad |= 2u;
#pragma unroll
            for (int j = 0; j < B; j++) {
                const bool f = (fm >> j) & 1;
                x[kk][j] = f ? r : x[kk][j];
                if (bit >= 0 && f) fw[kk][j / 4] |= (1u << bit) << (8 * (j % 4));
            }
            lc[s >> 2] += (uint64_t)__popcll(fm) << (16 * (s & 3));
        }
        if constexpr (WAVE) bad = wave_or_dpp(bad);
        else bad = group_or_u32(bad, G2);
        if (bad) return (bad & 1u) ? 1 : 2;
    }
    return 0;
}

// All FD steps for the time samples of this wave.  B channels per bin, BPL
// bins per lane, groups of G2 lanes per time sample.
template <int B, int BPL>
__device__ void fd_fast_f32(const F32Tile& k, const Segment& seg, float* tile, uint8_t* ftile, bool want_flags,
                            unsigned* tiny_n, int2* tiny_items, unsigned* wide_n, int2* wide_items, int gidx,
                            uint64_t cntp[4]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = kF32Block / 64;
    const int nbins = (int)(k.C / B);
    const int G2 = nbins > 64 ? 64 : pow2_ceil(nbins);
    const int CPW = 64 / G2;
    const int cw = lane / G2, gl = lane % G2;
    const int ncg = (k.nt + CPW - 1) / CPW;
    const uint32_t C = (uint32_t)k.C;
    for (int cg = wave; cg < ncg; cg += NW) {
        const int t = cg * CPW + cw;
        const bool colok = t < k.nt;
        float x[BPL][B];
        uint32_t fw[BPL][B / 4];
        bool act[BPL];
#pragma unroll
        for (int kk = 0; kk < BPL; kk++) {
            const int bin = gl + 64 * kk;
            act[kk] = colok && bin < nbins;
            const float* p = tile + (size_t)(colok ? t : 0) * k.Cp + (size_t)(act[kk] ? bin : 0) * (B + 4);
#pragma unroll
            for (int j = 0; j < B; j += 4) {
                const float4 q = act[kk] ? *(const float4*)(p + j) : make_float4(0.f, 0.f, 0.f, 0.f);
                x[kk][j] = q.x;
                x[kk][j + 1] = q.y;
                x[kk][j + 2] = q.z;
                x[kk][j + 3] = q.w;
            }
#pragma unroll
            for (int j = 0; j < B / 4; j++) fw[kk][j] = 0;
        }
        uint64_t lc[4];
        // two bins per lane means more than 64 bins: one time sample per wave
        const int res = fd_column_f32<B, BPL, false, BPL == 2>(x, fw, act, G2, C, seg, lc);
        if (!colok) continue;
        if (res) {
            // the tile keeps this time sample's post-TD values for the other kernel
            if (gl == 0) {
                unsigned* cnt = res == 1 ? wide_n : tiny_n;
                const unsigned slot = atomicAdd(cnt, 1u);
                (res == 1 ? wide_items : tiny_items)[slot] = make_int2(gidx, (int)(k.t0 + t));
            }
            continue;
        }
#pragma unroll
        for (int i = 0; i < 4; i++) cntp[i] += lc[i];
#pragma unroll
        for (int kk = 0; kk < BPL; kk++) {
            if (!act[kk]) continue;
            const int bin = gl + 64 * kk;
            float* p = tile + (size_t)t * k.Cp + (size_t)bin * (B + 4);
#pragma unroll
            for (int j = 0; j < B; j += 4) *(float4*)(p + j) = make_float4(x[kk][j], x[kk][j + 1], x[kk][j + 2], x[kk][j + 3]);
            if (want_flags) {
                uint32_t* fp = (uint32_t*)(ftile + (size_t)t * k.C + (size_t)bin * B);
#pragma unroll
                for (int j = 0; j < B / 4; j++) fp[j] |= fw[kk][j];
            }
        }
    }
}

__device__ inline int64_t phys_chan(int64_t c, int B) { return B ? c + (c / B) * 4 : c; }

}  // namespace

// Composite TD records of a run, one thread per float32 row, after every TD
// kernel of the run has written its raw records (Lo_j, H_j, r_j): in place,
// (Lc_j, Hc_j, v_j, bits_j) with [Lc_j, Hc_j] the intersection of the kept
// intervals of steps 0..j (a value inside it is untouched through step j),
// v_j the value a sample first cut at step j ends with (r_j, then replaced
// again by any later step that cuts it) and bits_j the flag bits it collects;
// fast[row] = the innermost interval [Lc, Hc] of the last step.
__global__ void k_td_compose_f32(float4* __restrict__ rec, float2* __restrict__ fast, int64_t rows, Segment seg) {
    const int n = seg.n_td;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        float4 raw[kMaxSteps];
        float4* rp = rec + r * n;
        for (int j = 0; j < n; j++) raw[j] = rp[j];
        float Lc = -INFINITY, Hc = INFINITY;
        for (int j = 0; j < n; j++) {
            Lc = fmaxf(Lc, raw[j].x);
            Hc = fminf(Hc, raw[j].y);
            float v = raw[j].z;
            uint32_t bits = seg.td[j].bit >= 0 ? 1u << seg.td[j].bit : 0u;
            for (int kk = j + 1; kk < n; kk++) {
                if (v < raw[kk].x || v > raw[kk].y) {
                    v = raw[kk].z;
                    if (seg.td[kk].bit >= 0) bits |= 1u << seg.td[kk].bit;
                }
            }
            rp[j] = make_float4(Lc, Hc, v, __uint_as_float(bits));
        }
        fast[r] = make_float2(Lc, Hc);
    }
}

hipError_t launch_td_compose_f32(float4* rec, float2* fast, int64_t rows, const Segment& seg, hipStream_t s) {
    if (rows <= 0 || seg.n_td == 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((rows + 255) / 256, 2048);
    hipLaunchKernelGGL(k_td_compose_f32, dim3(blocks), dim3(256), 0, s, rec, fast, rows, seg);
    return hipGetLastError();
}

// B = bin size of the fast FD path (0: no fast FD; every time sample of a run
// with FD steps then goes to the wide list).  BPL = bins per lane.
template <int B, int BPL>
__global__ __launch_bounds__(kF32Block) void k_fused_f32(const DevBeam* __restrict__ beams, int nbeams,
                                                         int64_t total_tiles, Segment seg,
                                                         const float4* __restrict__ rec,
                                                         const float2* __restrict__ fast,
                                                         unsigned* __restrict__ tiny_n, int2* __restrict__ tiny_items,
                                                         unsigned* __restrict__ wide_n, int2* __restrict__ wide_items,
                                                         unsigned long long* __restrict__ counts, int count_stride) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ unsigned long long s_cnt[kMaxSteps];
    __shared__ uint32_t s_exc[kF32Exc];   // (row << 8) | tile sample of the values a TD step cuts
    __shared__ uint32_t s_exc_n;
    const int tid = threadIdx.x;
    const int64_t g = xcd_remap(blockIdx.x, total_tiles);
    const int b = find_beam_by_tile(beams, nbeams, g);
    const DevBeam& bm = beams[b];
    F32Tile k;
    k.in = (const float*)bm.in;
    k.out = (float*)bm.out;
    k.flags = bm.flags;
    k.C = bm.C;
    k.T = bm.T;
    k.stride = bm.stride;
    k.Tt = bm.Tt;
    k.Cp = bm.Cp;
    k.t0 = (g - bm.tile0) * k.Tt;
    k.nt = (int)min((int64_t)k.Tt, k.T - k.t0);
    k.n_td = seg.n_td;
    k.rec = rec + bm.rec0 * seg.n_td;
    k.fast = fast + bm.rec0;
    const bool want_flags = seg.flags_mode != 0 && bm.flags != nullptr;
    const bool or_flags = seg.flags_mode == 2;
    const bool vec = (k.stride & 3) == 0 && (((uintptr_t)k.in | (uintptr_t)k.out) & 15) == 0;
    float* tile = (float*)lds;
    uint8_t* ftile = lds + (size_t)k.Tt * k.Cp * 4;
    const int tq_log = __ffs(k.Tt >> 2) - 1;   // 4-sample quads per tile row: a power of two
    const int TQ = 1 << tq_log;
    const int nitems = (int)k.C << tq_log;     // below 2^31: C < 2^24, Tt <= 64
    if (tid < kMaxSteps) s_cnt[tid] = 0;
    if (tid == 0) s_exc_n = 0;
    __syncthreads();

    // ---- phase 1: rows in, TD applied, into LDS (B > 0) or straight out.
    // The TD steps' composite records nest, so a value inside the row's
    // innermost kept interval is untouched by every step: one compare pair per
    // value.  Values outside it (rare) take the first step whose interval
    // excludes them: listed in LDS and mapped after the loop by all threads
    // together (their record loads in flight at once); past the list's
    // capacity, and when the tile goes straight out, mapped in place.  kB1
    // items per thread have their row loads and interval loads in flight
    // together.
    // 16 items (a 4096-channel tile's whole share of a thread) keep about
    // 64 KB of loads in flight per CU-resident work-group pair; four left the
    // phase waiting on memory latency.
    constexpr int kB1 = 16;
    for (int it0 = tid; it0 < nitems; it0 += kB1 * kF32Block) {
        float xs[kB1][4];
        float2 fr[kB1];
        int cs[kB1], qs[kB1];
        bool oks[kB1];
        // the batch's loads go out at raised wave priority (the other
        // work-group on the CU is then usually in its FD phase)
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int u = 0; u < kB1; u++) {
            const int it = it0 + u * kF32Block;
            const int c = it >> tq_log;
            const int q = it & (TQ - 1);
            const int64_t t = k.t0 + 4 * q;
            cs[u] = c;
            qs[u] = q;
            oks[u] = it < nitems && t < k.T;
            fr[u] = make_float2(-INFINITY, INFINITY);
            if (!oks[u]) continue;
            const float* p = k.in + (int64_t)c * k.stride + t;
            if (vec && t + 3 < k.T) {
                const float4 f = *(const float4*)p;
                xs[u][0] = f.x;
                xs[u][1] = f.y;
                xs[u][2] = f.z;
                xs[u][3] = f.w;
            } else {
#pragma unroll
                for (int jj = 0; jj < 4; jj++) xs[u][jj] = t + jj < k.T ? p[jj] : 0.0f;
            }
            if (k.n_td > 0) fr[u] = k.fast[c];
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int u = 0; u < kB1; u++) {
            if (!oks[u]) continue;
            const int c = cs[u];
            const int q = qs[u];
            const int64_t t = k.t0 + 4 * q;
            float* x = xs[u];
            uint32_t fb[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int uu = 0; uu < 4; uu++) {
                if (!(x[uu] < fr[u].x || x[uu] > fr[u].y)) continue;
                if (B > 0) {
                    const uint32_t slot = atomicAdd(&s_exc_n, 1u);
                    if (slot < (uint32_t)kF32Exc) {
                        s_exc[slot] = ((uint32_t)c << 8) | (uint32_t)(4 * q + uu);
                        continue;   // mapped after the loop
                    }
                }
                // the first step whose composite interval excludes x decides
                const float4* rp = k.rec + (int64_t)c * k.n_td;
                for (int j = 0; j < k.n_td; j++) {
                    const float4 r4 = rp[j];
                    if (x[uu] < r4.x || x[uu] > r4.y) {
                        x[uu] = r4.z;
                        fb[uu] = __float_as_uint(r4.w);
                        break;
                    }
                }
            }
            if (want_flags && or_flags) {
                const uint8_t* fp = k.flags + (int64_t)c * k.stride + t;
#pragma unroll
                for (int uu = 0; uu < 4; uu++)
                    if (t + uu < k.T) fb[uu] |= fp[uu];
            }
            if (B > 0) {
                const int pc = (int)phys_chan(c, B);
#pragma unroll
                for (int uu = 0; uu < 4; uu++) tile[(4 * q + uu) * k.Cp + pc] = x[uu];
                if (want_flags) {
#pragma unroll
                    for (int uu = 0; uu < 4; uu++) ftile[(4 * q + uu) * (int)k.C + c] = (uint8_t)fb[uu];
                }
            } else {
                float* op = k.out + (int64_t)c * k.stride + t;
                if (vec && t + 3 < k.T) {
                    *(float4*)op = make_float4(x[0], x[1], x[2], x[3]);
                } else {
#pragma unroll
                    for (int uu = 0; uu < 4; uu++)
                        if (t + uu < k.T) op[uu] = x[uu];
                }
                if (want_flags) {
                    uint8_t* fp = k.flags + (int64_t)c * k.stride + t;
#pragma unroll
                    for (int uu = 0; uu < 4; uu++)
                        if (t + uu < k.T) fp[uu] = (uint8_t)fb[uu];
                }
            }
        }
    }
    if (B > 0 && k.n_td > 0) {
        __syncthreads();   // the tile and the list are complete
        const uint32_t ne = min(s_exc_n, (uint32_t)kF32Exc);
        for (uint32_t e = tid; e < ne; e += kF32Block) {
            const uint32_t pos = s_exc[e];
            const int c = (int)(pos >> 8), ts = (int)(pos & 255u);
            const int pc = (int)phys_chan(c, B);
            float x = tile[ts * k.Cp + pc];
            uint32_t bits = 0;
            const float4* rp = k.rec + (int64_t)c * k.n_td;
            for (int j = 0; j < k.n_td; j++) {
                const float4 r4 = rp[j];
                if (x < r4.x || x > r4.y) {
                    x = r4.z;
                    bits = __float_as_uint(r4.w);
                    break;
                }
            }
            tile[ts * k.Cp + pc] = x;
            if (want_flags) ftile[ts * (int)k.C + c] |= (uint8_t)bits;
        }
    }
    if (B == 0) {
        // no fast FD for this beam: every time sample of the tile goes wide
        if (seg.n_fd > 0)
            for (int t = tid; t < k.nt; t += kF32Block) {
                const unsigned slot = atomicAdd(wide_n, 1u);
                wide_items[slot] = make_int2(bm.pad, (int)(k.t0 + t));
            }
        return;
    }
    __syncthreads();

    // ---- phase 2: FD steps
    uint64_t cntp[4] = {0, 0, 0, 0};
    if (seg.n_fd > 0) {
        if constexpr (B > 0)
            fd_fast_f32<B, BPL>(k, seg, tile, ftile, want_flags, tiny_n, tiny_items, wide_n, wide_items, bm.pad, cntp);
    }
    __syncthreads();

    // ---- phase 3: tile back to rows (sixteen items per thread per pass: their
    // LDS reads are issued together)
#pragma unroll 16
    for (int it = tid; it < nitems; it += kF32Block) {
        const int c = it >> tq_log;
        const int q = it & (TQ - 1);
        const int64_t t = k.t0 + 4 * q;
        if (t >= k.T) continue;
        const int pc = (int)phys_chan(c, B);
        float x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) x[u] = tile[(4 * q + u) * k.Cp + pc];
        float* op = k.out + (int64_t)c * k.stride + t;
        if (vec && t + 3 < k.T) {
            *(float4*)op = make_float4(x[0], x[1], x[2], x[3]);
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (t + u < k.T) op[u] = x[u];
        }
        if (want_flags) {
            uint8_t* fp = k.flags + (int64_t)c * k.stride + t;
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (t + u < k.T) fp[u] = ftile[(4 * q + u) * (int)k.C + c];
        }
    }
    if (counts && seg.n_fd > 0) {
        // per-step counts of this lane (16-bit fields), wave sums, then global
        for (int s = 0; s < seg.n_fd; s++) {
            const uint32_t v = (uint32_t)((cntp[s >> 2] >> (16 * (s & 3))) & 0xFFFFu);
            const uint32_t tot = wave_add_u32(v);
            if ((tid & 63) == 0 && tot) atomicAdd(&s_cnt[s], (unsigned long long)tot);
        }
        __syncthreads();
        if (tid < seg.n_fd && s_cnt[tid])
            atomicAdd(&counts[(int64_t)bm.cidx * count_stride + seg.fd[tid].ci], s_cnt[tid]);
    }
}

// Time samples the fused kernel listed (values below its window): every FD
// step in both windows, one wave per time sample read from the output (post-TD
// values), written back with the flag bits ORed in.  Launched once per fast
// bin shape; items of beams with another shape are left to their launch.
template <int B, int BPL>
__global__ __launch_bounds__(kF32Block) void k_fd_two_f32(const DevBeam* __restrict__ all, Segment seg,
                                                          const unsigned* __restrict__ tiny_n,
                                                          const int2* __restrict__ tiny_items,
                                                          unsigned* __restrict__ wide_n, int2* __restrict__ wide_items,
                                                          unsigned long long* __restrict__ counts, int count_stride) {
    constexpr int NW = kF32Block / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned n = *tiny_n;
    for (unsigned it = blockIdx.x * NW + wave; it < n; it += gridDim.x * NW) {
        const int2 item = tiny_items[it];
        const DevBeam& bm = all[item.x];
        if (bm.Tt != B || bm.Cp != BPL) continue;   // another launch's shape
        const int64_t t = item.y;
        const int nbins = (int)(bm.C / B);
        const int G2 = nbins > 64 ? 64 : pow2_ceil(nbins);
        float* out = (float*)bm.out;
        const bool want_flags = seg.flags_mode != 0 && bm.flags != nullptr;
        float x[BPL][B];
        uint32_t fw[BPL][B / 4];
        bool act[BPL];
#pragma unroll
        for (int kk = 0; kk < BPL; kk++) {
            const int bin = lane + 64 * kk;
            act[kk] = lane < G2 && bin < nbins;
#pragma unroll
            for (int j = 0; j < B; j++) x[kk][j] = act[kk] ? out[((int64_t)bin * B + j) * bm.stride + t] : 0.0f;
#pragma unroll
            for (int j = 0; j < B / 4; j++) fw[kk][j] = 0;
        }
        uint64_t lc[4];
        const int res = fd_column_f32<B, BPL, true>(x, fw, act, G2, (uint32_t)bm.C, seg, lc);
        if (res) {
            if (lane == 0) {
                const unsigned slot = atomicAdd(wide_n, 1u);
                wide_items[slot] = make_int2(item.x, (int)t);
            }
            continue;
        }
#pragma unroll
        for (int kk = 0; kk < BPL; kk++) {
            if (!act[kk]) continue;
            const int bin = lane + 64 * kk;
#pragma unroll
            for (int j = 0; j < B; j++) {
                const int64_t off = ((int64_t)bin * B + j) * bm.stride + t;
                out[off] = x[kk][j];
                const uint32_t f = (fw[kk][j / 4] >> (8 * (j % 4))) & 255u;
                if (want_flags && f) bm.flags[off] |= (uint8_t)f;
            }
        }
        if (counts) {
            for (int sidx = 0; sidx < seg.n_fd; sidx++) {
                const uint32_t v = (uint32_t)((lc[sidx >> 2] >> (16 * (sidx & 3))) & 0xFFFFu);
                const uint32_t tot = wave_add_u32(v);
                if (lane == 0 && tot)
                    atomicAdd(&counts[(int64_t)bm.cidx * count_stride + seg.fd[sidx].ci], (unsigned long long)tot);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Wide fallback kernels: work lists of rows / time samples, big integers
// ---------------------------------------------------------------------------
namespace {

constexpr int kWideNT = 256;
constexpr int kAccW = 2 * kAccS + kAccQ;   // counters per thread: +S, -S, S2

// value x after the first m TD steps of the records r
__device__ inline float td_apply_prefix(float x, const float4* r, int m) {
    for (int j = 0; j < m; j++) x = (x < r[j].x || x > r[j].y) ? r[j].z : x;
    return x;
}

}  // namespace

__global__ __launch_bounds__(kWideNT) void k_td_wide_f32(const DevBeam* __restrict__ all,
                                                         const unsigned* __restrict__ wide_n,
                                                         const int2* __restrict__ items, Segment seg,
                                                         float4* __restrict__ rec,
                                                         unsigned long long* __restrict__ counts,
                                                         int count_stride) {
    __shared__ uint64_t s_acc[kWideNT * kAccW];
    __shared__ uint64_t s_tot[kAccW];
    __shared__ float4 s_rec[kMaxSteps];
    __shared__ uint32_t s_hist[(kWideNT / 64) * 256], s_tot4[kWideNT / 64], s_sel[2];
    __shared__ unsigned long long s_cnt;
    const int tid = threadIdx.x;
    const unsigned nitems = *wide_n;
    for (unsigned it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 item = items[it];
        const DevBeam& bm = all[item.x];
        const int64_t c = item.y;
        const int64_t T = bm.T;
        const float* row = (const float*)bm.in + c * bm.stride;
        const uint32_t n = (uint32_t)T;
        for (int j = 0; j < seg.n_td; j++) {
            const SegStep& st = seg.td[j];
            uint64_t* a = s_acc + tid * kAccW;
            for (int l = 0; l < kAccW; l++) a[l] = 0;
            for (int64_t i = tid; i < T; i += kWideNT)
                acc_add_f32(a, a + kAccS, a + 2 * kAccS, __float_as_uint(td_apply_prefix(row[i], s_rec, j)));
            __syncthreads();
            for (int l = tid; l < kAccW; l += kWideNT) {
                uint64_t t = 0;
                for (int th = 0; th < kWideNT; th++) t += s_acc[th * kAccW + l];
                s_tot[l] = t;
            }
            float med = 0.0f;
            if (st.replace == RFIM_REPLACE_MEDIAN) {
                const uint32_t key = wg_select_key<kWideNT>((uint64_t)(n - 1) / 2, s_hist, s_tot4, s_sel, [&](auto&& add) {
                    for (int64_t i = tid; i < T; i += kWideNT)
                        add(f32_key(__float_as_uint(td_apply_prefix(row[i], s_rec, j))));
                });
                med = __uint_as_float(key_f32(key));
            }
            __syncthreads();
            if (tid == 0) {
                Big P, N, S1, S2, D, t;
                big_from_counters(P, s_tot, kAccS);
                big_from_counters(N, s_tot + kAccS, kAccS);
                big_from_counters(S2, s_tot + 2 * kAccS, kAccQ);
                big_sub(S1, P, N);
                big_mul_u64(D, S2, n);
                big_mul(t, S1, S1);
                big_sub(D, D, t);
                float lo, hi;
                big_thresholds(S1, n, 1u, D, st.kx, &lo, &hi);
                const float r = st.replace == RFIM_REPLACE_MEDIAN ? med : big_round_ratio_f32(S1, n, kRN);
                s_rec[j] = make_float4(lo, hi, r, 0.0f);
                rec[(bm.rec0 + c) * seg.n_td + j] = s_rec[j];
                s_cnt = 0;
            }
            __syncthreads();
            uint32_t cnt = 0;
            const float4 rj = s_rec[j];
            for (int64_t i = tid; i < T; i += kWideNT) {
                const float x = td_apply_prefix(row[i], s_rec, j);
                cnt += (x < rj.x || x > rj.y) ? 1u : 0u;
            }
            cnt = wave_add_u32(cnt);
            if ((tid & 63) == 0 && cnt) atomicAdd(&s_cnt, (unsigned long long)cnt);
            __syncthreads();
            if (tid == 0 && counts && s_cnt)
                atomicAdd(&counts[(int64_t)bm.cidx * count_stride + st.ci], s_cnt);
            __syncthreads();
        }
    }
}

namespace {

// exact sums of bin values p[0..B) (stride 1): +S, -S and S2 counters to Bigs
__device__ inline void bin_sums_big(const float* p, int64_t B, Big& S, Big& Q) {
    uint64_t a[kAccW];
    for (int l = 0; l < kAccW; l++) a[l] = 0;
    for (int64_t i = 0; i < B; i++) acc_add_f32(a, a + kAccS, a + 2 * kAccS, __float_as_uint(p[i]));
    Big P, N;
    big_from_counters(P, a, kAccS);
    big_from_counters(N, a + kAccS, kAccS);
    big_from_counters(Q, a + 2 * kAccS, kAccQ);
    big_sub(S, P, N);
}

// lower median (rank (B-1)/2, totalOrder) of p[0..B): the largest key v with
// #{x : key(x) < v} <= rank, bit by bit
__device__ inline float bin_median_scan(const float* p, int64_t B) {
    const int64_t rank = (B - 1) / 2;
    uint32_t prefix = 0;
    for (int bit = 31; bit >= 0; bit--) {
        const uint32_t cand = prefix | (1u << bit);
        int64_t below = 0;
        for (int64_t i = 0; i < B; i++) below += f32_key(__float_as_uint(p[i])) < cand ? 1 : 0;
        if (below <= rank) prefix = cand;
    }
    return __uint_as_float(key_f32(prefix));
}

}  // namespace

__global__ __launch_bounds__(kWideNT) void k_fd_wide_f32(const DevBeam* __restrict__ all,
                                                         const unsigned* __restrict__ wide_n,
                                                         const int2* __restrict__ items, Segment seg,
                                                         unsigned long long* __restrict__ counts,
                                                         int count_stride) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ Big s_big[kWideNT / 4];
    __shared__ unsigned long long s_cnt;
    const int tid = threadIdx.x;
    const unsigned nitems = *wide_n;
    for (unsigned it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 item = items[it];
        const DevBeam& bm = all[item.x];
        const int64_t t = item.y;
        const int64_t C = bm.C;
        float* col = (float*)lds;
        uint8_t* fl = lds + (size_t)C * 4;
        const bool want_flags = seg.flags_mode != 0 && bm.flags != nullptr;
        float* out = (float*)bm.out;
        for (int64_t c = tid; c < C; c += kWideNT) {
            col[c] = out[c * bm.stride + t];
            fl[c] = 0;
        }
        __syncthreads();
        for (int s = 0; s < seg.n_fd; s++) {
            const SegStep& st = seg.fd[s];
            const int64_t B = st.bin == 0 ? C : st.bin;
            const int64_t nb = C / B;
            // sum over bins of B*Q_b - S_b^2; the sum of Z_c^2 is B times that
            Big acc, Sb, Qb, t1;
            big_zero(acc);
            for (int64_t bb = tid; bb < nb; bb += kWideNT) {
                bin_sums_big(col + bb * B, B, Sb, Qb);
                big_mul_u64(t1, Qb, (uint64_t)B);
                big_mul(Sb, Sb, Sb);
                big_sub(t1, t1, Sb);
                big_add(acc, acc, t1);
            }
            // reduce the per-thread Bigs: four at a time per slot
            for (int round = 0; round < 4; round++) {
                if ((tid & 3) == round) {
                    if (round == 0) s_big[tid >> 2] = acc;
                    else big_add(s_big[tid >> 2], s_big[tid >> 2], acc);
                }
                __syncthreads();
            }
            if (tid == 0) {
                for (int i = 1; i < kWideNT / 4; i++) big_add(s_big[0], s_big[0], s_big[i]);
                s_cnt = 0;
            }
            __syncthreads();
            Big R;
            big_mul_u64(R, s_big[0], (uint64_t)B);
            uint32_t cnt = 0;
            for (int64_t bb = tid; bb < nb; bb += kWideNT) {
                float* p = col + bb * B;
                bin_sums_big(p, B, Sb, Qb);
                float lo, hi;
                big_thresholds(Sb, (uint32_t)B, (uint32_t)C, R, st.kx, &lo, &hi);
                bool any = false;
                for (int64_t i = 0; i < B; i++) any |= p[i] < lo || p[i] > hi;
                if (!any) continue;
                const float r = st.replace == RFIM_REPLACE_MEDIAN ? bin_median_scan(p, B)
                                                                  : big_round_ratio_f32(Sb, (uint32_t)B, kRN);
                for (int64_t i = 0; i < B; i++) {
                    if (p[i] < lo || p[i] > hi) {
                        p[i] = r;
                        cnt++;
                        if (st.bit >= 0) fl[bb * B + i] |= (uint8_t)(1u << st.bit);
                    }
                }
            }
            cnt = wave_add_u32(cnt);
            if ((tid & 63) == 0 && cnt) atomicAdd(&s_cnt, (unsigned long long)cnt);
            __syncthreads();
            if (tid == 0 && counts && s_cnt)
                atomicAdd(&counts[(int64_t)bm.cidx * count_stride + st.ci], s_cnt);
            __syncthreads();
        }
        for (int64_t c = tid; c < C; c += kWideNT) {
            out[c * bm.stride + t] = col[c];
            if (want_flags && fl[c]) bm.flags[c * bm.stride + t] |= fl[c];
        }
        __syncthreads();
    }
}

// appends items (gidx, 0..n-1) to a wide list: every row (or time sample) of
// a beam that the fast kernels do not handle
__global__ void k_list_all(unsigned* __restrict__ wide_n, int2* __restrict__ items, int gidx, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned slot = atomicAdd(wide_n, 1u);
        items[slot] = make_int2(gidx, (int)i);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_td_rows_f32(const DevBeam* d_beams, int nbeams, int64_t total_rows, int nt, int vpt,
                              const Segment& seg, float4* rec, unsigned* tiny_n, int2* tiny_items, unsigned* wide_n,
                              int2* wide_items, unsigned long long* counts, int count_stride, hipStream_t s) {
    if (total_rows <= 0) return hipSuccess;
    const dim3 grid((unsigned)total_rows);
#define RFIM_TDF(NT_, VPT_, VL_)                                                                        \
    if (nt == NT_ && vpt == VPT_) {                                                                     \
        hipLaunchKernelGGL((k_td_rows_f32<NT_, VPT_, VL_>), grid, dim3(NT_), 0, s, d_beams, nbeams, seg, rec, \
                           tiny_n, tiny_items, wide_n, wide_items, counts, count_stride);              \
        return hipGetLastError();                                                                       \
    }
    RFIM_TDF(256, 1, 0)
    RFIM_TDF(256, 4, 0)
    RFIM_TDF(256, 16, 0)
    RFIM_TDF(1024, 8, 0)
    RFIM_TDF(1024, 16, 0)
    RFIM_TDF(1024, 32, 0)
    RFIM_TDF(1024, 64, 32)
#undef RFIM_TDF
    return hipErrorInvalidValue;
}

hipError_t launch_fused_f32(const DevBeam* d_beams, int nbeams, int64_t total_tiles, int B, int bpl,
                            const Segment& seg, const float4* rec, const float2* fast, size_t lds_bytes,
                            unsigned* tiny_n,
                            int2* tiny_items, unsigned* wide_n, int2* wide_items, unsigned long long* counts,
                            int count_stride, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)total_tiles);
#define RFIM_FF(B_, BPL_)                                                                              \
    if (B == B_ && bpl == BPL_) {                                                                      \
        hipLaunchKernelGGL((k_fused_f32<B_, BPL_>), grid, dim3(kF32Block), lds_bytes, s, d_beams, nbeams, \
                           total_tiles, seg, rec, fast, tiny_n, tiny_items, wide_n, wide_items, counts, \
                           count_stride);                                                              \
        return hipGetLastError();                                                                      \
    }
    RFIM_FF(0, 1)
    RFIM_FF(8, 1)
    RFIM_FF(8, 2)
    RFIM_FF(16, 1)
    RFIM_FF(16, 2)
    RFIM_FF(32, 1)
    RFIM_FF(32, 2)
    RFIM_FF(64, 1)
#undef RFIM_FF
    return hipErrorInvalidValue;
}

hipError_t launch_td_two_f32(const DevBeam* d_all, const unsigned* tiny_n, const int2* tiny_items, int grid,
                             const Segment& seg, float4* rec, unsigned* wide_n, int2* wide_items,
                             unsigned long long* counts, int count_stride, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_td_two_f32, dim3(grid), dim3(1024), 0, s, d_all, seg, rec, tiny_n, tiny_items, wide_n,
                       wide_items, counts, count_stride);
    return hipGetLastError();
}

hipError_t launch_fd_two_f32(const DevBeam* d_all, const unsigned* tiny_n, const int2* tiny_items, int grid, int B,
                             int bpl, const Segment& seg, unsigned* wide_n, int2* wide_items,
                             unsigned long long* counts, int count_stride, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
#define RFIM_F2(B_, BPL_)                                                                            \
    if (B == B_ && bpl == BPL_) {                                                                    \
        hipLaunchKernelGGL((k_fd_two_f32<B_, BPL_>), dim3(grid), dim3(kF32Block), 0, s, d_all, seg, tiny_n, \
                           tiny_items, wide_n, wide_items, counts, count_stride);                    \
        return hipGetLastError();                                                                    \
    }
    RFIM_F2(8, 1)
    RFIM_F2(8, 2)
    RFIM_F2(16, 1)
    RFIM_F2(16, 2)
    RFIM_F2(32, 1)
    RFIM_F2(32, 2)
    RFIM_F2(64, 1)
#undef RFIM_F2
    return hipErrorInvalidValue;
}

hipError_t launch_td_wide_f32(const DevBeam* d_all, const unsigned* wide_n, const int2* items, int grid,
                              const Segment& seg, float4* rec, unsigned long long* counts, int count_stride,
                              hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_td_wide_f32, dim3(grid), dim3(kWideNT), 0, s, d_all, wide_n, items, seg, rec, counts,
                       count_stride);
    return hipGetLastError();
}

hipError_t launch_fd_wide_f32(const DevBeam* d_all, const unsigned* wide_n, const int2* items, int grid,
                              int64_t max_C, const Segment& seg, unsigned long long* counts, int count_stride,
                              hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fd_wide_f32, dim3(grid), dim3(kWideNT), (size_t)max_C * 5, s, d_all, wide_n, items, seg,
                       counts, count_stride);
    return hipGetLastError();
}

hipError_t launch_list_all(unsigned* wide_n, int2* items, int gidx, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_list_all, dim3(blocks), dim3(256), 0, s, wide_n, items, gidx, n);
    return hipGetLastError();
}

}  // namespace rfim
