// Incoherent dedispersion and detection statistics for gfx950 (RFIm,
// arXiv:2001.03389: the search stage that consumes the mitigated beams,
// Section I and Eq. 2; Section V-A checks that a dispersed pulse stays
// detectable after mitigation).
//
//  * Delays (Eq. 2, host): channel c (0 = lowest) centred at
//    f_c = f_low + (c + 1/2) * bw trails the top channel's centre by
//    k_DM * DM * (f_c^-2 - f_top^-2) seconds, k_DM = 4.15e3 MHz^2 pc^-1 cm^3 s,
//    rounded to the nearest sample (ties to even), evaluated in FP64.
//  * k_dedisp_u8 / k_dedisp_f32: series[d][t] = sum over channels c in
//    ascending order of x[c][t + delay_d(c)], t < nout.  A work-group owns
//    1024 consecutive output samples of DB consecutive DM trials; channels
//    are staged through LDS a few at a time, each channel's segment starting
//    at the block's smallest delay for it, so every trial of the block reads
//    the same staged bytes.  uint8: exact integer sums (int32 output), with
//    two outputs per 32-bit register in 16-bit fields inside a staged chunk;
//    float32: FP64 sums in channel order (bit-identical to a sequential FP64
//    loop over the channels).
//  * k_series_stats_*: per series, one work-group: mean, population standard
//    deviation, the largest value and its first index, and
//    SNR = (peak - mean) / std (0 for a constant series).  int32 series:
//    exact integer sums; float64 series: two passes in FP64.
//
// The path is adds and LDS reads (about DB * 1024 per staged channel and
// work-group against 1024 + spread staged samples); HBM traffic is one read
// of the beam per DM block and one write of the series.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "rfim_dev.h"
#include "rfim_exact.h"

namespace rfim {
namespace {

constexpr int kDdThreads = 256;
constexpr int kDdVT = 4;                    // consecutive output samples per thread
constexpr int kDdTT = kDdThreads * kDdVT;   // output samples per work-group
constexpr size_t kDdLds = 49152;            // staging bytes per work-group
constexpr double kKDM = 4.15e3;             // MHz^2 pc^-1 cm^3 s (Eq. 2)
constexpr int kDbU8 = 16;                   // DM trials per work-group (uint8)
constexpr int kDbF32 = 4;                   // DM trials per work-group (float32)

// uint8: DB trials x 4 outputs per thread; seg holds nc staged channel
// segments of L bytes (L a multiple of 4 with 8 bytes of slack past the last
// byte any thread reads).
template <int DB>
__global__ __launch_bounds__(kDdThreads) void k_dedisp_u8(const uint8_t* __restrict__ x, int64_t C, int64_t stride,
                                                          int64_t nsamp, const int32_t* __restrict__ base,
                                                          const int32_t* __restrict__ off, int ndm, int64_t nout,
                                                          int L, int CC, int32_t* __restrict__ series) {
    extern __shared__ __align__(16) uint32_t seg[];
    const int tid = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kDdTT;
    const int blk = blockIdx.y;
    const int32_t* bb = base + (int64_t)blk * C;
    const int32_t* oo = off + (int64_t)blk * C * DB;
    uint32_t acc[DB][4];
#pragma unroll
    for (int d = 0; d < DB; d++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc[d][v] = 0;
    for (int64_t c0 = 0; c0 < C; c0 += CC) {
        const int nc = (int)min((int64_t)CC, C - c0);
        __syncthreads();   // the previous chunk's reads are done
        for (int j = 0; j < nc; j++) {
            const int64_t s0 = t0 + bb[c0 + j];     // < nsamp: nout + the largest delay <= nsamp
            const uint8_t* row = x + (c0 + j) * stride + s0;
            const int64_t avail = nsamp - s0;
            uint8_t* dst = (uint8_t*)seg + (size_t)j * L;
            for (int i = tid; i < L; i += kDdThreads) dst[i] = i < avail ? ld_global<uint8_t>(row + i) : (uint8_t)0;
        }
        __syncthreads();
        // 16-bit fields: at most CC <= 257 bytes of 255 each per field
        uint32_t p02[DB], p13[DB];
#pragma unroll
        for (int d = 0; d < DB; d++) p02[d] = p13[d] = 0;
        for (int j = 0; j < nc; j++) {
            const uint32_t* sj = seg + (size_t)j * (L >> 2);
            const int32_t* oj = oo + (c0 + j) * DB;
#pragma unroll
            for (int d = 0; d < DB; d++) {
                const int o = 4 * tid + oj[d];
                const uint32_t w0 = sj[o >> 2], w1 = sj[(o >> 2) + 1];
                const uint32_t w = __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)(o & 3));
                p02[d] += w & 0x00FF00FFu;
                p13[d] += (w >> 8) & 0x00FF00FFu;
            }
        }
#pragma unroll
        for (int d = 0; d < DB; d++) {
            acc[d][0] += p02[d] & 0xFFFFu;
            acc[d][2] += p02[d] >> 16;
            acc[d][1] += p13[d] & 0xFFFFu;
            acc[d][3] += p13[d] >> 16;
        }
    }
#pragma unroll
    for (int d = 0; d < DB; d++) {
        const int dm = blk * DB + d;
        if (dm >= ndm) continue;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int64_t t = t0 + 4 * tid + v;
            if (t < nout) st_global<int32_t>(series + (int64_t)dm * nout + t, (int32_t)acc[d][v]);
        }
    }
}

// float32: FP64 sums, channels added in ascending order for every output.
template <int DB>
__global__ __launch_bounds__(kDdThreads) void k_dedisp_f32(const float* __restrict__ x, int64_t C, int64_t stride,
                                                           int64_t nsamp, const int32_t* __restrict__ base,
                                                           const int32_t* __restrict__ off, int ndm, int64_t nout,
                                                           int L, int CC, double* __restrict__ series) {
    extern __shared__ __align__(16) float segf[];
    const int tid = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kDdTT;
    const int blk = blockIdx.y;
    const int32_t* bb = base + (int64_t)blk * C;
    const int32_t* oo = off + (int64_t)blk * C * DB;
    double acc[DB][4];
#pragma unroll
    for (int d = 0; d < DB; d++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc[d][v] = 0.0;
    for (int64_t c0 = 0; c0 < C; c0 += CC) {
        const int nc = (int)min((int64_t)CC, C - c0);
        __syncthreads();
        for (int j = 0; j < nc; j++) {
            const int64_t s0 = t0 + bb[c0 + j];
            const float* row = x + (c0 + j) * stride + s0;
            const int64_t avail = nsamp - s0;
            float* dst = segf + (size_t)j * L;
            for (int i = tid; i < L; i += kDdThreads) dst[i] = i < avail ? ld_global<float>(row + i) : 0.0f;
        }
        __syncthreads();
        for (int j = 0; j < nc; j++) {
            const float* sj = segf + (size_t)j * L;
            const int32_t* oj = oo + (c0 + j) * DB;
#pragma unroll
            for (int d = 0; d < DB; d++) {
                const float* p = sj + 4 * tid + oj[d];
#pragma unroll
                for (int v = 0; v < 4; v++) acc[d][v] += (double)p[v];
            }
        }
    }
#pragma unroll
    for (int d = 0; d < DB; d++) {
        const int dm = blk * DB + d;
        if (dm >= ndm) continue;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int64_t t = t0 + 4 * tid + v;
            if (t < nout) st_global<double>(series + (int64_t)dm * nout + t, acc[d][v]);
        }
    }
}

// ---- detection statistics ----------------------------------------------------

constexpr int kStThreads = 256;

__device__ inline u128 u128_from_words(uint64_t lo, uint64_t hi) { return ((u128)hi << 64) | lo; }

// (value, index) pair that wins: larger value, then the smaller index
template <typename V>
__device__ inline void better(V& v, int64_t& i, V ov, int64_t oi) {
    if (ov > v || (ov == v && oi < i)) {
        v = ov;
        i = oi;
    }
}

// int32 series: exact S1 (i128), S2 (u128) and the first maximum; then the
// decisions in FP64 from the exact n^2 * variance = n * S2 - S1^2.
__global__ __launch_bounds__(kStThreads) void k_series_stats_i32(const int32_t* __restrict__ series, int64_t n,
                                                                double* __restrict__ out) {
    __shared__ int64_t s_s1[kStThreads];
    __shared__ uint64_t s_s2lo[kStThreads], s_s2hi[kStThreads];
    __shared__ int32_t s_pk[kStThreads];
    __shared__ int64_t s_at[kStThreads];
    const int tid = threadIdx.x;
    const int32_t* s = series + (int64_t)blockIdx.x * n;
    int64_t s1 = 0;
    u128 s2 = 0;
    int32_t pk = INT32_MIN;
    int64_t at = INT64_MAX;
    for (int64_t t = tid; t < n; t += kStThreads) {
        const int32_t v = ld_global<int32_t>(s + t);
        s1 += v;
        s2 += (u128)((int64_t)v * v);
        better(pk, at, v, t);
    }
    s_s1[tid] = s1;
    s_s2lo[tid] = (uint64_t)s2;
    s_s2hi[tid] = (uint64_t)(s2 >> 64);
    s_pk[tid] = pk;
    s_at[tid] = at;
    __syncthreads();
    for (int h = kStThreads / 2; h > 0; h >>= 1) {
        if (tid < h) {
            s_s1[tid] += s_s1[tid + h];
            const u128 a = u128_from_words(s_s2lo[tid], s_s2hi[tid]) +
                           u128_from_words(s_s2lo[tid + h], s_s2hi[tid + h]);
            s_s2lo[tid] = (uint64_t)a;
            s_s2hi[tid] = (uint64_t)(a >> 64);
            int32_t v = s_pk[tid];
            int64_t i = s_at[tid];
            better(v, i, s_pk[tid + h], s_at[tid + h]);
            s_pk[tid] = v;
            s_at[tid] = i;
        }
        __syncthreads();
    }
    if (tid == 0) {
        const i128 S1 = s_s1[0];
        const u128 S2 = u128_from_words(s_s2lo[0], s_s2hi[0]);
        const u128 a1 = S1 < 0 ? (u128)(-S1) : (u128)S1;
        const u128 dn = (u128)n * S2 - a1 * a1;
        const double nd = (double)n;
        const double m = (double)s_s1[0] / nd;
        const double var = (((double)(uint64_t)(dn >> 64)) * 0x1p64 + (double)(uint64_t)dn) / (nd * nd);
        const double sd = var > 0.0 ? sqrt(var) : 0.0;
        const double pkd = (double)s_pk[0];
        double* o = out + (int64_t)blockIdx.x * 5;
        o[0] = sd > 0.0 ? (pkd - m) / sd : 0.0;
        o[1] = pkd;
        o[2] = (double)s_at[0];
        o[3] = m;
        o[4] = sd;
    }
}

// float64 series: mean, then the sum of squared deviations, in FP64.
__global__ __launch_bounds__(kStThreads) void k_series_stats_f64(const double* __restrict__ series, int64_t n,
                                                                double* __restrict__ out) {
    __shared__ double s_a[kStThreads];
    __shared__ double s_pk[kStThreads];
    __shared__ int64_t s_at[kStThreads];
    const int tid = threadIdx.x;
    const double* s = series + (int64_t)blockIdx.x * n;
    double a = 0.0, pk = -INFINITY;
    int64_t at = INT64_MAX;
    for (int64_t t = tid; t < n; t += kStThreads) {
        const double v = ld_global<double>(s + t);
        a += v;
        better(pk, at, v, t);
    }
    s_a[tid] = a;
    s_pk[tid] = pk;
    s_at[tid] = at;
    __syncthreads();
    for (int h = kStThreads / 2; h > 0; h >>= 1) {
        if (tid < h) {
            s_a[tid] += s_a[tid + h];
            double v = s_pk[tid];
            int64_t i = s_at[tid];
            better(v, i, s_pk[tid + h], s_at[tid + h]);
            s_pk[tid] = v;
            s_at[tid] = i;
        }
        __syncthreads();
    }
    const double m = s_a[0] / (double)n;
    const double pkd = s_pk[0];
    const int64_t pat = s_at[0];
    __syncthreads();
    double q = 0.0;
    for (int64_t t = tid; t < n; t += kStThreads) {
        const double dv = ld_global<double>(s + t) - m;
        q += dv * dv;
    }
    s_a[tid] = q;
    __syncthreads();
    for (int h = kStThreads / 2; h > 0; h >>= 1) {
        if (tid < h) s_a[tid] += s_a[tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        const double var = s_a[0] / (double)n;
        const double sd = var > 0.0 ? sqrt(var) : 0.0;
        double* o = out + (int64_t)blockIdx.x * 5;
        o[0] = sd > 0.0 ? (pkd - m) / sd : 0.0;
        o[1] = pkd;
        o[2] = (double)pat;
        o[3] = m;
        o[4] = sd;
    }
}

}  // namespace
}  // namespace rfim

using namespace rfim;

struct rfim_dedisp {
    int device = -1;
    int64_t nchan = 0;
    int32_t ndm = 0;
    int32_t max_delay = 0;
    std::vector<int32_t> delays;   // [ndm][nchan], host copy
    // per DM block (db consecutive trials) and dtype: smallest delay of the
    // block per channel, each trial's delay above it, the staged segment
    // length and channels per staged chunk
    struct Blocks {
        int db = 1;
        int nblk = 0;
        int L = 0, CC = 1;
        int32_t* d_base = nullptr;
        int32_t* d_off = nullptr;
    } u8, f32;

    ~rfim_dedisp() {
        for (Blocks* b : {&u8, &f32}) {
            if (b->d_base) (void)hipFree(b->d_base);
            if (b->d_off) (void)hipFree(b->d_off);
        }
    }
};

namespace {

// Largest block size <= db_max (a power of two) whose staged segment of elem
// bytes per sample fits the staging budget, its tables uploaded.
rfim_status make_blocks(rfim_dedisp& dd, int db_max, size_t elem, rfim_dedisp::Blocks& out) {
    const int64_t C = dd.nchan;
    for (int db = db_max; db >= 1; db >>= 1) {
        const int nblk = (dd.ndm + db - 1) / db;
        int64_t spread = 0;
        std::vector<int32_t> base((size_t)nblk * C), off((size_t)nblk * C * db, 0);
        for (int b = 0; b < nblk; b++)
            for (int64_t c = 0; c < C; c++) {
                int32_t lo = INT32_MAX;
                for (int k = 0; k < db && b * db + k < dd.ndm; k++)
                    lo = std::min(lo, dd.delays[(size_t)(b * db + k) * C + c]);
                base[(size_t)b * C + c] = lo;
                for (int k = 0; k < db && b * db + k < dd.ndm; k++) {
                    const int32_t o = dd.delays[(size_t)(b * db + k) * C + c] - lo;
                    off[((size_t)b * C + c) * db + k] = o;
                    spread = std::max<int64_t>(spread, o);
                }
            }
        // segment: every output's 4 samples at offsets up to kDdTT - 4 + spread,
        // rounded to whole dwords, plus one dword of slack for the uint8 reads
        const int64_t L = ((kDdTT + spread + 3) / 4) * 4 + 8;
        if ((size_t)L * elem > kDdLds && db > 1) continue;
        if ((size_t)L * elem > kDdLds) return RFIM_ERR_UNSUPPORTED;
        out.db = db;
        out.nblk = nblk;
        out.L = (int)L;
        out.CC = (int)std::min<int64_t>(std::min<size_t>(kDdLds / ((size_t)L * elem), 256), C);
        if (hipMalloc(&out.d_base, base.size() * 4) != hipSuccess ||
            hipMalloc(&out.d_off, off.size() * 4) != hipSuccess)
            return RFIM_ERR_OUT_OF_MEMORY;
        if (hipMemcpy(out.d_base, base.data(), base.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(out.d_off, off.data(), off.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return RFIM_ERR_DEVICE;
        return RFIM_OK;
    }
    return RFIM_ERR_UNSUPPORTED;
}

}  // namespace

extern "C" {

rfim_status rfim_dedisp_create(int64_t nchan, double f_low_mhz, double chan_bw_mhz, double tsamp_s,
                               const double* dms, int32_t ndm, rfim_dedisp** out) {
    if (!out) return RFIM_ERR_INVALID_ARG;
    *out = nullptr;
    if (nchan < 1 || nchan >= ((int64_t)1 << 23) || ndm < 1 || ndm > 65535 || !dms) return RFIM_ERR_INVALID_ARG;
    if (!(f_low_mhz > 0.0) || !(chan_bw_mhz > 0.0) || !(tsamp_s > 0.0) || !std::isfinite(f_low_mhz) ||
        !std::isfinite(chan_bw_mhz) || !std::isfinite(tsamp_s))
        return RFIM_ERR_INVALID_ARG;
    rfim_dedisp* dd = new (std::nothrow) rfim_dedisp();
    if (!dd) return RFIM_ERR_OUT_OF_MEMORY;
    if (hipGetDevice(&dd->device) != hipSuccess) {
        delete dd;
        return RFIM_ERR_DEVICE;
    }
    dd->nchan = nchan;
    dd->ndm = ndm;
    dd->delays.resize((size_t)ndm * nchan);
    // Eq. 2, relative to the top channel's centre
    const double f_top = f_low_mhz + ((double)(nchan - 1) + 0.5) * chan_bw_mhz;
    for (int32_t d = 0; d < ndm; d++) {
        if (!(dms[d] >= 0.0) || !std::isfinite(dms[d])) {
            delete dd;
            return RFIM_ERR_INVALID_ARG;
        }
        for (int64_t c = 0; c < nchan; c++) {
            const double f = f_low_mhz + ((double)c + 0.5) * chan_bw_mhz;
            const double sec = kKDM * dms[d] * (1.0 / (f * f) - 1.0 / (f_top * f_top));
            const double smp = std::nearbyint(sec / tsamp_s);
            if (!(smp >= 0.0) || smp > 2147483647.0) {
                delete dd;
                return RFIM_ERR_INVALID_ARG;
            }
            dd->delays[(size_t)d * nchan + c] = (int32_t)smp;
            dd->max_delay = std::max(dd->max_delay, (int32_t)smp);
        }
    }
    rfim_status st = make_blocks(*dd, kDbU8, 1, dd->u8);
    if (st == RFIM_OK) st = make_blocks(*dd, kDbF32, 4, dd->f32);
    if (st != RFIM_OK) {
        delete dd;
        return st;
    }
    *out = dd;
    return RFIM_OK;
}

rfim_status rfim_dedisp_destroy(rfim_dedisp* dd) {
    delete dd;
    return RFIM_OK;
}

rfim_status rfim_dedisp_delays(const rfim_dedisp* dd, int32_t* host_delays, int32_t* max_delay) {
    if (!dd) return RFIM_ERR_INVALID_ARG;
    if (host_delays) std::memcpy(host_delays, dd->delays.data(), dd->delays.size() * sizeof(int32_t));
    if (max_delay) *max_delay = dd->max_delay;
    return RFIM_OK;
}

rfim_status rfim_dedisperse(const rfim_dedisp* dd, const rfim_beam* beam, int64_t nout, void* series,
                            void* stream) {
    if (!dd || !beam || !series || !beam->in) return RFIM_ERR_INVALID_ARG;
    const rfim_beam& b = *beam;
    if (b.dtype != RFIM_U8 && b.dtype != RFIM_F32) return RFIM_ERR_INVALID_ARG;
    if (b.nchan != dd->nchan || b.nsamp < 1 || b.row_stride < b.nsamp) return RFIM_ERR_INVALID_ARG;
    if (nout < 1 || nout + dd->max_delay > b.nsamp || nout >= ((int64_t)1 << 40)) return RFIM_ERR_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != dd->device) return RFIM_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const rfim_dedisp::Blocks& bk = b.dtype == RFIM_U8 ? dd->u8 : dd->f32;
    const dim3 grid((unsigned)((nout + kDdTT - 1) / kDdTT), (unsigned)bk.nblk);
    const size_t lds = (size_t)bk.CC * bk.L * (b.dtype == RFIM_U8 ? 1 : 4);
    if (b.dtype == RFIM_U8) {
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(kDdThreads), lds, s, (const uint8_t*)b.in, b.nchan, b.row_stride,
                               b.nsamp, bk.d_base, bk.d_off, dd->ndm, nout, bk.L, bk.CC, (int32_t*)series);
        };
        switch (bk.db) {
            case 16: go(k_dedisp_u8<16>); break;
            case 8: go(k_dedisp_u8<8>); break;
            case 4: go(k_dedisp_u8<4>); break;
            case 2: go(k_dedisp_u8<2>); break;
            default: go(k_dedisp_u8<1>); break;
        }
    } else {
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(kDdThreads), lds, s, (const float*)b.in, b.nchan, b.row_stride,
                               b.nsamp, bk.d_base, bk.d_off, dd->ndm, nout, bk.L, bk.CC, (double*)series);
        };
        switch (bk.db) {
            case 4: go(k_dedisp_f32<4>); break;
            case 2: go(k_dedisp_f32<2>); break;
            default: go(k_dedisp_f32<1>); break;
        }
    }
    return hipGetLastError() == hipSuccess ? RFIM_OK : RFIM_ERR_DEVICE;
}

rfim_status rfim_series_stats(int32_t dtype, const void* series, int32_t nseries, int64_t n, double* stats,
                              void* stream) {
    if (!series || !stats || nseries < 1 || n < 1 || n >= ((int64_t)1 << 32)) return RFIM_ERR_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    if (dtype == RFIM_U8)
        hipLaunchKernelGGL(k_series_stats_i32, dim3(nseries), dim3(kStThreads), 0, s, (const int32_t*)series, n,
                           stats);
    else if (dtype == RFIM_F32)
        hipLaunchKernelGGL(k_series_stats_f64, dim3(nseries), dim3(kStThreads), 0, s, (const double*)series, n,
                           stats);
    else
        return RFIM_ERR_INVALID_ARG;
    return hipGetLastError() == hipSuccess ? RFIM_OK : RFIM_ERR_DEVICE;
}

}  // extern "C"
