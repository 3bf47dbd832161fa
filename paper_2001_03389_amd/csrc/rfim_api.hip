// Host side of the C ABI declared in include/rfim.h: argument validation,
// splitting a step list into runs of [TD steps][FD steps], launch planning
// (kernel shapes per beam), the launch program of a call (beam tables + an
// ordered list of kernel launches), workspaces, plans and HIP-graph capture.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "rfim_internal.h"
#include "rfim_tune.h"

namespace rfim {

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_zero_u64, dim3(blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

__global__ void k_or_error(const unsigned* __restrict__ src, unsigned* __restrict__ sticky) {
    if (threadIdx.x == 0 && *src) *sticky |= *src;
}

// folds a launch's error word into the workspace's sticky one (read by
// rfim_plan_flag_counts)
hipError_t launch_or_error(const unsigned* src, unsigned* sticky, hipStream_t s) {
    hipLaunchKernelGGL(k_or_error, dim3(1), dim3(64), 0, s, src, sticky);
    return hipGetLastError();
}

KExact make_k(double k) {
    // the exact binary value k = mk * 2^ek (mk odd) is kept for every k > 0:
    // the float32 wide path compares against sums far beyond 2^128
    KExact r{};
    r.k = k;
    if (k > 0.0) {
        int e = 0;
        double f = std::frexp(k, &e);
        uint64_t mk = (uint64_t)std::ldexp(f, 53);
        int ek = e - 53;
        while ((mk & 1) == 0) {
            mk >>= 1;
            ek++;
        }
        unsigned __int128 m2 = (unsigned __int128)mk * mk;
        r.mk2_lo = (uint64_t)m2;
        r.mk2_hi = (uint64_t)(m2 >> 64);
        r.mk2_bits = 0;
        for (unsigned __int128 t = m2; t; t >>= 1) r.mk2_bits++;
        r.ek = ek;
    }
    if (k < std::ldexp(1.0, -64)) {   // includes 0: k^2 * V < 1 for every V < 2^128
        r.mode = 1;
    } else if (k >= std::ldexp(1.0, 20)) {   // k^2 >= 2^40 > n - 1 and > C: nothing can be cut
        r.mode = 2;
    } else {
        r.mode = 0;
    }
    return r;
}

size_t elem_size(int32_t dt) { return dt == RFIM_U8 ? 1 : 4; }

namespace {

constexpr int kRing = 64;   // table staging slots per workspace
// largest uint8 fused-kernel tile (bytes of LDS); the default budget (tuning
// parameter) leaves three work-groups per CU
constexpr size_t kLdsMax = 131072;

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

size_t beam_span(const rfim_beam& b) {
    return (size_t)((b.nchan - 1) * b.row_stride + b.nsamp) * elem_size(b.dtype);
}

// The step list as runs of [consecutive TD steps][consecutive FD steps]; the
// TD steps of a run are all masked or all unmasked (a change starts a new run,
// and with it a new mask).
std::vector<Segment> segments_of(const rfim_step* steps, int32_t nsteps) {
    std::vector<Segment> out;
    int s = 0;
    while (s < nsteps) {
        Segment seg;
        std::memset(&seg, 0, sizeof(seg));
        if (steps[s].domain == RFIM_TD_MASKED) seg.td_masked = 1;
        const int32_t td_kind = seg.td_masked ? RFIM_TD_MASKED : RFIM_TD;
        while (s < nsteps && steps[s].domain == td_kind) {
            SegStep& d = seg.td[seg.n_td++];
            d.kx = make_k(steps[s].k);
            d.replace = steps[s].replace;
            d.bit = s < 8 ? s : -1;
            d.ci = s;
            d.bin = 0;
            s++;
        }
        while (s < nsteps && steps[s].domain == RFIM_FD) {
            SegStep& d = seg.fd[seg.n_fd++];
            d.kx = make_k(steps[s].k);
            d.replace = steps[s].replace;
            d.bit = s < 8 ? s : -1;
            d.ci = s;
            d.bin = steps[s].bin_size;
            s++;
        }
        out.push_back(seg);
    }
    return out;
}

// LDS a work-group may use (the device limit, queried once)
size_t lds_limit() {
    static size_t lim = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            return (size_t)65536;
        return (size_t)v;
    }();
    return lim;
}

// uint8 fused-kernel tile for one beam: Tt samples (power of two in [4, cap])
// and Cp LDS bytes per time sample
bool tile_shape_u8(const rfim_beam& b, bool flags, int cap, size_t budget, int32_t* Tt, int32_t* Cp) {
    if (b.nchan >= ((int64_t)1 << 24)) return false;   // worklist packs the row in 24 bits
    // 16-byte aligned time samples (vector LDS reads), padded off a multiple
    // of 256 bytes so the transposed stores of neighbouring lanes spread over banks
    int64_t cp = ((b.nchan + 15) / 16) * 16;
    if (cp % 256 == 0 || cp % 256 == 128) cp += 16;
    size_t per = (size_t)cp * (flags ? 2 : 1);
    int t = 4;
    while (t * 2 <= cap && t < 64) t *= 2;
    while (t > 4 && per * t > budget) t >>= 1;
    if (per * t > std::min(kLdsMax, lds_limit() - 4096)) return false;
    *Tt = t;
    *Cp = (int32_t)cp;
    return true;
}

struct Slot {
    void* h = nullptr;  // pinned staging
    void* d = nullptr;  // device copy read by the kernels
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
};

}  // namespace

rfim_status validate(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps,
                     int32_t nsteps) {
    if (nbeams < 0 || nsteps < 0 || nsteps > kMaxSteps) return RFIM_ERR_INVALID_ARG;
    if (nbeams > 0 && !beams) return RFIM_ERR_INVALID_ARG;
    if (nsteps > 0 && !steps) return RFIM_ERR_INVALID_ARG;
    for (int s = 0; s < nsteps; s++) {
        const rfim_step& st = steps[s];
        if (st.domain != RFIM_TD && st.domain != RFIM_FD && st.domain != RFIM_TD_MASKED)
            return RFIM_ERR_INVALID_ARG;
        if (st.replace != RFIM_REPLACE_MEAN && st.replace != RFIM_REPLACE_MEDIAN)
            return RFIM_ERR_INVALID_ARG;
        if (!std::isfinite(st.k) || st.k < 0.0) return RFIM_ERR_INVALID_ARG;
        if (st.domain == RFIM_FD && st.bin_size < 0) return RFIM_ERR_INVALID_ARG;
    }
    for (int i = 0; i < nbeams; i++) {
        const rfim_beam& b = beams[i];
        if (b.dtype != RFIM_U8 && b.dtype != RFIM_F32) return RFIM_ERR_INVALID_ARG;
        if (b.reserved != 0) return RFIM_ERR_INVALID_ARG;
        if (b.nchan < 1 || b.nchan >= ((int64_t)1 << 31)) return RFIM_ERR_INVALID_ARG;
        if (b.nsamp < 1 || b.nsamp >= ((int64_t)1 << 31)) return RFIM_ERR_INVALID_ARG;
        if (b.row_stride < b.nsamp) return RFIM_ERR_INVALID_ARG;
        if (!b.in || !b.out) return RFIM_ERR_INVALID_ARG;
        if (b.flags && nsteps > 8) return RFIM_ERR_INVALID_ARG;
        size_t span = beam_span(b);
        if (b.in != b.out && overlaps(b.in, span, b.out, span)) return RFIM_ERR_INVALID_ARG;
        if (b.flags) {
            size_t fspan = (size_t)((b.nchan - 1) * b.row_stride + b.nsamp);
            if (overlaps(b.flags, fspan, b.in, span) || overlaps(b.flags, fspan, b.out, span))
                return RFIM_ERR_INVALID_ARG;
        }
        for (int s = 0; s < nsteps; s++) {
            if (steps[s].domain != RFIM_FD) continue;
            int64_t B = steps[s].bin_size == 0 ? b.nchan : steps[s].bin_size;
            if (B < 1 || b.nchan % B != 0) return RFIM_ERR_INVALID_ARG;
        }
    }
    // masked TD steps run on the uint8 row histograms only
    for (int s = 0; s < nsteps; s++)
        if (steps[s].domain == RFIM_TD_MASKED)
            for (int i = 0; i < nbeams; i++)
                if (beams[i].dtype != RFIM_U8) return RFIM_ERR_UNSUPPORTED;
    return RFIM_OK;
}

struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
};

struct Workspace {
    int device = -1;
    bool fixed = false;  // plan workspace: never grows
    bool timing = false;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    std::mutex mu;
    void* d_work = nullptr;
    size_t work_cap = 0;
    hipEvent_t last_done = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_last = false;
    Slot ring[kRing];
    int next = 0;

    ~Workspace() {
        if (has_last) (void)hipEventSynchronize(last_done);
        clear_timing();
        for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
        for (auto& s : ring) {
            if (s.used) (void)hipEventSynchronize(s.ev);
            if (s.h) (void)hipHostFree(s.h);
            if (s.d) (void)hipFree(s.d);
            if (s.ev) (void)hipEventDestroy(s.ev);
        }
        if (d_work) (void)hipFree(d_work);
        if (last_done) (void)hipEventDestroy(last_done);
    }

    rfim_status init(int dev) {
        device = dev;
        if (hipEventCreateWithFlags(&last_done, hipEventDisableTiming) != hipSuccess)
            return RFIM_ERR_DEVICE;
        for (auto& s : ring)
            if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess)
                return RFIM_ERR_DEVICE;
        return RFIM_OK;
    }

    void clear_timing() {
        for (auto& t : timed) {
            event_pool.push_back(t.a);
            event_pool.push_back(t.b);
        }
        timed.clear();
    }

    hipEvent_t take_event() {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }

    // brackets one launch with events when timing is on
    template <typename F>
    hipError_t timed_launch(int kind, hipStream_t s, F&& launch) {
        if (!timing || kind < 0) return launch();
        hipEvent_t a = take_event(), b = take_event();
        if (!a || !b) return hipErrorOutOfMemory;
        hipError_t e = hipEventRecord(a, s);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(b, s);
        timed.push_back({kind, a, b});
        return e;
    }

    rfim_status reserve_work(size_t bytes) {
        if (bytes <= work_cap) return RFIM_OK;
        if (fixed) return RFIM_ERR_INVALID_ARG;
        if (has_last && hipEventSynchronize(last_done) != hipSuccess) return RFIM_ERR_DEVICE;
        if (d_work) (void)hipFree(d_work);
        d_work = nullptr;
        work_cap = 0;
        size_t cap = std::max<size_t>(bytes, (size_t)1 << 20);
        if (hipMalloc(&d_work, cap) != hipSuccess) return RFIM_ERR_OUT_OF_MEMORY;
        if (hipMemset(d_work, 0, cap) != hipSuccess) return RFIM_ERR_DEVICE;   // sticky error words start clear
        work_cap = cap;
        return RFIM_OK;
    }

    // a staging slot able to hold `bytes`, free of any pending copy
    rfim_status slot(size_t bytes, Slot** out) {
        Slot& s = ring[next];
        next = (next + 1) % kRing;
        if (s.used && hipEventSynchronize(s.ev) != hipSuccess) return RFIM_ERR_DEVICE;
        s.used = false;
        if (s.cap < bytes) {
            if (fixed && s.cap) return RFIM_ERR_INVALID_ARG;
            if (s.h) (void)hipHostFree(s.h);
            if (s.d) (void)hipFree(s.d);
            s.h = s.d = nullptr;
            s.cap = 0;
            size_t cap = std::max<size_t>(bytes, 4096);
            if (hipHostMalloc(&s.h, cap, hipHostMallocDefault) != hipSuccess)
                return RFIM_ERR_OUT_OF_MEMORY;
            if (hipMalloc(&s.d, cap) != hipSuccess) return RFIM_ERR_OUT_OF_MEMORY;
            s.cap = cap;
        }
        *out = &s;
        return RFIM_OK;
    }
};

namespace {

std::mutex g_ws_mu;
std::vector<Workspace*> g_ws;  // per device, created on first use, kept for the process

rfim_status device_workspace(Workspace** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RFIM_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1, nullptr);
    if (!g_ws[dev]) {
        Workspace* w = new (std::nothrow) Workspace();
        if (!w) return RFIM_ERR_OUT_OF_MEMORY;
        rfim_status st = w->init(dev);
        if (st != RFIM_OK) {
            delete w;
            return st;
        }
        g_ws[dev] = w;
    }
    *out = g_ws[dev];
    return RFIM_OK;
}

// Kernel shapes of a call, chosen from the beam shapes, the steps and the
// tuning parameters.
struct LaunchPlan {
    TuneParams tune;
    std::vector<Segment> segs;
    std::vector<int> u8_beams;   // indices of uint8 beams
    std::vector<int> f32_beams;  // indices of float32 beams
    std::vector<int32_t> Tt, Cp; // uint8 tile per beam
    int64_t u8_rows = 0, u8_tiles = 0;
    size_t u8_lds = 0;
    int max_td = 0;
    int nsteps = 0;
    // float32: TD kernel shape per beam (nt x vpt; nt == 0: every row wide),
    // fused-kernel shape per segment and beam (fast FD bin B, 0 = none)
    std::vector<int32_t> f_nt, f_vpt;
    struct F32Shape {
        int32_t B = 0, bpl = 1, Tt = 64, Cp = 0;
        size_t lds = 0;
    };
    std::vector<std::vector<F32Shape>> f_shape;   // [segment][float32 beam]
    int64_t f32_rows = 0, f32_cols = 0, f32_maxC = 0;
    // workspace layout (byte offsets)
    size_t off_u8rec = 0, off_f32rec = 0, off_wide = 0, off_tditems = 0, off_fditems = 0;
    size_t off_tdtiny = 0, off_fdtiny = 0, off_f32fast = 0;
    size_t count_bytes = 0, work_bytes = 0;
    // uint8 persistent schedule: control words [next item per queue, error,
    // done per uint8 beam] (zeroed before each launch), the sticky error word,
    // LDS and grid
    size_t off_ctl = 0, off_err = 0, ctl_words = 0;
    size_t persist_lds = 0;
    int persist_grid = 0;
    uint32_t spin_limit = 1u << 22, wait_extra = 0;
};

// True when, for every uint8 beam and FD step of the run, each lane's share
// of a bin (a whole bin, or B/(lanes per bin) when bins span several lanes) is
// a multiple of 16 bytes; bins then start 16-byte aligned because Cp is.
bool fd_vec_ok(const rfim_beam* beams, const LaunchPlan& lp, const Segment& seg) {
    for (int bi : lp.u8_beams) {
        const rfim_beam& b = beams[bi];
        const int G = kBlock / lp.Tt[bi];
        for (int s = 0; s < seg.n_fd; s++) {
            const int64_t B = seg.fd[s].bin == 0 ? b.nchan : seg.fd[s].bin;
            const int64_t nb = b.nchan / B;
            int64_t lpb = 1;
            if (nb < G && (G % nb) == 0 && (B % (16 * (G / nb))) == 0) lpb = G / nb;
            if ((B / lpb) % 16 != 0) return false;
        }
    }
    return true;
}

// FD path of the uint8 fused kernel for one beam and run: the 32-channel
// path when every FD step of the run uses 32-channel bins, the tile is 16,
// 32 or 64 samples wide (4, 8 or 16 lanes per time sample) and every lane's
// bins fit its registers; otherwise the general path (16-byte reads when the
// whole launch allows them).
int32_t fd_path_u8(const rfim_beam& b, int Tt, const Segment& seg, bool vec) {
    if (seg.n_fd == 0) return RFIM_FD_PATH_NONE;
    bool b32 = vec && (b.nchan % 32) == 0 && (b.nchan / 32) <= (int64_t)kB32MaxBins * (kBlock / Tt);
    for (int s = 0; s < seg.n_fd; s++) b32 &= seg.fd[s].bin == 32 || (seg.fd[s].bin == 0 && b.nchan == 32);
    if (b32 && Tt == 32) return RFIM_FD_PATH_U8_BIN32_G8;
    if (b32 && Tt == 16) return RFIM_FD_PATH_U8_BIN32_G16;
    if (b32 && Tt == 64) return RFIM_FD_PATH_U8_BIN32_G4;
    return vec ? RFIM_FD_PATH_U8_VEC : RFIM_FD_PATH_U8_BYTES;
}

// Shapes of the float32 kernels for every float32 beam of the call.
rfim_status plan_f32(const rfim_beam* beams, LaunchPlan* lp) {
    const int nf = (int)lp->f32_beams.size();
    lp->f_nt.assign(nf, 0);
    lp->f_vpt.assign(nf, 0);
    lp->f_shape.assign(lp->segs.size(), std::vector<LaunchPlan::F32Shape>(nf));
    bool any_fd = false;
    for (auto& sg : lp->segs) any_fd |= sg.n_fd > 0;
    const size_t budget = std::min(lp->tune.f32_lds, lds_limit());
    for (int j = 0; j < nf; j++) {
        const rfim_beam& b = beams[lp->f32_beams[j]];
        // exact wide sums are sized for fewer than 2^24 samples per row / column
        if (b.nchan >= ((int64_t)1 << 24) || b.nsamp >= ((int64_t)1 << 24)) return RFIM_ERR_UNSUPPORTED;
        // a time sample of the wide FD kernel lives in LDS (value + flag byte)
        if (any_fd && (size_t)b.nchan * 5 > 98304) return RFIM_ERR_UNSUPPORTED;
        const int64_t T = b.nsamp;
        int nt = 0, vpt = 0;
        if (T <= 256) { nt = 256; vpt = 1; }
        else if (T <= 1024) { nt = 256; vpt = 4; }
        else if (T <= 4096) { nt = 256; vpt = 16; }
        else if (T <= 8192) { nt = 1024; vpt = 8; }
        else if (T <= 16384) { nt = 1024; vpt = 16; }
        else if (T <= 32768) { nt = 1024; vpt = 32; }
        else if (T <= 65536) { nt = 1024; vpt = 64; }
        lp->f_nt[j] = nt;   // 0: rows longer than the register-resident kernel holds go wide
        lp->f_vpt[j] = vpt;
        lp->f32_rows += b.nchan;
        lp->f32_cols += b.nsamp;
        lp->f32_maxC = std::max<int64_t>(lp->f32_maxC, b.nchan);
        for (size_t si = 0; si < lp->segs.size(); si++) {
            const Segment& sg = lp->segs[si];
            LaunchPlan::F32Shape& sh = lp->f_shape[si][j];
            sh = LaunchPlan::F32Shape();
            int64_t B = -1;
            for (int s = 0; s < sg.n_fd; s++) {
                const int64_t Bs = sg.fd[s].bin == 0 ? b.nchan : sg.fd[s].bin;
                B = (B == -1 || B == Bs) ? Bs : 0;
            }
            const int64_t nbins = B > 0 ? b.nchan / B : 0;
            const bool fast = sg.n_fd > 0 && (B == 8 || B == 16 || B == 32 || B == 64) &&
                              nbins <= (B == 64 ? 64 : 128);
            if (fast) {
                const int32_t Cp = (int32_t)(nbins * (B + 4));
                const size_t per = (size_t)Cp * 4 + (b.flags ? (size_t)b.nchan : 0);
                int t = 4;
                while (t * 2 <= lp->tune.f32_tile_cap && t < 64) t *= 2;
                while (t > 4 && per * t > budget) t >>= 1;
                if (per * t <= lds_limit()) {
                    sh.B = (int32_t)B;
                    sh.bpl = nbins > 64 ? 2 : 1;
                    sh.Cp = Cp;
                    sh.Tt = t;
                    sh.lds = per * t;
                }
            }
        }
    }
    return RFIM_OK;
}

rfim_status make_launch_plan(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps,
                             int32_t nsteps, bool want_counts, const TuneParams& tune, LaunchPlan* lp) {
    lp->tune = tune;
    lp->segs = segments_of(steps, nsteps);
    lp->nsteps = nsteps;
    lp->Tt.assign(nbeams, 0);
    lp->Cp.assign(nbeams, 0);
    for (auto& s : lp->segs) lp->max_td = std::max(lp->max_td, s.n_td);
    for (int i = 0; i < nbeams; i++) {
        const rfim_beam& b = beams[i];
        if (b.dtype == RFIM_F32) {
            lp->f32_beams.push_back(i);
            continue;
        }
        lp->u8_beams.push_back(i);
        if (!tile_shape_u8(b, b.flags != nullptr, tune.u8_tile_cap, tune.u8_lds, &lp->Tt[i], &lp->Cp[i]))
            return RFIM_ERR_UNSUPPORTED;
        lp->u8_rows += b.nchan;
        lp->u8_tiles += (b.nsamp + lp->Tt[i] - 1) / lp->Tt[i];
        size_t lds = (size_t)lp->Tt[i] * lp->Cp[i] * (b.flags ? 2 : 1);
        lp->u8_lds = std::max(lp->u8_lds, lds);
    }
    if (lp->u8_rows >= ((int64_t)1 << 31) || lp->u8_tiles >= ((int64_t)1 << 31))
        return RFIM_ERR_UNSUPPORTED;
    rfim_status fs = plan_f32(beams, lp);
    if (fs != RFIM_OK) return fs;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    lp->count_bytes = want_counts ? al((size_t)nbeams * kCountStride * sizeof(unsigned long long)) : 0;
    lp->off_u8rec = lp->count_bytes;
    lp->off_f32rec = lp->off_u8rec + al((size_t)lp->u8_rows * std::max(1, lp->max_td) * 4);
    lp->off_wide = lp->off_f32rec + al((size_t)lp->f32_rows * std::max(1, lp->max_td) * 16);
    lp->off_tditems = lp->off_wide + (lp->f32_beams.empty() ? 0 : 256);
    lp->off_fditems = lp->off_tditems + al((size_t)lp->f32_rows * 8);
    lp->off_tdtiny = lp->off_fditems + al((size_t)lp->f32_cols * 8);
    lp->off_fdtiny = lp->off_tdtiny + al((size_t)lp->f32_rows * 8);
    lp->off_f32fast = lp->off_fdtiny + al((size_t)lp->f32_cols * 8);
    lp->work_bytes = lp->off_f32fast + al((size_t)lp->f32_rows * 8);
    // the sticky error word of the persistent schedule (zeroed with the workspace)
    lp->off_err = lp->work_bytes;
    lp->work_bytes += 256;
    if (tune.u8_sched == 1 && !lp->u8_beams.empty()) {
        lp->ctl_words = (kPersistQueues + 1 + lp->u8_beams.size() + 1) / 2;   // 64-bit words
        lp->off_ctl = lp->work_bytes;
        lp->work_bytes += al(lp->ctl_words * 8);
        lp->persist_lds = std::max(lp->u8_lds, td_group_lds_bytes());
        if (lp->persist_lds > std::min(kLdsMax, lds_limit() - 4096)) return RFIM_ERR_UNSUPPORTED;
        lp->persist_grid = persist_u8_grid(lp->persist_lds, true);
        if (const char* e = std::getenv("RFIM_SPIN_LIMIT")) lp->spin_limit = (uint32_t)std::strtoul(e, nullptr, 10);
        if (const char* e = std::getenv("RFIM_WAIT_EXTRA")) lp->wait_extra = (uint32_t)std::strtoul(e, nullptr, 10);
    }
    return RFIM_OK;
}

hipError_t g_last_error = hipSuccess;

rfim_status dev_err(hipError_t e) {
    g_last_error = e;
    return e == hipSuccess ? RFIM_OK : RFIM_ERR_DEVICE;
}

// ---------------------------------------------------------------------------
// The launch program of a call: every beam table of the call in one blob and
// the ordered kernel launches that read them.  Built on the host per call (or
// once for a captured graph), then enqueued on one stream.
// ---------------------------------------------------------------------------
enum Op {
    OP_ZERO_COUNTS, OP_TD_U8, OP_FUSED_U8, OP_PERSIST_U8, OP_ZERO_WIDE, OP_TD_F32, OP_TD_TWO, OP_LIST_ALL, OP_TD_WIDE,
    OP_TD_COMPOSE,
    OP_FUSED_F32, OP_FD_TWO, OP_FD_WIDE
};

struct Launch {
    int op = 0;
    int seg = -1;       // index into Program::segs
    int table = -1;     // first DevBeam of its table in the blob
    int nbeams = 0;
    int64_t total = 0;  // rows / tiles / list length
    int a = 0, b = 0;   // TD f32 (nt, vpt); fused f32 (B, bpl); wide (grid); list (gidx)
    size_t lds = 0;
    bool vec = false;
    PersistQueues qs{};   // persistent uint8 launch: item range of each queue
};

struct Program {
    std::vector<DevBeam> blob;
    std::vector<Segment> segs;
    std::vector<Launch> launches;
};

DevBeam dev_beam(const rfim_beam& b, bool first_seg) {
    DevBeam d;
    std::memset(&d, 0, sizeof(d));
    d.in = first_seg ? b.in : b.out;
    d.out = b.out;
    d.flags = b.flags;
    d.C = b.nchan;
    d.T = b.nsamp;
    d.stride = b.row_stride;
    return d;
}

void build_u8(const rfim_beam* beams, const LaunchPlan& lp, Program& pg) {
    const int nu8 = (int)lp.u8_beams.size();
    if (nu8 == 0) return;
    for (size_t si = 0; si < lp.segs.size(); si++) {
        Segment seg = lp.segs[si];
        bool any_flags = false;
        for (int j = 0; j < nu8; j++) any_flags |= beams[lp.u8_beams[j]].flags != nullptr;
        seg.flags_mode = any_flags ? (si == 0 ? 1 : 2) : 0;
        const int sidx = (int)pg.segs.size();
        pg.segs.push_back(seg);
        const int table = (int)pg.blob.size();
        const bool vec = fd_vec_ok(beams, lp, seg);
        auto items_of = [&](int bi) {
            const rfim_beam& b = beams[bi];
            const int64_t ntiles = (b.nsamp + lp.Tt[bi] - 1) / lp.Tt[bi];
            return (seg.n_td > 0 ? (b.nchan + kBlock / 64 - 1) / (kBlock / 64) : 0) + ntiles;
        };
        // table order: the call's order, or for the persistent schedule queue
        // by queue (beams dealt largest first to the least loaded queue)
        std::vector<int> order(lp.u8_beams);
        PersistQueues qs;
        std::memset(&qs, 0, sizeof qs);
        if (lp.tune.u8_sched == 1) {
            std::vector<int> by_size(lp.u8_beams);
            std::stable_sort(by_size.begin(), by_size.end(), [&](int a, int b) { return items_of(a) > items_of(b); });
            std::vector<std::vector<int>> q(kPersistQueues);
            std::vector<int64_t> load(kPersistQueues, 0);
            for (int bi : by_size) {
                const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                q[k].push_back(bi);
                load[k] += items_of(bi);
            }
            order.clear();
            int64_t base = 0;
            for (int k = 0; k < kPersistQueues; k++) {
                std::sort(q[k].begin(), q[k].end());
                qs.base[k] = base;
                for (int bi : q[k]) order.push_back(bi);
                base += load[k];
            }
            qs.base[kPersistQueues] = base;
        }
        int64_t row = 0, tile = 0, item = 0;
        for (int bi : order) {
            DevBeam d = dev_beam(beams[bi], si == 0);
            d.row0 = row;
            d.rec0 = row;
            d.tile0 = tile;
            d.Tt = lp.Tt[bi];
            d.Cp = lp.Cp[bi];
            d.cidx = bi;
            d.path = fd_path_u8(beams[bi], d.Tt, seg, vec);
            d.item0 = item;
            const int64_t ntiles = (d.T + d.Tt - 1) / d.Tt;
            item += items_of(bi);
            row += d.C;
            tile += ntiles;
            pg.blob.push_back(d);
        }
        if (lp.tune.u8_sched == 1) {
            Launch L;
            L.op = OP_PERSIST_U8;
            L.seg = sidx;
            L.table = table;
            L.nbeams = nu8;
            L.total = item;
            L.lds = lp.persist_lds;
            L.vec = vec;
            L.qs = qs;
            pg.launches.push_back(L);
            continue;
        }
        if (seg.n_td > 0) {
            Launch L;
            L.op = OP_TD_U8;
            L.seg = sidx;
            L.table = table;
            L.nbeams = nu8;
            L.total = row;
            pg.launches.push_back(L);
        }
        Launch L;
        L.op = OP_FUSED_U8;
        L.seg = sidx;
        L.table = table;
        L.nbeams = nu8;
        L.total = tile;
        L.lds = lp.u8_lds;
        L.vec = vec;
        pg.launches.push_back(L);
    }
}

// float32 beams: per run of [TD][FD] steps, TD rows (register-resident kernel
// per row-length class, wide fallback for the rows it lists), then the fused
// TD-apply + FD pass per bin class and the wide fallback for the time samples
// it lists.
void build_f32(const rfim_beam* beams, const LaunchPlan& lp, Program& pg) {
    const int nf = (int)lp.f32_beams.size();
    if (nf == 0) return;
    static const int td_shapes[7][2] = {{256, 1}, {256, 4}, {256, 16}, {1024, 8}, {1024, 16}, {1024, 32}, {1024, 64}};
    static const int fd_shapes[8][2] = {{0, 1}, {8, 1}, {8, 2}, {16, 1}, {16, 2}, {32, 1}, {32, 2}, {64, 1}};
    for (size_t si = 0; si < lp.segs.size(); si++) {
        Segment seg = lp.segs[si];
        bool any_flags = false;
        for (int j = 0; j < nf; j++) any_flags |= beams[lp.f32_beams[j]].flags != nullptr;
        seg.flags_mode = any_flags ? (si == 0 ? 1 : 2) : 0;
        const int sidx = (int)pg.segs.size();
        pg.segs.push_back(seg);
        // table of every float32 beam (the wide kernels index it)
        const int all = (int)pg.blob.size();
        int64_t rows = 0, cols = 0;
        for (int j = 0; j < nf; j++) {
            DevBeam d = dev_beam(beams[lp.f32_beams[j]], si == 0);
            d.rec0 = rows;
            d.cidx = lp.f32_beams[j];
            d.pad = j;
            d.Tt = lp.f_shape[si][j].B;     // the two-window FD kernel's shape
            d.Cp = lp.f_shape[si][j].bpl;
            rows += d.C;
            cols += d.T;
            pg.blob.push_back(d);
        }
        Launch Z;
        Z.op = OP_ZERO_WIDE;
        Z.seg = sidx;
        pg.launches.push_back(Z);
        if (seg.n_td > 0) {
            for (auto& sh : td_shapes) {
                const int table = (int)pg.blob.size();
                int64_t row = 0;
                int n = 0;
                for (int j = 0; j < nf; j++) {
                    if (lp.f_nt[j] != sh[0] || lp.f_vpt[j] != sh[1]) continue;
                    DevBeam d = pg.blob[all + j];
                    d.row0 = row;
                    row += d.C;
                    pg.blob.push_back(d);
                    n++;
                }
                if (!n) continue;
                Launch L;
                L.op = OP_TD_F32;
                L.seg = sidx;
                L.table = table;
                L.nbeams = n;
                L.total = row;
                L.a = sh[0];
                L.b = sh[1];
                pg.launches.push_back(L);
            }
            {
                Launch L;   // rows with values below the first window
                L.op = OP_TD_TWO;
                L.seg = sidx;
                L.table = all;
                L.a = (int)std::min<int64_t>(rows, 256);
                pg.launches.push_back(L);
            }
            for (int j = 0; j < nf; j++) {
                if (lp.f_nt[j] != 0) continue;
                Launch L;
                L.op = OP_LIST_ALL;
                L.seg = sidx;
                L.total = pg.blob[all + j].C;
                L.a = j;
                L.b = 0;   // the TD list
                pg.launches.push_back(L);
            }
            Launch W;
            W.op = OP_TD_WIDE;
            W.seg = sidx;
            W.table = all;
            W.nbeams = nf;
            W.a = (int)std::min<int64_t>(rows, 512);
            pg.launches.push_back(W);
            Launch K;   // composite records of every float32 row of the run
            K.op = OP_TD_COMPOSE;
            K.seg = sidx;
            K.total = rows;
            pg.launches.push_back(K);
        }
        for (auto& fsh : fd_shapes) {
            const int table = (int)pg.blob.size();
            int64_t tile = 0;
            size_t lds = 0;
            int n = 0;
            for (int j = 0; j < nf; j++) {
                const LaunchPlan::F32Shape& sh = lp.f_shape[si][j];
                if (sh.B != fsh[0] || (sh.B && sh.bpl != fsh[1])) continue;
                DevBeam d = pg.blob[all + j];
                d.tile0 = tile;
                d.Tt = sh.Tt;
                d.Cp = sh.Cp;
                tile += (d.T + sh.Tt - 1) / sh.Tt;
                lds = std::max(lds, sh.lds);
                pg.blob.push_back(d);
                n++;
            }
            if (!n) continue;
            Launch L;
            L.op = OP_FUSED_F32;
            L.seg = sidx;
            L.table = table;
            L.nbeams = n;
            L.total = tile;
            L.a = fsh[0];
            L.b = fsh[1];
            L.lds = lds;
            pg.launches.push_back(L);
        }
        if (seg.n_fd > 0) {
            for (auto& fsh : fd_shapes) {
                if (!fsh[0]) continue;
                bool any = false;
                for (int j = 0; j < nf; j++)
                    any |= lp.f_shape[si][j].B == fsh[0] && lp.f_shape[si][j].bpl == fsh[1];
                if (!any) continue;
                Launch L;   // time samples with values below the first window
                L.op = OP_FD_TWO;
                L.seg = sidx;
                L.table = all;
                L.a = (int)std::min<int64_t>((cols + 3) / 4, 512);
                L.b = fsh[0];
                L.nbeams = fsh[1];
                pg.launches.push_back(L);
            }
            Launch W;
            W.op = OP_FD_WIDE;
            W.seg = sidx;
            W.table = all;
            W.nbeams = nf;
            W.a = (int)std::min<int64_t>(cols, 512);
            pg.launches.push_back(W);
        }
    }
}

void build_program(const rfim_beam* beams, int32_t nbeams, const LaunchPlan& lp, bool want_counts, Program& pg) {
    pg = Program();
    if (want_counts) {
        Launch Z;
        Z.op = OP_ZERO_COUNTS;
        Z.total = (int64_t)nbeams * kCountStride;
        pg.launches.push_back(Z);
    }
    build_u8(beams, lp, pg);
    build_f32(beams, lp, pg);
}

// Enqueues the program on `stream`; d_blob is the device copy of pg.blob and
// wbase the device workspace laid out by lp.  ws (may be null) times the
// launches when its timing is on.
rfim_status enqueue(const Program& pg, const LaunchPlan& lp, const DevBeam* d_blob, char* wbase, Workspace* ws,
                    hipStream_t stream, bool want_counts) {
    auto timed = [&](int kind, auto&& launch) -> hipError_t {
        return ws ? ws->timed_launch(kind, stream, launch) : launch();
    };
    uint32_t* u8rec = (uint32_t*)(wbase + lp.off_u8rec);
    unsigned long long* counts = want_counts ? (unsigned long long*)wbase : nullptr;
    float4* frec = (float4*)(wbase + lp.off_f32rec);
    unsigned* wide_td_n = (unsigned*)(wbase + lp.off_wide);
    unsigned* wide_fd_n = (unsigned*)(wbase + lp.off_wide + 8);
    int2* td_items = (int2*)(wbase + lp.off_tditems);
    int2* fd_items = (int2*)(wbase + lp.off_fditems);
    unsigned* tiny_td_n = (unsigned*)(wbase + lp.off_wide + 16);
    unsigned* tiny_fd_n = (unsigned*)(wbase + lp.off_wide + 24);
    int2* td_tiny = (int2*)(wbase + lp.off_tdtiny);
    int2* fd_tiny = (int2*)(wbase + lp.off_fdtiny);
    float2* ffast = (float2*)(wbase + lp.off_f32fast);
    for (const Launch& L : pg.launches) {
        const DevBeam* tab = L.table >= 0 ? d_blob + L.table : nullptr;
        const Segment& seg = pg.segs[L.seg >= 0 ? L.seg : 0];
        hipError_t e = hipSuccess;
        switch (L.op) {
            case OP_ZERO_COUNTS:
                e = launch_zero_u64(counts, L.total, stream);
                break;
            case OP_TD_U8:
                e = timed(RFIM_KERNEL_TD_ROWS_U8, [&] {
                    return launch_td_rows_u8(tab, L.nbeams, L.total, lp.tune.u8_td_rows, seg, u8rec, counts,
                                             kCountStride, stream);
                });
                break;
            case OP_FUSED_U8:
                e = timed(RFIM_KERNEL_FUSED_U8, [&] {
                    return launch_fused_u8(tab, L.nbeams, L.total, seg, u8rec, L.lds, L.vec, counts, kCountStride, stream);
                });
                break;
            case OP_PERSIST_U8: {
                unsigned* ctl = (unsigned*)(wbase + lp.off_ctl);
                e = launch_zero_u64((unsigned long long*)ctl, (int64_t)lp.ctl_words, stream);
                if (e == hipSuccess)
                    e = timed(RFIM_KERNEL_PERSIST_U8, [&] {
                        return launch_persist_u8(tab, L.nbeams, L.qs, seg, u8rec, L.lds, L.vec, counts,
                                                 kCountStride, ctl, lp.spin_limit, lp.wait_extra, lp.persist_grid,
                                                 stream);
                    });
                if (e == hipSuccess)
                    e = launch_or_error(ctl + kPersistQueues, (unsigned*)(wbase + lp.off_err), stream);
                break;
            }
            case OP_ZERO_WIDE:
                e = launch_zero_u64((unsigned long long*)wide_td_n, 4, stream);
                break;
            case OP_TD_F32:
                e = timed(RFIM_KERNEL_TD_ROWS_F32, [&] {
                    return launch_td_rows_f32(tab, L.nbeams, L.total, L.a, L.b, seg, frec, tiny_td_n, td_tiny,
                                              wide_td_n, td_items, counts, kCountStride, stream);
                });
                break;
            case OP_TD_TWO:
                e = timed(RFIM_KERNEL_TD_TWO_F32, [&] {
                    return launch_td_two_f32(tab, tiny_td_n, td_tiny, L.a, seg, frec, wide_td_n, td_items, counts,
                                             kCountStride, stream);
                });
                break;
            case OP_FD_TWO:
                e = timed(RFIM_KERNEL_FD_TWO_F32, [&] {
                    return launch_fd_two_f32(tab, tiny_fd_n, fd_tiny, L.a, L.b, L.nbeams, seg, wide_fd_n, fd_items,
                                             counts, kCountStride, stream);
                });
                break;
            case OP_LIST_ALL:
                e = launch_list_all(L.b ? wide_fd_n : wide_td_n, L.b ? fd_items : td_items, L.a, L.total, stream);
                break;
            case OP_TD_COMPOSE:
                e = launch_td_compose_f32(frec, ffast, L.total, seg, stream);
                break;
            case OP_TD_WIDE:
                e = timed(RFIM_KERNEL_TD_WIDE_F32, [&] {
                    return launch_td_wide_f32(tab, wide_td_n, td_items, L.a, seg, frec, counts, kCountStride, stream);
                });
                break;
            case OP_FUSED_F32:
                e = timed(RFIM_KERNEL_FUSED_F32, [&] {
                    return launch_fused_f32(tab, L.nbeams, L.total, L.a, L.b, seg, frec, ffast, L.lds, tiny_fd_n, fd_tiny,
                                            wide_fd_n, fd_items, counts, kCountStride, stream);
                });
                break;
            case OP_FD_WIDE:
                e = timed(RFIM_KERNEL_FD_WIDE_F32, [&] {
                    return launch_fd_wide_f32(tab, wide_fd_n, fd_items, L.a, lp.f32_maxC, seg, counts, kCountStride, stream);
                });
                break;
        }
        if (e != hipSuccess) return dev_err(e);
    }
    return RFIM_OK;
}

// Builds and enqueues a whole step list, staging the beam tables through the
// workspace ring in one copy.
rfim_status execute(const rfim_beam* beams, int32_t nbeams, const LaunchPlan& lp, Workspace& ws,
                    hipStream_t stream, bool want_counts) {
    if (ws.has_last && ws.last_stream != stream) {
        // the shared workspace may still be in use by a call on another stream
        if (hipStreamWaitEvent(stream, ws.last_done, 0) != hipSuccess) return RFIM_ERR_DEVICE;
    }
    rfim_status st = ws.reserve_work(lp.work_bytes);
    if (st != RFIM_OK) return st;
    Program pg;
    build_program(beams, nbeams, lp, want_counts, pg);
    Slot* sl = nullptr;
    const size_t bytes = sizeof(DevBeam) * std::max<size_t>(1, pg.blob.size());
    st = ws.slot(bytes, &sl);
    if (st != RFIM_OK) return st;
    std::memcpy(sl->h, pg.blob.data(), sizeof(DevBeam) * pg.blob.size());
    if (hipMemcpyAsync(sl->d, sl->h, bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return RFIM_ERR_DEVICE;
    st = enqueue(pg, lp, (const DevBeam*)sl->d, (char*)ws.d_work, &ws, stream, want_counts);
    if (st != RFIM_OK) return st;
    if (hipEventRecord(sl->ev, stream) != hipSuccess) return RFIM_ERR_DEVICE;
    sl->used = true;
    if (hipEventRecord(ws.last_done, stream) != hipSuccess) return RFIM_ERR_DEVICE;
    ws.last_stream = stream;
    ws.has_last = true;
    return RFIM_OK;
}

// Number of DevBeam entries the program of these shapes uses (plans size
// their staging slots with it).
size_t program_entries(const rfim_beam* beams, int32_t nbeams, const LaunchPlan& lp) {
    Program pg;
    build_program(beams, nbeams, lp, true, pg);
    return pg.blob.size();
}

}  // namespace
}  // namespace rfim

using namespace rfim;

struct rfim_plan {
    int device = -1;
    std::vector<rfim_beam> shapes;
    std::vector<rfim_step> steps;
    LaunchPlan lp;
    Workspace ws;
    // captured graph of one run with fixed buffers
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* d_blob = nullptr;

    ~rfim_plan() {
        if (ws.has_last) (void)hipEventSynchronize(ws.last_done);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_blob) (void)hipFree(d_blob);
    }
};

namespace {

rfim_status check_plan_match(const rfim_plan* plan, const rfim_beam* beams, int32_t nbeams,
                             const rfim_step* steps, int32_t nsteps) {
    if ((int32_t)plan->shapes.size() != nbeams || (int32_t)plan->steps.size() != nsteps)
        return RFIM_ERR_INVALID_ARG;
    for (int i = 0; i < nbeams; i++) {
        const rfim_beam &a = beams[i], &p = plan->shapes[i];
        if (a.dtype != p.dtype || a.nchan != p.nchan || a.nsamp != p.nsamp || a.row_stride != p.row_stride ||
            (a.flags == nullptr) != (p.flags == nullptr))
            return RFIM_ERR_INVALID_ARG;
    }
    if (nsteps && std::memcmp(steps, plan->steps.data(), sizeof(rfim_step) * (size_t)nsteps) != 0)
        return RFIM_ERR_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return RFIM_ERR_INVALID_ARG;
    return RFIM_OK;
}

// With no step to run, out-of-place beams still receive a copy of the input
// and flags are cleared.
rfim_status copy_through(const rfim_beam* beams, int32_t nbeams, hipStream_t stream) {
    for (int i = 0; i < nbeams; i++) {
        const rfim_beam& b = beams[i];
        size_t es = elem_size(b.dtype);
        if (b.in != b.out &&
            hipMemcpy2DAsync(b.out, b.row_stride * es, b.in, b.row_stride * es, b.nsamp * es, b.nchan,
                             hipMemcpyDeviceToDevice, stream) != hipSuccess)
            return RFIM_ERR_DEVICE;
        if (b.flags && hipMemset2DAsync(b.flags, b.row_stride, 0, b.nsamp, b.nchan, stream) != hipSuccess)
            return RFIM_ERR_DEVICE;
    }
    return RFIM_OK;
}

}  // namespace

extern "C" {

const char* rfim_status_string(rfim_status s) {
    switch (s) {
        case RFIM_OK: return "ok";
        case RFIM_ERR_INVALID_ARG: return "invalid argument";
        case RFIM_ERR_UNSUPPORTED: return "unsupported by this build";
        case RFIM_ERR_OUT_OF_MEMORY: return "out of memory";
        case RFIM_ERR_DEVICE: return "HIP device or runtime error";
        case RFIM_ERR_BUDGET: return "HBM budget exhausted";
        case RFIM_ERR_MISMATCH: return "a tuning candidate's output differs from the default configuration's";
        case RFIM_ERR_SCRATCH: return "the call needs more than the fixed scratch array of the no-allocation entry point";
    }
    return "unknown status";
}

const char* rfim_version(void) { return "0.2.0"; }

rfim_status rfim_pipeline_run(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps,
                              int32_t nsteps, rfim_plan* plan, void* stream) {
    rfim_status st = validate(beams, nbeams, steps, nsteps);
    if (st != RFIM_OK) return st;
    if (nbeams == 0 || nsteps == 0) return copy_through(beams, nbeams, (hipStream_t)stream);
    if (plan) {
        st = check_plan_match(plan, beams, nbeams, steps, nsteps);
        if (st != RFIM_OK) return st;
        std::lock_guard<std::mutex> lk(plan->ws.mu);
        return execute(beams, nbeams, plan->lp, plan->ws, (hipStream_t)stream, true);
    }
    LaunchPlan lp;
    st = make_launch_plan(beams, nbeams, steps, nsteps, false, default_tune(), &lp);
    if (st != RFIM_OK) return st;
    Workspace* ws = nullptr;
    st = device_workspace(&ws);
    if (st != RFIM_OK) return st;
    std::lock_guard<std::mutex> lk(ws->mu);
    return execute(beams, nbeams, lp, *ws, (hipStream_t)stream, false);
}

rfim_status rfim_td_sigma_cut(const rfim_beam* beams, int32_t nbeams, double k, int32_t replace,
                              void* stream) {
    rfim_step s{RFIM_TD, replace, k, 0};
    return rfim_pipeline_run(beams, nbeams, &s, 1, nullptr, stream);
}

rfim_status rfim_fd_sigma_cut(const rfim_beam* beams, int32_t nbeams, double k, int64_t bin_size,
                              int32_t replace, void* stream) {
    rfim_step s{RFIM_FD, replace, k, bin_size};
    return rfim_pipeline_run(beams, nbeams, &s, 1, nullptr, stream);
}

}  // extern "C"

namespace rfim {

// a plan with explicit tuning parameters (the autotuner times candidates)
rfim_status plan_create_tuned(const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps, int32_t nsteps,
                              const TuneParams& tune, rfim_plan** out) {
    if (!out) return RFIM_ERR_INVALID_ARG;
    *out = nullptr;
    if (nbeams < 1 || nsteps < 1) return RFIM_ERR_INVALID_ARG;
    // shape-only validation: pointers are not dereferenced, use dummies
    std::vector<rfim_beam> tmp(shapes, shapes + nbeams);
    for (auto& b : tmp) b.in = b.out = (void*)(uintptr_t)4096;
    rfim_status st = validate(tmp.data(), nbeams, steps, nsteps);
    if (st != RFIM_OK) return st;
    rfim_plan* p = new (std::nothrow) rfim_plan();
    if (!p) return RFIM_ERR_OUT_OF_MEMORY;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return RFIM_ERR_DEVICE;
    }
    p->shapes.assign(shapes, shapes + nbeams);
    p->steps.assign(steps, steps + nsteps);
    st = make_launch_plan(shapes, nbeams, steps, nsteps, true, tune, &p->lp);
    if (st == RFIM_OK) st = p->ws.init(p->device);
    if (st == RFIM_OK) st = p->ws.reserve_work(p->lp.work_bytes);
    if (st == RFIM_OK) {
        // pre-size every staging slot for the beam tables of this plan
        size_t bytes = sizeof(DevBeam) * std::max<size_t>(1, program_entries(shapes, nbeams, p->lp));
        for (int i = 0; i < kRing && st == RFIM_OK; i++) {
            Slot* sl = nullptr;
            st = p->ws.slot(bytes, &sl);
        }
        p->ws.next = 0;
    }
    if (st != RFIM_OK) {
        delete p;
        return st;
    }
    p->ws.fixed = true;
    *out = p;
    return RFIM_OK;
}

}  // namespace rfim

extern "C" {

rfim_status rfim_plan_create(const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps,
                             int32_t nsteps, const char* tune_cache_path, rfim_plan** out) {
    if (!out) return RFIM_ERR_INVALID_ARG;
    *out = nullptr;
    TuneParams tune = default_tune();
    if (tune_cache_path && *tune_cache_path && nbeams > 0 && shapes && nsteps > 0 && steps) {
        const rfim_status st = tune_cache_lookup(tune_cache_path, shapes, nbeams, steps, nsteps, &tune);
        if (st != RFIM_OK && st != RFIM_ERR_UNSUPPORTED) return st;   // UNSUPPORTED: no entry yet
    }
    return plan_create_tuned(shapes, nbeams, steps, nsteps, tune, out);
}

rfim_status rfim_plan_destroy(rfim_plan* plan) {
    if (!plan) return RFIM_ERR_INVALID_ARG;
    delete plan;
    return RFIM_OK;
}

rfim_status rfim_plan_capture(rfim_plan* plan, const rfim_beam* beams, int32_t nbeams, void* stream) {
    if (!plan) return RFIM_ERR_INVALID_ARG;
    std::vector<rfim_step> steps = plan->steps;
    rfim_status st = validate(beams, nbeams, steps.data(), (int32_t)steps.size());
    if (st != RFIM_OK) return st;
    st = check_plan_match(plan, beams, nbeams, steps.data(), (int32_t)steps.size());
    if (st != RFIM_OK) return st;
    std::lock_guard<std::mutex> lk(plan->ws.mu);
    Workspace& ws = plan->ws;
    if (ws.has_last && hipEventSynchronize(ws.last_done) != hipSuccess) return RFIM_ERR_DEVICE;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->d_blob) (void)hipFree(plan->d_blob);
    plan->exec = nullptr;
    plan->graph = nullptr;
    plan->d_blob = nullptr;
    Program pg;
    build_program(beams, nbeams, plan->lp, true, pg);
    // the graph reads its beam tables from plan-owned device memory written
    // once here: replays carry no copies or memsets
    const size_t bytes = sizeof(DevBeam) * std::max<size_t>(1, pg.blob.size());
    if (hipMalloc(&plan->d_blob, bytes) != hipSuccess) return RFIM_ERR_OUT_OF_MEMORY;
    if (hipMemcpy(plan->d_blob, pg.blob.data(), sizeof(DevBeam) * pg.blob.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
        return RFIM_ERR_DEVICE;
    const bool timing = ws.timing;
    ws.timing = false;   // no timing events inside a graph
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        ws.timing = timing;
        return RFIM_ERR_DEVICE;
    }
    st = enqueue(pg, plan->lp, (const DevBeam*)plan->d_blob, (char*)ws.d_work, &ws, s, true);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    ws.timing = timing;
    if (st != RFIM_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return st != RFIM_OK ? st : RFIM_ERR_DEVICE;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return RFIM_ERR_DEVICE;
    }
    plan->graph = g;
    plan->exec = ex;
    return RFIM_OK;
}

rfim_status rfim_plan_replay(rfim_plan* plan, void* stream) {
    if (!plan) return RFIM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(plan->ws.mu);
    if (!plan->exec) return RFIM_ERR_INVALID_ARG;
    Workspace& ws = plan->ws;
    hipStream_t s = (hipStream_t)stream;
    if (ws.has_last && ws.last_stream != s && hipStreamWaitEvent(s, ws.last_done, 0) != hipSuccess)
        return RFIM_ERR_DEVICE;
    if (hipGraphLaunch(plan->exec, s) != hipSuccess) return RFIM_ERR_DEVICE;
    if (hipEventRecord(ws.last_done, s) != hipSuccess) return RFIM_ERR_DEVICE;
    ws.last_stream = s;
    ws.has_last = true;
    return RFIM_OK;
}

rfim_status rfim_plan_replay_on(rfim_plan* plan, const rfim_beam* beams, int32_t nbeams, void* stream) {
    if (!plan) return RFIM_ERR_INVALID_ARG;
    std::vector<rfim_step> steps = plan->steps;
    rfim_status st = validate(beams, nbeams, steps.data(), (int32_t)steps.size());
    if (st != RFIM_OK) return st;
    st = check_plan_match(plan, beams, nbeams, steps.data(), (int32_t)steps.size());
    if (st != RFIM_OK) return st;
    std::lock_guard<std::mutex> lk(plan->ws.mu);
    if (!plan->exec) return RFIM_ERR_INVALID_ARG;
    Workspace& ws = plan->ws;
    hipStream_t s = (hipStream_t)stream;
    if (ws.has_last && ws.last_stream != s && hipStreamWaitEvent(s, ws.last_done, 0) != hipSuccess)
        return RFIM_ERR_DEVICE;
    // same shapes, so the same program layout: only the tables' pointers change
    Program pg;
    build_program(beams, nbeams, plan->lp, true, pg);
    Slot* sl = nullptr;
    const size_t bytes = sizeof(DevBeam) * std::max<size_t>(1, pg.blob.size());
    st = ws.slot(bytes, &sl);
    if (st != RFIM_OK) return st;
    std::memcpy(sl->h, pg.blob.data(), sizeof(DevBeam) * pg.blob.size());
    if (hipMemcpyAsync(plan->d_blob, sl->h, sizeof(DevBeam) * pg.blob.size(), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return RFIM_ERR_DEVICE;
    if (hipGraphLaunch(plan->exec, s) != hipSuccess) return RFIM_ERR_DEVICE;
    if (hipEventRecord(sl->ev, s) != hipSuccess) return RFIM_ERR_DEVICE;
    sl->used = true;
    if (hipEventRecord(ws.last_done, s) != hipSuccess) return RFIM_ERR_DEVICE;
    ws.last_stream = s;
    ws.has_last = true;
    return RFIM_OK;
}

rfim_status rfim_plan_flag_counts(const rfim_plan* plan, uint64_t* host_out) {
    if (!plan || !host_out) return RFIM_ERR_INVALID_ARG;
    rfim_plan* p = const_cast<rfim_plan*>(plan);
    std::lock_guard<std::mutex> lk(p->ws.mu);
    const int nb = (int)p->shapes.size(), ns = (int)p->steps.size();
    if (!p->ws.has_last) {
        std::memset(host_out, 0, sizeof(uint64_t) * (size_t)nb * ns);
        return RFIM_OK;
    }
    if (hipEventSynchronize(p->ws.last_done) != hipSuccess) return RFIM_ERR_DEVICE;
    std::vector<unsigned long long> tmp((size_t)nb * kCountStride);
    if (hipMemcpy(tmp.data(), (char*)p->ws.d_work, tmp.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return RFIM_ERR_DEVICE;
    for (int b = 0; b < nb; b++)
        for (int s = 0; s < ns; s++) host_out[(size_t)b * ns + s] = tmp[(size_t)b * kCountStride + s];
    // a persistent launch whose bounded wait ran out left its output incomplete
    unsigned err = 0;
    char* ep = (char*)p->ws.d_work + p->lp.off_err;
    if (hipMemcpy(&err, ep, sizeof err, hipMemcpyDeviceToHost) != hipSuccess) return RFIM_ERR_DEVICE;
    if (err) {
        (void)hipMemset(ep, 0, sizeof err);
        return RFIM_ERR_DEVICE;
    }
    return RFIM_OK;
}

rfim_status rfim_plan_describe(const rfim_plan* plan, int32_t beam, int32_t run, rfim_plan_beam_info* out) {
    if (!plan || !out || beam < 0 || beam >= (int32_t)plan->shapes.size() || run < 0 ||
        run >= (int32_t)plan->lp.segs.size())
        return RFIM_ERR_INVALID_ARG;
    const LaunchPlan& lp = plan->lp;
    const rfim_beam& b = plan->shapes[beam];
    const Segment& seg = lp.segs[run];
    std::memset(out, 0, sizeof(*out));
    out->dtype = b.dtype;
    if (b.dtype == RFIM_U8) {
        out->tile_samples = lp.Tt[beam];
        out->tile_pitch = lp.Cp[beam];
        out->lds_bytes = (int64_t)lp.u8_lds;
        out->fd_path = fd_path_u8(b, lp.Tt[beam], seg, fd_vec_ok(plan->shapes.data(), lp, seg));
        return RFIM_OK;
    }
    int j = 0;
    while (lp.f32_beams[j] != beam) j++;
    const LaunchPlan::F32Shape& sh = lp.f_shape[run][j];
    out->td_threads = lp.f_nt[j];
    out->td_values_per_lane = lp.f_vpt[j];
    out->fd_bin = sh.B;
    out->fd_bins_per_lane = sh.B ? sh.bpl : 0;
    out->tile_samples = sh.B ? sh.Tt : 0;
    out->tile_pitch = sh.B ? sh.Cp : 0;
    out->lds_bytes = (int64_t)sh.lds;
    out->fd_path = seg.n_fd == 0 ? RFIM_FD_PATH_NONE : (sh.B ? RFIM_FD_PATH_F32_FAST : RFIM_FD_PATH_F32_WIDE);
    return RFIM_OK;
}

rfim_status rfim_plan_set_timing(rfim_plan* plan, int32_t enable) {
    if (!plan) return RFIM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(plan->ws.mu);
    if (plan->ws.has_last && hipEventSynchronize(plan->ws.last_done) != hipSuccess)
        return RFIM_ERR_DEVICE;
    plan->ws.clear_timing();
    plan->ws.timing = enable != 0;
    return RFIM_OK;
}

rfim_status rfim_plan_kernel_times(rfim_plan* plan, int32_t kind, uint64_t* launches,
                                   double* total_ms) {
    if (!plan || !launches || !total_ms || kind < 0 || kind >= RFIM_KERNEL_KINDS)
        return RFIM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(plan->ws.mu);
    if (plan->ws.has_last && hipEventSynchronize(plan->ws.last_done) != hipSuccess)
        return RFIM_ERR_DEVICE;
    uint64_t n = 0;
    double ms = 0.0;
    for (auto& t : plan->ws.timed) {
        if (t.kind != kind) continue;
        float e = 0.f;
        if (hipEventElapsedTime(&e, t.a, t.b) != hipSuccess) return RFIM_ERR_DEVICE;
        ms += e;
        n++;
    }
    *launches = n;
    *total_ms = ms;
    return RFIM_OK;
}

}  // extern "C"


// ---------------------------------------------------------------------------
// rfim_pipeline_run_noalloc: the plan-less run with its workspace and launch
// tables in a fixed device array instead of allocated memory.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[RFIM_NOALLOC_SCRATCH_BYTES];

namespace rfim {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch`.  In host code the
// array's name is only a host-side stand-in: kernels and copies must use the
// address the runtime returns for the current device.
rfim_status scratch_of_current_device(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RFIM_ERR_DEVICE;
    if (dev < 0 || dev >= kMaxDevices) return RFIM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return dev_err(e != hipSuccess ? e : hipErrorInvalidSymbol);
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return RFIM_OK;
}

// Launch tables reach the device as kernel arguments (copied at launch), so
// no pinned staging buffer is needed.
constexpr int kBlobWords = 240;
struct BlobChunk {
    uint64_t w[kBlobWords];
};

__global__ void k_store_words(uint64_t* __restrict__ dst, BlobChunk c, int n) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = c.w[i];
}

}  // namespace
}  // namespace rfim

extern "C" rfim_status rfim_pipeline_run_noalloc(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps,
                                                 int32_t nsteps, void* stream) {
    rfim_status st = validate(beams, nbeams, steps, nsteps);
    if (st != RFIM_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    if (nbeams == 0 || nsteps == 0) return copy_through(beams, nbeams, s);
    LaunchPlan lp;
    st = make_launch_plan(beams, nbeams, steps, nsteps, false, default_tune(), &lp);
    if (st != RFIM_OK) return st;
    Program pg;
    build_program(beams, nbeams, lp, false, pg);
    static_assert(sizeof(DevBeam) % 8 == 0, "launch tables are copied in 8-byte words");
    const size_t blob_off = (lp.work_bytes + 255) & ~(size_t)255;
    const size_t blob_bytes = sizeof(DevBeam) * pg.blob.size();
    if (blob_off + blob_bytes > (size_t)RFIM_NOALLOC_SCRATCH_BYTES) return RFIM_ERR_SCRATCH;
    void* base = nullptr;
    st = scratch_of_current_device(&base);
    if (st != RFIM_OK) return st;
    char* wbase = (char*)base;
    const uint64_t* words = (const uint64_t*)pg.blob.data();
    const size_t nwords = blob_bytes / 8;
    for (size_t w0 = 0; w0 < nwords; w0 += kBlobWords) {
        BlobChunk c;
        const int n = (int)std::min<size_t>(kBlobWords, nwords - w0);
        std::memcpy(c.w, words + w0, (size_t)n * 8);
        hipLaunchKernelGGL(k_store_words, dim3(1), dim3(256), 0, s, (uint64_t*)(wbase + blob_off) + w0, c, n);
        if (hipGetLastError() != hipSuccess) return RFIM_ERR_DEVICE;
    }
    return enqueue(pg, lp, (const DevBeam*)(wbase + blob_off), wbase, nullptr, s, false);
}
