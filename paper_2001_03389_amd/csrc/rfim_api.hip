// Host side of the C ABI declared in include/rfim.h: argument validation,
// splitting a step list into runs of [TD steps][FD steps], per-launch beam
// tables, workspaces, plans and kernel launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "rfim_internal.h"

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

namespace {

constexpr int kRing = 64;                 // descriptor staging slots per workspace
// fused-kernel tile LDS per work-group: 160 KB per CU shared by 3 work-groups,
// less the kernel's static LDS (TD exception worklist and counters)
constexpr size_t kLdsBudget = 51200;
constexpr size_t kLdsMax = 65536;

KExact make_k(double k) {
    KExact r{};
    r.k = k;
    if (k < std::ldexp(1.0, -64)) {   // includes 0: k^2 * V < 1 for every V < 2^128
        r.mode = 1;
        return r;
    }
    if (k >= std::ldexp(1.0, 20)) {   // k^2 >= 2^40 > n - 1: nothing can be cut
        r.mode = 2;
        return r;
    }
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
    r.mode = 0;
    return r;
}

size_t elem_size(int32_t dt) { return dt == RFIM_U8 ? 1 : 4; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

size_t beam_span(const rfim_beam& b) {
    return (size_t)((b.nchan - 1) * b.row_stride + b.nsamp) * elem_size(b.dtype);
}

rfim_status validate(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps,
                     int32_t nsteps) {
    if (nbeams < 0 || nsteps < 0 || nsteps > kMaxSteps) return RFIM_ERR_INVALID_ARG;
    if (nbeams > 0 && !beams) return RFIM_ERR_INVALID_ARG;
    if (nsteps > 0 && !steps) return RFIM_ERR_INVALID_ARG;
    for (int s = 0; s < nsteps; s++) {
        const rfim_step& st = steps[s];
        if (st.domain != RFIM_TD && st.domain != RFIM_FD) return RFIM_ERR_INVALID_ARG;
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
    return RFIM_OK;
}

// The step list as runs of [consecutive TD steps][consecutive FD steps].
std::vector<Segment> segments_of(const rfim_step* steps, int32_t nsteps) {
    std::vector<Segment> out;
    int s = 0;
    while (s < nsteps) {
        Segment seg;
        std::memset(&seg, 0, sizeof(seg));
        while (s < nsteps && steps[s].domain == RFIM_TD) {
            SegStep& d = seg.td[seg.n_td++];
            d.kx = make_k(steps[s].k);
            d.replace = steps[s].replace;
            d.bit = s < 8 ? s : -1;
            d.bin = 0;
            s++;
        }
        while (s < nsteps && steps[s].domain == RFIM_FD) {
            SegStep& d = seg.fd[seg.n_fd++];
            d.kx = make_k(steps[s].k);
            d.replace = steps[s].replace;
            d.bit = s < 8 ? s : -1;
            d.bin = steps[s].bin_size;
            s++;
        }
        out.push_back(seg);
    }
    return out;
}

// Tile geometry of the fused kernel for one beam.
// Largest fused-kernel tile width allowed (samples, power of two in [4, 64]);
// RFIM_TILE_T in the environment caps it (tuning experiments).
int tile_cap() {
    static int cap = [] {
        const char* e = std::getenv("RFIM_TILE_T");
        int v = e ? std::atoi(e) : 64;
        int p = 4;
        while (p * 2 <= v && p < 64) p *= 2;
        return p;
    }();
    return cap;
}

bool tile_shape(const rfim_beam& b, bool flags, int32_t* Tt, int32_t* Cp) {
    if (b.nchan >= ((int64_t)1 << 24)) return false;   // worklist packs the row in 24 bits
    // 16-byte aligned time samples (vector LDS reads), padded off a multiple
    // of 256 bytes so the transposed stores of neighbouring lanes spread over banks
    int64_t cp = ((b.nchan + 15) / 16) * 16;
    if (cp % 256 == 0 || cp % 256 == 128) cp += 16;
    size_t per = (size_t)cp * (flags ? 2 : 1);
    int t = tile_cap();
    while (t > 4 && per * t > kLdsBudget) t >>= 1;
    if (per * t > kLdsMax) return false;
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
    hipStream_t aux = nullptr;          // second stream of the chunked schedule
    std::vector<hipEvent_t> chunk_ev;   // events of the chunked schedule

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
        for (hipEvent_t e : chunk_ev) (void)hipEventDestroy(e);
        if (aux) (void)hipStreamDestroy(aux);
    }

    // the auxiliary stream and at least n events for the chunked schedule
    rfim_status chunk_resources(size_t n) {
        if (!aux && hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) != hipSuccess)
            return RFIM_ERR_DEVICE;
        while (chunk_ev.size() < n) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return RFIM_ERR_DEVICE;
            chunk_ev.push_back(e);
        }
        return RFIM_OK;
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
        if (!timing) return launch();
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

// Everything one call needs to know about its launches.
struct LaunchPlan {
    // uint8 beams are processed in chunks of consecutive beams (by index in
    // u8_beams): chunk i is [chunk_begin[i], chunk_begin[i+1]).  With a TD
    // run, the row-statistics kernel of chunk i+1 (on an internal stream) runs
    // beside the fused kernel of chunk i, whose reads then come mostly from the
    // 256 MB Infinity Cache because chunk i was just read.
    std::vector<int> chunk_begin;
    std::vector<Segment> segs;
    std::vector<int> u8_beams;   // indices of uint8 beams
    std::vector<int> f32_beams;  // indices of float32 beams
    std::vector<int32_t> Tt, Cp; // per beam
    int64_t u8_rows = 0, u8_tiles = 0;
    size_t u8_lds = 0;
    int max_td = 0;
    size_t rec_bytes = 0, count_bytes = 0;
    int nsteps = 0;
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

rfim_status make_launch_plan(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps,
                             int32_t nsteps, bool want_counts, LaunchPlan* lp) {
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
        if (!tile_shape(b, b.flags != nullptr, &lp->Tt[i], &lp->Cp[i])) return RFIM_ERR_UNSUPPORTED;
        lp->u8_rows += b.nchan;
        lp->u8_tiles += (b.nsamp + lp->Tt[i] - 1) / lp->Tt[i];
        size_t lds = (size_t)lp->Tt[i] * lp->Cp[i] * (b.flags ? 2 : 1);
        lp->u8_lds = std::max(lp->u8_lds, lds);
    }
    if (!lp->f32_beams.empty()) return RFIM_ERR_UNSUPPORTED;
    if (lp->u8_rows >= ((int64_t)1 << 31) || lp->u8_tiles >= ((int64_t)1 << 31))
        return RFIM_ERR_UNSUPPORTED;
    {
        static const size_t chunk_bytes = [] {
            // off by default: measured slower on the 40-beam workload (3.1 vs
            // 1.5 ms per step) because the small per-chunk launches lose more
            // than the cache reuse gains
            const char* e = std::getenv("RFIM_CHUNK_MB");
            long v = e ? std::atol(e) : 0;
            return (size_t)(v > 0 ? v : 0) << 20;
        }();
        size_t acc = 0;
        lp->chunk_begin.clear();
        lp->chunk_begin.push_back(0);
        for (int j = 0; j < (int)lp->u8_beams.size(); j++) {
            const rfim_beam& b = beams[lp->u8_beams[j]];
            const size_t bytes = (size_t)b.nchan * (size_t)b.nsamp;
            if (chunk_bytes && acc > 0 && acc + bytes > chunk_bytes) {
                lp->chunk_begin.push_back(j);
                acc = 0;
            }
            acc += bytes;
        }
        lp->chunk_begin.push_back((int)lp->u8_beams.size());
    }
    lp->rec_bytes = (size_t)lp->u8_rows * std::max(1, lp->max_td) * 4;
    lp->rec_bytes = (lp->rec_bytes + 255) & ~(size_t)255;
    lp->count_bytes = want_counts ? (size_t)nbeams * 8 * sizeof(unsigned long long) : 0;
    return RFIM_OK;
}

hipError_t g_last_error = hipSuccess;

rfim_status dev_err(hipError_t e) {
    g_last_error = e;
    return e == hipSuccess ? RFIM_OK : RFIM_ERR_DEVICE;
}

// Enqueue a whole step list.  counts (device, nullable): [nbeams][8].
rfim_status execute(const rfim_beam* beams, int32_t nbeams, const LaunchPlan& lp, Workspace& ws,
                    hipStream_t stream, bool want_counts) {
    if (ws.has_last && ws.last_stream != stream) {
        // the shared workspace may still be in use by a call on another stream
        if (hipStreamWaitEvent(stream, ws.last_done, 0) != hipSuccess) return RFIM_ERR_DEVICE;
    }
    rfim_status st = ws.reserve_work(lp.rec_bytes + lp.count_bytes);
    if (st != RFIM_OK) return st;
    uint32_t* d_rec = (uint32_t*)ws.d_work;
    unsigned long long* d_counts =
        want_counts ? (unsigned long long*)((char*)ws.d_work + lp.rec_bytes) : nullptr;
    if (d_counts) {
        st = dev_err(launch_zero_u64(d_counts, (int64_t)nbeams * 8, stream));
        if (st != RFIM_OK) return st;
    }
    const int nu8 = (int)lp.u8_beams.size();
    const int nchunks = (int)lp.chunk_begin.size() - 1;
    for (size_t si = 0; si < lp.segs.size() && nu8 > 0; si++) {
        Segment seg = lp.segs[si];
        bool any_flags = false;
        for (int j = 0; j < nu8; j++) any_flags |= beams[lp.u8_beams[j]].flags != nullptr;
        seg.flags_mode = any_flags ? (si == 0 ? 1 : 2) : 0;
        const bool chunked = seg.n_td > 0 && nchunks > 1;
        hipStream_t ts = stream;   // stream of the row-statistics kernels
        if (chunked) {
            st = ws.chunk_resources(1 + 2 * (size_t)nchunks);
            if (st != RFIM_OK) return st;
            ts = ws.aux;
            // fork: the aux stream starts after everything already on `stream`
            if (hipEventRecord(ws.chunk_ev[0], stream) != hipSuccess ||
                hipStreamWaitEvent(ts, ws.chunk_ev[0], 0) != hipSuccess)
                return RFIM_ERR_DEVICE;
        }
        const int nparts = chunked ? nchunks : 1;
        int64_t row_base = 0;
        for (int ci = 0; ci < nparts; ci++) {
            const int jb = chunked ? lp.chunk_begin[ci] : 0, je = chunked ? lp.chunk_begin[ci + 1] : nu8;
            const int nt = je - jb;
            std::vector<DevBeam> tab(nt);
            int64_t row = 0, tile = 0;
            for (int j = 0; j < nt; j++) {
                const int bi = lp.u8_beams[jb + j];
                const rfim_beam& b = beams[bi];
                DevBeam& d = tab[j];
                d.in = si == 0 ? b.in : b.out;
                d.out = b.out;
                d.flags = b.flags;
                d.C = b.nchan;
                d.T = b.nsamp;
                d.stride = b.row_stride;
                d.row0 = row;
                d.tile0 = tile;
                d.Tt = lp.Tt[bi];
                d.Cp = lp.Cp[bi];
                d.cidx = bi;
                d.pad = 0;
                row += b.nchan;
                tile += (b.nsamp + d.Tt - 1) / d.Tt;
            }
            Slot* sl = nullptr;
            const size_t bytes = sizeof(DevBeam) * (size_t)nt;
            st = ws.slot(bytes, &sl);
            if (st != RFIM_OK) return st;
            std::memcpy(sl->h, tab.data(), bytes);
            if (chunked && ci >= 2) {
                // keep the statistics at most two chunks ahead of the fused
                // pass, so the chunk it reads is still cached
                if (hipStreamWaitEvent(ts, ws.chunk_ev[1 + 2 * (ci - 2) + 1], 0) != hipSuccess)
                    return RFIM_ERR_DEVICE;
            }
            st = dev_err(hipMemcpyAsync(sl->d, sl->h, bytes, hipMemcpyHostToDevice, ts));
            if (st != RFIM_OK) return st;
            const DevBeam* d_tab = (const DevBeam*)sl->d;
            uint32_t* rec = d_rec + row_base * std::max(1, seg.n_td);
            if (seg.n_td > 0) {
                st = dev_err(ws.timed_launch(RFIM_KERNEL_TD_ROWS_U8, ts, [&] {
                    return launch_td_rows_u8(d_tab, nt, row, seg, rec, d_counts, 8, ts);
                }));
                if (st != RFIM_OK) return st;
            }
            if (chunked) {
                hipEvent_t td_done = ws.chunk_ev[1 + 2 * ci];
                if (hipEventRecord(td_done, ts) != hipSuccess || hipStreamWaitEvent(stream, td_done, 0) != hipSuccess)
                    return RFIM_ERR_DEVICE;
            }
            const bool vec = fd_vec_ok(beams, lp, seg);
            st = dev_err(ws.timed_launch(RFIM_KERNEL_FUSED_U8, stream, [&] {
                return launch_fused_u8(d_tab, nt, tile, seg, rec, lp.u8_lds, vec, d_counts, 8, stream);
            }));
            if (st != RFIM_OK) return st;
            if (chunked && hipEventRecord(ws.chunk_ev[1 + 2 * ci + 1], stream) != hipSuccess)
                return RFIM_ERR_DEVICE;
            if (hipEventRecord(sl->ev, stream) != hipSuccess) return RFIM_ERR_DEVICE;
            sl->used = true;
            row_base += row;
        }
    }
    if (hipEventRecord(ws.last_done, stream) != hipSuccess) return RFIM_ERR_DEVICE;
    ws.last_stream = stream;
    ws.has_last = true;
    return RFIM_OK;
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
};

extern "C" {

const char* rfim_status_string(rfim_status s) {
    switch (s) {
        case RFIM_OK: return "ok";
        case RFIM_ERR_INVALID_ARG: return "invalid argument";
        case RFIM_ERR_UNSUPPORTED: return "unsupported by this build";
        case RFIM_ERR_OUT_OF_MEMORY: return "out of memory";
        case RFIM_ERR_DEVICE: return "HIP device or runtime error";
        case RFIM_ERR_BUDGET: return "HBM budget exhausted";
    }
    return "unknown status";
}

const char* rfim_version(void) { return "0.1.0"; }

rfim_status rfim_pipeline_run(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps,
                              int32_t nsteps, rfim_plan* plan, void* stream) {
    rfim_status st = validate(beams, nbeams, steps, nsteps);
    if (st != RFIM_OK) return st;
    if (nbeams == 0 || nsteps == 0) {
        // nothing to cut: out-of-place beams still receive a copy of the input
        for (int i = 0; i < nbeams; i++) {
            const rfim_beam& b = beams[i];
            size_t es = elem_size(b.dtype);
            if (b.in != b.out &&
                hipMemcpy2DAsync(b.out, b.row_stride * es, b.in, b.row_stride * es, b.nsamp * es,
                                 b.nchan, hipMemcpyDeviceToDevice, (hipStream_t)stream) != hipSuccess)
                return RFIM_ERR_DEVICE;
            if (b.flags &&
                hipMemset2DAsync(b.flags, b.row_stride, 0, b.nsamp, b.nchan, (hipStream_t)stream) !=
                    hipSuccess)
                return RFIM_ERR_DEVICE;
        }
        return RFIM_OK;
    }
    if (plan) {
        if ((int32_t)plan->shapes.size() != nbeams || (int32_t)plan->steps.size() != nsteps)
            return RFIM_ERR_INVALID_ARG;
        for (int i = 0; i < nbeams; i++) {
            const rfim_beam &a = beams[i], &p = plan->shapes[i];
            if (a.dtype != p.dtype || a.nchan != p.nchan || a.nsamp != p.nsamp ||
                a.row_stride != p.row_stride || (a.flags == nullptr) != (p.flags == nullptr))
                return RFIM_ERR_INVALID_ARG;
        }
        if (std::memcmp(steps, plan->steps.data(), sizeof(rfim_step) * (size_t)nsteps) != 0)
            return RFIM_ERR_INVALID_ARG;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return RFIM_ERR_INVALID_ARG;
        std::lock_guard<std::mutex> lk(plan->ws.mu);
        return execute(beams, nbeams, plan->lp, plan->ws, (hipStream_t)stream, true);
    }
    LaunchPlan lp;
    st = make_launch_plan(beams, nbeams, steps, nsteps, false, &lp);
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

rfim_status rfim_plan_create(const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps,
                             int32_t nsteps, const char* tune_cache_path, rfim_plan** out) {
    (void)tune_cache_path;
    if (!out) return RFIM_ERR_INVALID_ARG;
    *out = nullptr;
    if (nbeams < 1 || nsteps < 1) return RFIM_ERR_INVALID_ARG;
    // shape-only validation: pointers are not dereferenced, use dummies
    std::vector<rfim_beam> tmp(shapes, shapes + nbeams);
    for (auto& b : tmp) {
        b.in = b.out = (void*)(uintptr_t)4096;
    }
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
    st = make_launch_plan(shapes, nbeams, steps, nsteps, true, &p->lp);
    if (st == RFIM_OK) st = p->ws.init(p->device);
    if (st == RFIM_OK) st = p->ws.reserve_work(p->lp.rec_bytes + p->lp.count_bytes);
    if (st == RFIM_OK) {
        // pre-size every staging slot for the beam tables of this plan
        size_t bytes = sizeof(DevBeam) * (size_t)std::max<size_t>(1, nbeams);
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

rfim_status rfim_plan_destroy(rfim_plan* plan) {
    if (!plan) return RFIM_ERR_INVALID_ARG;
    delete plan;
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
    std::vector<unsigned long long> tmp((size_t)nb * 8);
    if (hipMemcpy(tmp.data(), (char*)p->ws.d_work + p->lp.rec_bytes, tmp.size() * 8,
                  hipMemcpyDeviceToHost) != hipSuccess)
        return RFIM_ERR_DEVICE;
    for (int b = 0; b < nb; b++)
        for (int s = 0; s < ns; s++) host_out[(size_t)b * ns + s] = s < 8 ? tmp[(size_t)b * 8 + s] : 0;
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
