// Auto-tuner and tuning cache (Section III of the paper: the kernels'
// parameters are tuned per setup and platform, and the configurations found
// are saved for production runs).
//
// rfim_autotune allocates beams of the requested shapes, fills them on the
// device with a deterministic pattern shaped like channelised telescope data,
// and times every candidate configuration with HIP events.  Every candidate's
// outputs and flags must be bit-identical to the default configuration's (the
// cuts are exact, so every launch shape must agree): a difference is a defect
// and fails the call.  The fastest candidate is written to the JSON cache
// file under a key made of the beam shapes and the step list, with the table
// of all candidates' times; rfim_plan_create reads it back.
//
// Cache file: one JSON object; each entry sits on its own line,
//   "<key>": {"u8_tile_cap": 64, "f32_lds": 81920, "f32_tile_cap": 64, "u8_lds": 51200, "u8_sched": 0,
//             "u8_td_rows": 4, "ms": 1.5, "candidates": 9, "table": [[64, 51200, 0, 4, 81920, 64, 1.5], ...]}
// (table rows: u8 tile cap, u8 LDS, u8 schedule, u8 TD rows per work-group, f32 LDS, f32 tile cap,
// ms per run)
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "rfim_tune.h"

namespace rfim {

TuneParams default_tune() {
    TuneParams p;
    if (const char* e = std::getenv("RFIM_TILE_T")) {
        const int v = std::atoi(e);
        if (v >= 4) p.u8_tile_cap = v;
    }
    if (const char* e = std::getenv("RFIM_F32_LDS")) {
        const long v = std::atol(e);
        if (v > 0) p.f32_lds = (size_t)v;
    }
    if (const char* e = std::getenv("RFIM_F32_TILE_T")) {
        const int v = std::atoi(e);
        if (v >= 4) p.f32_tile_cap = v;
    }
    if (const char* e = std::getenv("RFIM_U8_LDS")) {
        const long v = std::atol(e);
        if (v >= 4096) p.u8_lds = (size_t)v;
    }
    if (const char* e = std::getenv("RFIM_U8_SCHED")) {
        const int v = std::atoi(e);
        if (v == 0 || v == 1) p.u8_sched = v;
    }
    if (const char* e = std::getenv("RFIM_U8_TD_ROWS")) {
        const int v = std::atoi(e);
        if (v == 2 || v == 4 || v == 8) p.u8_td_rows = v;
    }
    return p;
}

std::string tune_key(const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps, int32_t nsteps) {
    std::string k;
    char buf[160];
    for (int i = 0; i < nbeams; i++) {
        const rfim_beam& b = shapes[i];
        std::snprintf(buf, sizeof buf, "%s%s%lldx%lld/%lld%s", i ? "," : "", b.dtype == RFIM_U8 ? "u8:" : "f32:",
                      (long long)b.nchan, (long long)b.nsamp, (long long)b.row_stride, b.flags ? "+f" : "");
        k += buf;
    }
    k += ";";
    for (int s = 0; s < nsteps; s++) {
        const rfim_step& st = steps[s];
        std::snprintf(buf, sizeof buf, "%s%s:%.17g:%s:%lld", s ? "," : "", st.domain == RFIM_TD ? "td" : st.domain == RFIM_FD ? "fd" : "tdm", st.k,
                      st.replace == RFIM_REPLACE_MEDIAN ? "median" : "mean", (long long)st.bin_size);
        k += buf;
    }
    return k;
}

namespace {

std::vector<std::string> read_lines(const char* path, bool* exists) {
    std::vector<std::string> lines;
    std::ifstream f(path);
    *exists = (bool)f;
    std::string l;
    while (f && std::getline(f, l)) lines.push_back(l);
    return lines;
}

// value of "name": <number> within an entry line
bool field(const std::string& line, const char* name, double* v) {
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    const char* s = line.c_str() + p + pat.size();
    char* end = nullptr;
    *v = std::strtod(s, &end);
    return end != s;
}

std::string entry_prefix(const std::string& key) { return "  \"" + key + "\": {"; }

}  // namespace

rfim_status tune_cache_lookup(const char* path, const rfim_beam* shapes, int32_t nbeams,
                              const rfim_step* steps, int32_t nsteps, TuneParams* out) {
    bool exists = false;
    const std::vector<std::string> lines = read_lines(path, &exists);
    if (!exists) return RFIM_ERR_UNSUPPORTED;
    const std::string pre = entry_prefix(tune_key(shapes, nbeams, steps, nsteps));
    for (const std::string& l : lines) {
        if (l.compare(0, pre.size(), pre) != 0) continue;
        double a = 0, b = 0, c = 0, d = 51200, e = 0, f = 4;
        if (!field(l, "u8_tile_cap", &a) || !field(l, "f32_lds", &b) || !field(l, "f32_tile_cap", &c))
            return RFIM_ERR_INVALID_ARG;
        (void)field(l, "u8_lds", &d);       // optional, default budget
        (void)field(l, "u8_sched", &e);     // optional, default schedule
        (void)field(l, "u8_td_rows", &f);   // optional, default rows per work-group
        if (a < 4 || a > 64 || b < 1024 || b > (1 << 20) || c < 4 || c > 64 || d < 4096 || d > (1 << 20) ||
            (e != 0 && e != 1) || (f != 2 && f != 4 && f != 8))
            return RFIM_ERR_INVALID_ARG;
        out->u8_td_rows = (int)f;
        out->u8_tile_cap = (int)a;
        out->f32_lds = (size_t)b;
        out->f32_tile_cap = (int)c;
        out->u8_lds = (size_t)d;
        out->u8_sched = (int)e;
        return RFIM_OK;
    }
    return RFIM_ERR_UNSUPPORTED;
}

rfim_status tune_cache_store(const char* path, const rfim_beam* shapes, int32_t nbeams,
                             const rfim_step* steps, int32_t nsteps, const TuneParams& p, double ms,
                             const std::vector<TuneRow>& table) {
    bool exists = false;
    const std::vector<std::string> lines = read_lines(path, &exists);
    const std::string pre = entry_prefix(tune_key(shapes, nbeams, steps, nsteps));
    std::vector<std::string> entries;
    for (const std::string& l : lines) {
        if (l.size() < 4 || l.compare(0, 3, "  \"") != 0) continue;   // braces and blank lines
        if (l.compare(0, pre.size(), pre) == 0) continue;             // replaced below
        std::string e = l;
        if (!e.empty() && e.back() == ',') e.pop_back();
        entries.push_back(e);
    }
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "\"u8_tile_cap\": %d, \"f32_lds\": %zu, \"f32_tile_cap\": %d, \"u8_lds\": %zu, "
                  "\"u8_sched\": %d, \"u8_td_rows\": %d, \"ms\": %.6f, \"candidates\": %zu, \"table\": [",
                  p.u8_tile_cap, p.f32_lds, p.f32_tile_cap, p.u8_lds, p.u8_sched, p.u8_td_rows, ms, table.size());
    std::string e = pre + buf;
    // table rows: [u8 tile cap, u8 LDS, u8 schedule, u8 TD rows, f32 LDS, f32 tile cap, ms per run]
    for (size_t i = 0; i < table.size(); i++) {
        const TuneRow& r = table[i];
        std::snprintf(buf, sizeof buf, "%s[%d, %zu, %d, %d, %zu, %d, %.6f]", i ? ", " : "", r.p.u8_tile_cap,
                      r.p.u8_lds, r.p.u8_sched, r.p.u8_td_rows, r.p.f32_lds, r.p.f32_tile_cap, r.ms);
        e += buf;
    }
    e += "]}";
    entries.push_back(e);
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return RFIM_ERR_INVALID_ARG;
        f << "{\n";
        for (size_t i = 0; i < entries.size(); i++) f << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
        f << "}\n";
        if (!f) return RFIM_ERR_INVALID_ARG;
    }
    if (std::rename(tmp.c_str(), path) != 0) return RFIM_ERR_INVALID_ARG;
    return RFIM_OK;
}

namespace {

// ---- device helpers of the tuner -------------------------------------------

__device__ inline uint32_t mix32(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}

// Deterministic test pattern shaped like channelised telescope data: per
// channel a level and a spread (uint8: level 60..100, spread 6..12; float32:
// level 0, spread 1), approximately normal noise (a sum of four uniforms),
// about 1.3 % of channels carrying persistent narrow-band interference of
// 5..20 spreads, and broadband impulses of 8 spreads in all channels at about
// 0.24 % of the time samples.  Samples past T in a row are zero.
__global__ void k_fill(void* p, int dtype, int64_t rows, int64_t stride, int64_t T, uint64_t seed) {
    const int64_t n = rows * stride;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / stride, t = i - r * stride;
        const uint32_t h = mix32(seed * 0x9E3779B97F4A7C15ull + (uint64_t)i);
        const uint32_t h2 = mix32((seed + 0x5851F42Dull) * 0xD1B54A32D192ED03ull + (uint64_t)i);
        const uint32_t hr = mix32(seed ^ (0xABCDull + (uint64_t)r * 77));
        const uint32_t ht = mix32((seed << 20) ^ (0x1234567ull + (uint64_t)t * 131));
        const float u = ((float)(h & 0xFFFFu) + (float)(h >> 16) + (float)(h2 & 0xFFFFu) + (float)(h2 >> 16)) *
                        (1.0f / 65536.0f);
        float z = (u - 2.0f) * 1.7320508f;   // mean 0, variance 1
        if (((hr >> 16) % 77u) == 0u) z += 5.0f + (float)((hr >> 24) & 15u);
        if ((ht % 417u) == 0u) z += 8.0f;
        if (dtype == RFIM_U8) {
            const float level = 60.0f + (float)(hr % 41u), spread = 6.0f + (float)((hr >> 8) % 7u);
            float v = rintf(level + spread * z);
            v = v < 0.0f ? 0.0f : (v > 255.0f ? 255.0f : v);
            ((uint8_t*)p)[i] = (uint8_t)(t < T ? (int)v : 0);
        } else {
            ((float*)p)[i] = t < T ? z : 0.0f;
        }
    }
}

// number of differing bytes between a and b over bytes [0, row_bytes) of
// each of `rows` rows `pitch` bytes apart (padding past nsamp is never
// written by the kernels and is not compared)
__global__ void k_count_diff(const uint8_t* a, const uint8_t* b, int64_t rows, int64_t pitch, int64_t row_bytes,
                             unsigned long long* out) {
    unsigned long long c = 0;
    const int64_t n = rows * row_bytes;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / row_bytes, t = i - r * row_bytes;
        c += a[r * pitch + t] != b[r * pitch + t];
    }
    if (c) atomicAdd(out, c);
}

struct TBeam {
    void* in = nullptr;
    void* out = nullptr;
    void* ref = nullptr;
    uint8_t* fl = nullptr;
    uint8_t* fref = nullptr;
    size_t bytes = 0, fbytes = 0;
};

void free_beams(std::vector<TBeam>& tb) {
    for (auto& t : tb) {
        if (t.in) (void)hipFree(t.in);
        if (t.out) (void)hipFree(t.out);
        if (t.ref) (void)hipFree(t.ref);
        if (t.fl) (void)hipFree(t.fl);
        if (t.fref) (void)hipFree(t.fref);
    }
    tb.clear();
}

}  // namespace
}  // namespace rfim

using namespace rfim;

extern "C" {

rfim_status rfim_tune_lookup(const char* path, const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps,
                             int32_t nsteps, int64_t* params) {
    if (!path || !shapes || nbeams < 1 || !steps || nsteps < 1 || !params) return RFIM_ERR_INVALID_ARG;
    TuneParams p;
    const rfim_status st = tune_cache_lookup(path, shapes, nbeams, steps, nsteps, &p);
    if (st != RFIM_OK) return st;
    params[0] = p.u8_tile_cap;
    params[1] = (int64_t)p.f32_lds;
    params[2] = p.f32_tile_cap;
    params[3] = (int64_t)p.u8_lds;
    params[4] = p.u8_sched;
    params[5] = p.u8_td_rows;
    return RFIM_OK;
}

rfim_status rfim_tune_store(const char* path, const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps,
                            int32_t nsteps, const int64_t* params, double ms) {
    if (!path || !shapes || nbeams < 1 || !steps || nsteps < 1 || !params) return RFIM_ERR_INVALID_ARG;
    TuneParams p;
    p.u8_tile_cap = (int)params[0];
    p.f32_lds = (size_t)params[1];
    p.f32_tile_cap = (int)params[2];
    p.u8_lds = (size_t)params[3];
    p.u8_sched = (int)params[4];
    p.u8_td_rows = (int)params[5];
    if (p.u8_tile_cap < 4 || p.u8_tile_cap > 64 || p.f32_lds < 1024 || p.f32_lds > (1u << 20) ||
        p.f32_tile_cap < 4 || p.f32_tile_cap > 64 || p.u8_lds < 4096 || p.u8_lds > (1u << 20) ||
        (p.u8_sched != 0 && p.u8_sched != 1) || (p.u8_td_rows != 2 && p.u8_td_rows != 4 && p.u8_td_rows != 8))
        return RFIM_ERR_INVALID_ARG;
    return tune_cache_store(path, shapes, nbeams, steps, nsteps, p, ms, {});
}

rfim_status rfim_autotune(const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps, int32_t nsteps,
                          const char* tune_cache_path, void* stream, double* best_ms) {
    if (!shapes || nbeams < 1 || !steps || nsteps < 1 || !tune_cache_path) return RFIM_ERR_INVALID_ARG;
    std::vector<rfim_beam> sh(shapes, shapes + nbeams);
    for (auto& b : sh) b.in = b.out = (void*)(uintptr_t)4096;
    rfim_status st = validate(sh.data(), nbeams, steps, nsteps);
    if (st != RFIM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    bool any_u8 = false, any_f32 = false;
    for (auto& b : sh) (b.dtype == RFIM_U8 ? any_u8 : any_f32) = true;

    // beams with the test pattern, outputs and reference outputs
    std::vector<TBeam> tb(nbeams);
    for (int i = 0; i < nbeams && st == RFIM_OK; i++) {
        const rfim_beam& b = shapes[i];
        TBeam& t = tb[i];
        t.bytes = (size_t)b.nchan * (size_t)b.row_stride * elem_size(b.dtype);
        t.fbytes = b.flags ? (size_t)b.nchan * (size_t)b.row_stride : 0;
        if (hipMalloc(&t.in, t.bytes) != hipSuccess || hipMalloc(&t.out, t.bytes) != hipSuccess ||
            hipMalloc(&t.ref, t.bytes) != hipSuccess)
            st = RFIM_ERR_OUT_OF_MEMORY;
        if (st == RFIM_OK && t.fbytes &&
            (hipMalloc((void**)&t.fl, t.fbytes) != hipSuccess || hipMalloc((void**)&t.fref, t.fbytes) != hipSuccess))
            st = RFIM_ERR_OUT_OF_MEMORY;
        if (st == RFIM_OK) {
            hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, t.in, b.dtype, b.nchan, b.row_stride, b.nsamp,
                               (uint64_t)(i + 1));
            if (hipGetLastError() != hipSuccess) st = RFIM_ERR_DEVICE;
        }
    }
    unsigned long long* d_diff = nullptr;
    if (st == RFIM_OK && hipMalloc(&d_diff, sizeof(unsigned long long)) != hipSuccess) st = RFIM_ERR_OUT_OF_MEMORY;
    if (st != RFIM_OK) {
        free_beams(tb);
        if (d_diff) (void)hipFree(d_diff);
        return st;
    }
    auto beams_to = [&](bool ref) {
        std::vector<rfim_beam> v(sh);
        for (int i = 0; i < nbeams; i++) {
            v[i].in = tb[i].in;
            v[i].out = ref ? tb[i].ref : tb[i].out;
            v[i].flags = shapes[i].flags ? (ref ? tb[i].fref : tb[i].fl) : nullptr;
        }
        return v;
    };

    // Search: the default first (it produces the reference outputs), then the
    // uint8 axes (tile cap, LDS budget, schedule, TD rows per work-group) on
    // the default float32 setting, then the float32 axes (LDS budget, tile
    // cap) on the best uint8 setting found.
    const TuneParams def = default_tune();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = RFIM_ERR_DEVICE;
    double best = 1e30;
    TuneParams bestp = def;
    std::vector<TuneRow> table;
    const int reps = 5;
    size_t ci = 0;
    auto same = [](const TuneParams& x, const TuneParams& y) {
        return x.u8_tile_cap == y.u8_tile_cap && x.u8_lds == y.u8_lds && x.u8_sched == y.u8_sched &&
               x.u8_td_rows == y.u8_td_rows && x.f32_lds == y.f32_lds && x.f32_tile_cap == y.f32_tile_cap;
    };
    auto evaluate = [&](const TuneParams& cand) {
        if (st != RFIM_OK) return;
        if (ci > 0 && same(cand, def)) return;   // the default was timed first
        const bool ref = ci == 0;
        ci++;
        rfim_plan* plan = nullptr;
        const rfim_status pc = plan_create_tuned(shapes, nbeams, steps, nsteps, cand, &plan);
        if (pc != RFIM_OK) {
            // a candidate whose tiles do not fit this device is not applicable;
            // the default must always be
            if (ref || pc != RFIM_ERR_UNSUPPORTED) st = pc;
            return;
        }
        const std::vector<rfim_beam> bv = beams_to(ref);
        st = rfim_pipeline_run(bv.data(), nbeams, steps, nsteps, plan, stream);   // warm-up (the reference first)
        if (st == RFIM_OK && !ref) {
            // bit-identical to the default configuration over [0, nsamp) of every row
            if (hipMemsetAsync(d_diff, 0, sizeof(unsigned long long), s) != hipSuccess) st = RFIM_ERR_DEVICE;
            for (int i = 0; i < nbeams && st == RFIM_OK; i++) {
                const rfim_beam& b = shapes[i];
                const int64_t es = (int64_t)elem_size(b.dtype);
                hipLaunchKernelGGL(k_count_diff, dim3(1024), dim3(256), 0, s, (const uint8_t*)tb[i].out,
                                   (const uint8_t*)tb[i].ref, b.nchan, b.row_stride * es, b.nsamp * es, d_diff);
                if (tb[i].fbytes)
                    hipLaunchKernelGGL(k_count_diff, dim3(1024), dim3(256), 0, s, (const uint8_t*)tb[i].fl,
                                       (const uint8_t*)tb[i].fref, b.nchan, b.row_stride, b.nsamp, d_diff);
                if (hipGetLastError() != hipSuccess) st = RFIM_ERR_DEVICE;
            }
            unsigned long long diff = 0;
            if (st == RFIM_OK &&
                (hipMemcpyAsync(&diff, d_diff, sizeof diff, hipMemcpyDeviceToHost, s) != hipSuccess ||
                 hipStreamSynchronize(s) != hipSuccess))
                st = RFIM_ERR_DEVICE;
            if (st == RFIM_OK && diff != 0) {
                std::fprintf(stderr,
                             "rfim_autotune: candidate (u8 tile cap %d, u8 LDS %zu, u8 schedule %d, u8 TD rows %d, "
                             "f32 LDS %zu, f32 tile cap %d) differs from the default configuration in %llu bytes\n",
                             cand.u8_tile_cap, cand.u8_lds, cand.u8_sched, cand.u8_td_rows, cand.f32_lds,
                             cand.f32_tile_cap, diff);
                st = RFIM_ERR_MISMATCH;
            }
        }
        if (st == RFIM_OK) {
            if (hipEventRecord(e0, s) != hipSuccess) st = RFIM_ERR_DEVICE;
            for (int r = 0; r < reps && st == RFIM_OK; r++)
                st = rfim_pipeline_run(bv.data(), nbeams, steps, nsteps, plan, stream);
            float ms = 0.f;
            if (st == RFIM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = RFIM_ERR_DEVICE;
            if (st == RFIM_OK) {
                const double per = ms / reps;
                table.push_back({cand, per});
                if (per < best) {
                    best = per;
                    bestp = cand;
                }
            }
        }
        (void)rfim_plan_destroy(plan);
    };
    evaluate(def);
    if (any_u8) {
        for (int a : {16, 32, 64})
            for (size_t ul : {(size_t)51200, (size_t)102400})
                for (int sc : {0, 1})
                    for (int rows : {2, 4, 8}) {
                        TuneParams p = def;
                        p.u8_tile_cap = a;
                        p.u8_lds = ul;
                        p.u8_sched = sc;
                        p.u8_td_rows = rows;
                        evaluate(p);
                    }
    }
    if (any_f32) {
        const TuneParams base = bestp;
        for (size_t l : {(size_t)40960, (size_t)81920, (size_t)163840})
            for (int c : {8, 64}) {
                TuneParams p = base;
                p.f32_lds = l;
                p.f32_tile_cap = c;
                if (!same(p, base)) evaluate(p);
            }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    free_beams(tb);
    (void)hipFree(d_diff);
    if (st != RFIM_OK) return st;
    if (best_ms) *best_ms = best;
    return tune_cache_store(tune_cache_path, shapes, nbeams, steps, nsteps, bestp, best, table);
}

}  // extern "C"
