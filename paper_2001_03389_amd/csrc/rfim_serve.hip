// Streaming serve loop: batches of one shape arrive per beam (each AMBER batch
// of Section IV; at the telescope's real-time rate one per batch period), are
// admitted against an HBM budget, mitigated in place in device memory
// (Section VI: mitigation happens in GPU memory) and completed with a latency.
//
// The loop is driven by its caller: rfim_serve_submit on each arrival and
// rfim_serve_poll as often as convenient, both with times on one clock.  A
// poll harvests finished launches (latency = completion - arrival) and forms
// batches of ready arrivals: a batch launches when it is full or when its
// oldest arrival has waited max_wait_s.  Three launch forms:
//   PER_CALL -- one rfim_pipeline_run per arrival, then a stream synchronise
//               (the plain form a user writes first);
//   BATCHED  -- up to max_batch arrivals per rfim_pipeline_run with a plan;
//   GRAPH    -- as BATCHED, through a HIP graph per batch size, rebound to the
//               batch's buffers on every replay.
// Memory: a pool of arrival slots (hbm_budget / batch bytes), at most
// ring_depth slots in flight per beam; an arrival that finds its beam's ring
// full or the pool empty is refused (RFIM_ERR_BUDGET).
// A mock executor (no HIP calls) models launches as cost_launch + k*cost_beam
// on one in-order device, so the scheduling logic is testable without a GPU.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "rfim_internal.h"
#include "rfim_tune.h"

namespace {

struct Arrival {
    int32_t beam;
    int32_t slot;
    double t_arr;
    void* dst;   // device output (nullptr: in place in the slot)
};

struct Running {
    std::vector<Arrival> arr;
    hipEvent_t done = nullptr;
    double t_end = 0.0;   // mock executor: modelled completion time
};

}  // namespace

struct rfim_serve {
    rfim_serve_config cfg;
    std::vector<rfim_step> steps;
    size_t bytes = 0;
    int nslots = 0;
    char* pool = nullptr;
    std::vector<int> free_slots;
    std::map<int32_t, int> in_flight;   // per beam
    std::deque<Arrival> pending;
    std::deque<Running> running;
    std::vector<hipEvent_t> events;
    hipStream_t stream = nullptr;
    hipEvent_t ref = nullptr;
    hipEvent_t src_ready = nullptr;   // orders slot copies after the caller's stream
    double t_ref = 0.0;
    std::chrono::steady_clock::time_point t0;
    std::map<int, rfim_plan*> plans;   // by batch size
    std::map<int, bool> captured;
    double mock_free = 0.0;
    rfim_serve_stats st{};
    uint64_t batch_sum = 0;
    std::vector<double> lat;

    double clock_now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    ~rfim_serve() {
        if (!cfg.mock) {
            if (stream) (void)hipStreamSynchronize(stream);
            for (auto& kv : plans) (void)rfim_plan_destroy(kv.second);
            for (auto& r : running)
                if (r.done) (void)hipEventDestroy(r.done);
            for (hipEvent_t e : events) (void)hipEventDestroy(e);
            if (ref) (void)hipEventDestroy(ref);
            if (src_ready) (void)hipEventDestroy(src_ready);
            if (pool) (void)hipFree(pool);
            if (stream) (void)hipStreamDestroy(stream);
        }
    }
};

namespace {

rfim_status take_event(rfim_serve* s, hipEvent_t* e) {
    if (!s->events.empty()) {
        *e = s->events.back();
        s->events.pop_back();
        return RFIM_OK;
    }
    return hipEventCreate(e) == hipSuccess ? RFIM_OK : RFIM_ERR_DEVICE;
}

// completions of every finished launch, in launch order
rfim_status harvest(rfim_serve* s, double now) {
    while (!s->running.empty()) {
        Running& r = s->running.front();
        double t_done;
        if (s->cfg.mock) {
            if (r.t_end > now) break;
            t_done = r.t_end;
        } else {
            const hipError_t q = hipEventQuery(r.done);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return RFIM_ERR_DEVICE;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s->ref, r.done) != hipSuccess) return RFIM_ERR_DEVICE;
            t_done = s->t_ref + ms * 1e-3;
            s->events.push_back(r.done);
        }
        for (const Arrival& a : r.arr) {
            const double l = std::max(0.0, t_done - a.t_arr);
            s->lat.push_back(l);
            if (l > s->cfg.deadline_s) s->st.deadline_misses++;
            s->free_slots.push_back(a.slot);
            if (--s->in_flight[a.beam] == 0) s->in_flight.erase(a.beam);
            s->st.completed++;
        }
        s->running.pop_front();
    }
    return RFIM_OK;
}

rfim_status launch_batch(rfim_serve* s, std::vector<Arrival>&& batch, double now) {
    const int k = (int)batch.size();
    Running r;
    if (s->cfg.mock) {
        const double start = std::max(now, s->mock_free);
        r.t_end = start + s->cfg.mock_launch_s + k * s->cfg.mock_beam_s;
        s->mock_free = r.t_end;
    } else {
        std::vector<rfim_beam> beams(k);
        for (int i = 0; i < k; i++) {
            rfim_beam& b = beams[i];
            std::memset(&b, 0, sizeof(b));
            b.dtype = s->cfg.dtype;
            b.nchan = s->cfg.nchan;
            b.nsamp = s->cfg.nsamp;
            b.row_stride = s->cfg.nsamp;
            void* slotp = s->pool + (size_t)batch[i].slot * s->bytes;
            b.in = slotp;
            b.out = batch[i].dst ? batch[i].dst : slotp;
            b.flags = nullptr;
        }
        rfim_plan*& plan = s->plans[k];
        if (!plan) {
            const rfim_status ps = rfim_plan_create(beams.data(), k, s->steps.data(), (int32_t)s->steps.size(),
                                                    nullptr, &plan);
            if (ps != RFIM_OK) {
                plan = nullptr;
                return ps;
            }
        }
        rfim_status rs;
        if (s->cfg.mode == RFIM_SERVE_GRAPH) {
            if (!s->captured[k]) {
                rs = rfim_plan_capture(plan, beams.data(), k, s->stream);
                if (rs == RFIM_OK) rs = rfim_plan_replay(plan, s->stream);
                s->captured[k] = rs == RFIM_OK;
            } else {
                rs = rfim_plan_replay_on(plan, beams.data(), k, s->stream);
            }
        } else {
            rs = rfim_pipeline_run(beams.data(), k, s->steps.data(), (int32_t)s->steps.size(), plan, s->stream);
        }
        if (rs != RFIM_OK) return rs;
        rfim_status es = take_event(s, &r.done);
        if (es != RFIM_OK) return es;
        if (hipEventRecord(r.done, s->stream) != hipSuccess) return RFIM_ERR_DEVICE;
        if (s->cfg.mode == RFIM_SERVE_PER_CALL && hipStreamSynchronize(s->stream) != hipSuccess)
            return RFIM_ERR_DEVICE;
    }
    r.arr = std::move(batch);
    s->running.push_back(std::move(r));
    s->st.launches++;
    s->batch_sum += (uint64_t)k;
    return RFIM_OK;
}

rfim_status form_batches(rfim_serve* s, double now, bool force) {
    const int maxb = s->cfg.mode == RFIM_SERVE_PER_CALL ? 1 : s->cfg.max_batch;
    while (!s->pending.empty()) {
        const int k = (int)std::min<size_t>((size_t)maxb, s->pending.size());
        if (k < maxb && !force && now - s->pending.front().t_arr < s->cfg.max_wait_s) break;
        std::vector<Arrival> batch(s->pending.begin(), s->pending.begin() + k);
        s->pending.erase(s->pending.begin(), s->pending.begin() + k);
        rfim_status rs = launch_batch(s, std::move(batch), now);
        if (rs != RFIM_OK) return rs;
        if (s->cfg.mode == RFIM_SERVE_PER_CALL) {
            rs = harvest(s, now);   // the launch has completed
            if (rs != RFIM_OK) return rs;
        }
    }
    return RFIM_OK;
}

}  // namespace

extern "C" {

rfim_status rfim_serve_create(const rfim_serve_config* cfg, const rfim_step* steps, int32_t nsteps,
                              rfim_serve** out) {
    if (!cfg || !out) return RFIM_ERR_INVALID_ARG;
    *out = nullptr;
    const rfim_serve_config& c = *cfg;
    if (c.reserved != 0 || c.ring_depth < 1 || c.max_batch < 1 || c.max_batch > 4096 || c.hbm_budget < 1 ||
        !(c.max_wait_s >= 0.0) || !(c.deadline_s > 0.0) ||
        (c.mode != RFIM_SERVE_PER_CALL && c.mode != RFIM_SERVE_BATCHED && c.mode != RFIM_SERVE_GRAPH) ||
        (c.mock != 0 && c.mock != 1) || !(c.mock_launch_s >= 0.0) || !(c.mock_beam_s >= 0.0))
        return RFIM_ERR_INVALID_ARG;
    rfim_beam shape;
    std::memset(&shape, 0, sizeof(shape));
    shape.dtype = c.dtype;
    shape.nchan = c.nchan;
    shape.nsamp = c.nsamp;
    shape.row_stride = c.nsamp;
    shape.in = shape.out = (void*)(uintptr_t)4096;
    rfim_status vs = rfim::validate(&shape, 1, steps, nsteps);
    if (vs != RFIM_OK) return vs;
    if (nsteps < 1) return RFIM_ERR_INVALID_ARG;
    const size_t bytes = (size_t)c.nchan * (size_t)c.nsamp * rfim::elem_size(c.dtype);
    const int64_t nslots = c.hbm_budget / (int64_t)bytes;
    if (nslots < 1) return RFIM_ERR_BUDGET;
    if (nslots > (1 << 30)) return RFIM_ERR_INVALID_ARG;
    rfim_serve* s = new (std::nothrow) rfim_serve();
    if (!s) return RFIM_ERR_OUT_OF_MEMORY;
    s->cfg = c;
    s->steps.assign(steps, steps + nsteps);
    s->bytes = bytes;
    s->nslots = (int)nslots;
    s->t0 = std::chrono::steady_clock::now();
    s->free_slots.reserve((size_t)nslots);
    for (int i = (int)nslots - 1; i >= 0; i--) s->free_slots.push_back(i);
    if (!c.mock) {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return RFIM_ERR_DEVICE;
        }
        if (hipMalloc((void**)&s->pool, (size_t)nslots * bytes) != hipSuccess) {
            s->pool = nullptr;
            delete s;
            return RFIM_ERR_OUT_OF_MEMORY;
        }
        // device timeline: completion times are read relative to this event
        if (hipEventCreate(&s->ref) != hipSuccess || hipEventRecord(s->ref, s->stream) != hipSuccess ||
            hipEventSynchronize(s->ref) != hipSuccess ||
            hipEventCreateWithFlags(&s->src_ready, hipEventDisableTiming) != hipSuccess) {
            delete s;
            return RFIM_ERR_DEVICE;
        }
        s->t_ref = s->clock_now();
    }
    *out = s;
    return RFIM_OK;
}

double rfim_serve_now(const rfim_serve* s) { return s ? s->clock_now() : 0.0; }

rfim_status rfim_serve_submit(rfim_serve* s, int32_t beam, const void* src, int32_t src_on_host, void* src_stream,
                              void* dst, double arrival_s) {
    if (!s || beam < 0 || (!s->cfg.mock && !src)) return RFIM_ERR_INVALID_ARG;
    s->st.submitted++;
    auto it = s->in_flight.find(beam);
    if (it != s->in_flight.end() && it->second >= s->cfg.ring_depth) {
        s->st.rejected_ring++;
        return RFIM_ERR_BUDGET;
    }
    if (s->free_slots.empty()) {
        s->st.rejected_budget++;
        return RFIM_ERR_BUDGET;
    }
    const int slot = s->free_slots.back();
    if (!s->cfg.mock) {
        if (!src_on_host && src_stream) {
            // the copy waits for the work the caller queued on src's stream
            if (hipEventRecord(s->src_ready, (hipStream_t)src_stream) != hipSuccess ||
                hipStreamWaitEvent(s->stream, s->src_ready, 0) != hipSuccess)
                return RFIM_ERR_DEVICE;
        }
        const hipMemcpyKind kind = src_on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        if (hipMemcpyAsync(s->pool + (size_t)slot * s->bytes, src, s->bytes, kind, s->stream) != hipSuccess)
            return RFIM_ERR_DEVICE;
    }
    s->free_slots.pop_back();
    s->in_flight[beam]++;
    s->pending.push_back({beam, slot, arrival_s, dst});
    s->st.admitted++;
    s->st.max_backlog = std::max<uint64_t>(s->st.max_backlog, s->pending.size());
    return RFIM_OK;
}

rfim_status rfim_serve_poll(rfim_serve* s, double now_s, uint64_t* completed_total) {
    if (!s) return RFIM_ERR_INVALID_ARG;
    rfim_status rs = harvest(s, now_s);
    if (rs == RFIM_OK) rs = form_batches(s, now_s, false);
    if (rs == RFIM_OK) rs = harvest(s, now_s);
    if (completed_total) *completed_total = s->st.completed;
    return rs;
}

rfim_status rfim_serve_drain(rfim_serve* s, double now_s) {
    if (!s) return RFIM_ERR_INVALID_ARG;
    rfim_status rs = form_batches(s, now_s, true);
    if (rs != RFIM_OK) return rs;
    if (s->cfg.mock) return harvest(s, std::max(now_s, s->mock_free));
    if (hipStreamSynchronize(s->stream) != hipSuccess) return RFIM_ERR_DEVICE;
    return harvest(s, now_s);
}

rfim_status rfim_serve_get_stats(rfim_serve* s, rfim_serve_stats* out) {
    if (!s || !out) return RFIM_ERR_INVALID_ARG;
    *out = s->st;
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto rank = [&](double q) {   // nearest rank
        if (v.empty()) return 0.0;
        size_t i = (size_t)std::ceil(q * (double)v.size());
        i = i == 0 ? 0 : i - 1;
        return v[std::min(i, v.size() - 1)];
    };
    out->p50_s = rank(0.50);
    out->p99_s = rank(0.99);
    out->max_s = v.empty() ? 0.0 : v.back();
    out->mean_batch = s->st.launches ? (double)s->batch_sum / (double)s->st.launches : 0.0;
    out->slots = (uint64_t)s->nslots;
    out->in_flight = (uint64_t)(s->nslots - (int)s->free_slots.size());
    return RFIM_OK;
}

rfim_status rfim_serve_destroy(rfim_serve* s) {
    if (!s) return RFIM_ERR_INVALID_ARG;
    delete s;
    return RFIM_OK;
}

}  // extern "C"
