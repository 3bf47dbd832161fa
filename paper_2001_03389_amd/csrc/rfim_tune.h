// Tuning parameters of a plan, the tuning cache (a JSON file of saved
// configurations, Section III of the paper: configurations found by the
// auto-tuner are saved and reused in production) and the host helpers the
// auto-tuner shares with the plan code.
#pragma once

#include <string>
#include <vector>

#include "rfim_internal.h"

namespace rfim {

struct TuneParams {
    int u8_tile_cap = 64;        // largest uint8 fused-kernel tile (samples, power of two)
    size_t f32_lds = 81920;      // LDS budget of a float32 fused work-group (bytes)
    int f32_tile_cap = 64;       // largest float32 fused-kernel tile (samples)
    size_t u8_lds = 51200;       // LDS budget of a uint8 fused work-group (bytes)
    int u8_sched = 0;            // uint8 schedule: 0 = TD pass then fused pass over the whole call,
                                 // 1 = one persistent beam-major launch per run
    int u8_td_rows = 4;          // uint8 TD pass: rows (waves) per work-group, 2, 4 or 8
};

// Defaults; RFIM_TILE_T, RFIM_F32_LDS, RFIM_F32_TILE_T, RFIM_U8_LDS, RFIM_U8_SCHED and
// RFIM_U8_TD_ROWS in the environment override them (experiments).
TuneParams default_tune();

// Cache key of an ordered list of beam shapes (dtype, nchan, nsamp,
// row_stride, flags on/off) and a step list.
std::string tune_key(const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps, int32_t nsteps);

// RFIM_OK and *out filled when the cache holds the key; RFIM_ERR_UNSUPPORTED
// when the file or the key is missing; RFIM_ERR_INVALID_ARG for a malformed
// entry.
rfim_status tune_cache_lookup(const char* path, const rfim_beam* shapes, int32_t nbeams,
                              const rfim_step* steps, int32_t nsteps, TuneParams* out);

// One timed candidate of a tuning run.
struct TuneRow {
    TuneParams p;
    double ms;
};

// Adds or replaces the key's entry (the file is rewritten through a
// temporary and a rename); `table` (may be empty) is recorded with it.
rfim_status tune_cache_store(const char* path, const rfim_beam* shapes, int32_t nbeams,
                             const rfim_step* steps, int32_t nsteps, const TuneParams& p, double ms,
                             const std::vector<TuneRow>& table);

// Host helpers defined in rfim_api.hip.
KExact make_k(double k);
size_t elem_size(int32_t dt);
rfim_status validate(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps, int32_t nsteps);
rfim_status plan_create_tuned(const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps, int32_t nsteps,
                              const TuneParams& tune, rfim_plan** out);

}  // namespace rfim
