/*
 * rfim.h -- C ABI of the MI355X (gfx950) RFI-mitigation library: iterative
 * time-domain and frequency-domain sigma cuts on channelised beam data
 * (RFIm, arXiv:2001.03389, Section IV).
 *
 * Data model
 *   A beam is a [nchan][row_stride] array in GPU memory, time fastest; samples
 *   [0, nsamp) of each channel row are processed, the rest of the row is never
 *   read or written.  Element type uint8 or float32 (finite values only).
 *   Beams are independent: no statistic ever crosses beams (Section V-B runs
 *   many beams side by side).
 *
 * Steps (Section IV)
 *   TD (time domain, Fig. 2): per channel, over the nsamp samples of the batch,
 *     mean mu and population standard deviation sigma; a sample with
 *     |x - mu| > k*sigma (strict, two-sided) is replaced.
 *   FD (frequency domain, Fig. 3): per time sample, channels are grouped into
 *     bins of bin_size consecutive channels (0 = one bin of all channels); the
 *     bin mean is subtracted from each channel, the same k*sigma test runs on
 *     these mean-corrected values over all channels, and the ORIGINAL value of
 *     an outlier is replaced by its bin's replacement value.
 *   Replacement strategy (Section IV, the strategy parameter): RFIM_REPLACE_MEAN
 *     = the step's mean rounded to the element type (uint8: nearest integer,
 *     ties to even; float32: nearest float32, ties to even); RFIM_REPLACE_MEDIAN
 *     = the lower median (rank floor((n-1)/2); float32 ordered by IEEE
 *     totalOrder).
 *   Each step reads the data as left by the previous step; the paper iterates
 *   the cuts (three iterations in production, Section V-B).
 *
 * Exactness
 *   Sums are exact integers and k is used as the exact binary value of the
 *   double, so flags and outputs are bit-identical to an exact evaluation of
 *   the definitions above, independent of launch shape.
 *
 * Asynchrony, ownership, errors
 *   Calls validate their arguments on the host and return synchronously with
 *   an error code; work is then enqueued on `stream` (a hipStream_t, NULL =
 *   the null stream) and the call returns without waiting.  The caller owns
 *   every in/out/flags buffer and must keep them alive until the stream
 *   reaches the work.  Calls without a plan use a library-owned workspace that
 *   may grow (hipMalloc) on first use of a larger shape; calls with a plan
 *   never allocate.  A device fault surfaces as RFIM_ERR_DEVICE from a later
 *   call or from the caller's own synchronisation.
 */
#ifndef RFIM_H
#define RFIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RFIM_OK = 0,
    RFIM_ERR_INVALID_ARG = -1,   /* argument outside the documented domain */
    RFIM_ERR_UNSUPPORTED = -2,   /* valid, but not handled by this build */
    RFIM_ERR_OUT_OF_MEMORY = -3, /* workspace allocation failed */
    RFIM_ERR_DEVICE = -4,        /* HIP runtime or device error */
    RFIM_ERR_BUDGET = -5,        /* admission refused: HBM budget exhausted */
    RFIM_ERR_MISMATCH = -6,      /* auto-tuner: a candidate configuration's output differs from the default's */
    RFIM_ERR_SCRATCH = -7        /* rfim_pipeline_run_noalloc: the call does not fit its fixed scratch array */
} rfim_status;

typedef enum { RFIM_U8 = 0, RFIM_F32 = 1 } rfim_dtype;
typedef enum { RFIM_REPLACE_MEAN = 0, RFIM_REPLACE_MEDIAN = 1 } rfim_replace;
/* RFIM_TD_MASKED: a TD step whose statistics, cut and replacement value use
 * only the samples of the row that no earlier step of the same run of
 * consecutive RFIM_TD_MASKED steps replaced (a reading of the iterated TD cut
 * of Sections IV and V-A in which a cut sample is set aside, not re-tested);
 * the run's mask starts empty, so its first step is an RFIM_TD step, and a
 * sample it cut keeps that step's replacement value and flag bit.  A row whose
 * samples are all set aside is left as it is.  uint8 beams only: a call with
 * a float32 beam returns RFIM_ERR_UNSUPPORTED. */
typedef enum { RFIM_TD = 0, RFIM_FD = 1, RFIM_TD_MASKED = 2 } rfim_domain;

/* One beam.  `in` and `out` are device pointers to [nchan][row_stride]
 * elements; out == in processes in place (the original data is then
 * overwritten), otherwise the two must not overlap.  `flags` (device, may be
 * NULL) is a [nchan][row_stride] uint8 array whose bit j is set where step j
 * replaced the sample; requires nsteps <= 8.  Constraints: 1 <= nchan < 2^31,
 * 1 <= nsamp < 2^31, row_stride >= nsamp.  float32 beams: values must be
 * finite; nchan and nsamp below 2^24, and nchan <= 19660 when the steps
 * include FD, else RFIM_ERR_UNSUPPORTED. */
typedef struct {
    int32_t dtype;    /* rfim_dtype */
    int32_t reserved; /* must be 0 */
    int64_t nchan;
    int64_t nsamp;
    int64_t row_stride; /* elements between consecutive channels */
    const void* in;
    void* out;
    uint8_t* flags;
} rfim_beam;

/* One step.  k must be finite and >= 0.  bin_size (FD only) must divide
 * nchan of every beam; 0 means a single bin of all channels. */
typedef struct {
    int32_t domain;  /* rfim_domain */
    int32_t replace; /* rfim_replace */
    double k;
    int64_t bin_size;
} rfim_step;

typedef struct rfim_plan rfim_plan; /* opaque */

/* Time-domain sigma cut (Section IV, Fig. 2): one TD step with threshold k
 * and replacement strategy r on each beam. */
rfim_status rfim_td_sigma_cut(const rfim_beam* beams, int32_t nbeams, double k, int32_t replace,
                              void* stream);

/* Frequency-domain sigma cut (Section IV, Fig. 3): one FD step with bins of
 * bin_size consecutive channels (0 = all channels). */
rfim_status rfim_fd_sigma_cut(const rfim_beam* beams, int32_t nbeams, double k, int64_t bin_size,
                              int32_t replace, void* stream);

/* Runs steps[0..nsteps) in order on every beam (the iterated TD + FD
 * mitigation of Section V).  plan may be NULL (library workspace) or a plan
 * created for the same beam shapes and steps. */
rfim_status rfim_pipeline_run(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps,
                              int32_t nsteps, rfim_plan* plan, void* stream);

/* Bytes of the fixed device scratch array of rfim_pipeline_run_noalloc. */
#define RFIM_NOALLOC_SCRATCH_BYTES (32u << 20)

/* rfim_pipeline_run for callers that cannot allocate: code under HIP-graph
 * capture, tight serving loops and harnesses that forbid hipMalloc.  It
 * calls no hipMalloc, hipHostMalloc or hipFree: the workspace and launch
 * tables of the call live in a file-scope device array of
 * RFIM_NOALLOC_SCRATCH_BYTES bytes (32 MiB), one copy per GPU, held from the
 * library's load until the process ends; launch tables reach it as kernel
 * arguments.  Beams, steps, results and argument errors are those of
 * rfim_pipeline_run(beams, nbeams, steps, nsteps, NULL, stream), with the
 * default kernel configuration and no flag counts.  Returns
 * RFIM_ERR_SCRATCH, before enqueuing anything, when the call needs more
 * (per TD step 4 bytes per uint8 row and 16 per float32 row; 24 bytes per
 * float32 row and 16 per float32 time sample; about 100 bytes of launch table
 * per beam and run: 16 float32 beams of 4096 x 65536 need about 22 MB).  Every call on a
 * GPU uses that GPU's one array and leaves its contents behind: calls that
 * overlap on one GPU (two streams, two host threads) race and must be
 * serialised by the caller; calls in order on one stream are safe. */
rfim_status rfim_pipeline_run_noalloc(const rfim_beam* beams, int32_t nbeams, const rfim_step* steps,
                                      int32_t nsteps, void* stream);

/* Creates a plan for beams of these shapes and dtypes (pointers are ignored,
 * except that a run must pass flags exactly where the shapes did) and this
 * step list: chooses kernel configurations (from the tuning cache
 * at tune_cache_path if given and present, else defaults) and allocates the
 * device workspace, so that rfim_pipeline_run with the plan never allocates.
 * Section III: tuned configurations are saved and reused in production. */
rfim_status rfim_plan_create(const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps,
                             int32_t nsteps, const char* tune_cache_path, rfim_plan** out);
rfim_status rfim_plan_destroy(rfim_plan* plan);

/* HIP-graph form of a plan (batched runs replayed without host work):
 * rfim_plan_capture records one run of the plan on these beams (shapes as the
 * plan's; the buffers are baked into the graph) into a graph owned by the
 * plan, replacing any earlier one; rfim_plan_replay launches it on `stream`.
 * The graph holds only kernel nodes (its beam tables are written once, at
 * capture).  Replays of one plan must not overlap. */
rfim_status rfim_plan_capture(rfim_plan* plan, const rfim_beam* beams, int32_t nbeams, void* stream);
rfim_status rfim_plan_replay(rfim_plan* plan, void* stream);
/* Replays the captured graph on other buffers of the plan's shapes: the
 * graph's beam tables are rewritten (one host-to-device copy on `stream`
 * ahead of the launch) with these beams' pointers.  Serving loops use it to
 * run each batch of arrivals through one graph launch. */
rfim_status rfim_plan_replay_on(rfim_plan* plan, const rfim_beam* beams, int32_t nbeams, void* stream);

/* Auto-tuner (Section III: parameters tuned per setup and platform, the
 * configurations saved for production).  Times every candidate kernel
 * configuration (uint8 tile cap and LDS budget, uint8 schedule, uint8 TD rows
 * per work-group, float32 LDS budget and tile cap: the uint8 axes on the
 * default float32 setting, then the float32 axes on the best uint8 one) for
 * these shapes and steps on freshly allocated beams filled
 * on the device with a deterministic pattern shaped like channelised
 * telescope data (per-channel level and spread, narrow-band channels,
 * broadband impulses), and stores the fastest in the JSON cache file
 * tune_cache_path (created or updated) with the table of every candidate's
 * time, where rfim_plan_create finds it.  Every candidate's output and flags
 * (samples [0, nsamp) of each row) must equal the default configuration's
 * byte for byte: the cuts are exact, so a difference is a defect, and the call
 * returns RFIM_ERR_MISMATCH (the candidate is named on stderr) without
 * writing the cache.  Synchronises `stream`; allocates (hipMalloc) three times
 * the shapes' bytes for the duration of the call.  *best_ms (may be NULL)
 * receives the best time per run. */
rfim_status rfim_autotune(const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps, int32_t nsteps,
                          const char* tune_cache_path, void* stream, double* best_ms);

/* Number of tuning parameters of a cache entry. */
#define RFIM_TUNE_NPARAMS 6

/* Tuning-cache access without a GPU: rfim_tune_lookup fills
 * params[RFIM_TUNE_NPARAMS] = {uint8 tile cap (samples), float32 LDS budget
 * (bytes), float32 tile cap, uint8 LDS budget (bytes), uint8 schedule (0 = a
 * TD pass then a fused pass over all beams of the call, 1 = one persistent
 * beam-major launch per run of [TD][FD] steps), uint8 TD rows per work-group
 * (2, 4 or 8)} for the key of these shapes
 * and steps (RFIM_ERR_UNSUPPORTED: no entry or no file); rfim_tune_store adds
 * or replaces that entry (RFIM_ERR_INVALID_ARG for values out of range). */
rfim_status rfim_tune_lookup(const char* path, const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps,
                             int32_t nsteps, int64_t* params);
rfim_status rfim_tune_store(const char* path, const rfim_beam* shapes, int32_t nbeams, const rfim_step* steps,
                            int32_t nsteps, const int64_t* params, double ms);

/* Per (beam, step) number of replaced samples of the most recent run with
 * this plan, copied to host_out[nbeams * nsteps]; synchronises the plan's
 * last stream. */
rfim_status rfim_plan_flag_counts(const rfim_plan* plan, uint64_t* host_out);

/* Which frequency-domain code path a plan runs for one beam and one run of
 * [TD steps][FD steps] (the launch shapes are the plan's; the outputs do not
 * depend on them). */
typedef enum {
    RFIM_FD_PATH_NONE = 0,         /* the run has no FD step */
    RFIM_FD_PATH_U8_BIN32_G4 = 1,  /* uint8, 32-channel bins, 4 lanes per time sample (64-sample tiles) */
    RFIM_FD_PATH_U8_BIN32_G8 = 2,  /* uint8, 32-channel bins, 8 lanes per time sample (32-sample tiles) */
    RFIM_FD_PATH_U8_BIN32_G16 = 3, /* uint8, 32-channel bins, 16 lanes per time sample (16-sample tiles) */
    RFIM_FD_PATH_U8_VEC = 4,       /* uint8, any bins, 16-byte LDS reads and dot4 sums */
    RFIM_FD_PATH_U8_BYTES = 5,     /* uint8, any bins, byte-wise */
    RFIM_FD_PATH_F32_FAST = 6,     /* float32, bins held in registers (bin size 8, 16, 32 or 64) */
    RFIM_FD_PATH_F32_WIDE = 7      /* float32, every time sample through the big-integer kernel */
} rfim_fd_path;

typedef struct {
    int32_t dtype;              /* rfim_dtype */
    int32_t fd_path;            /* rfim_fd_path */
    int32_t tile_samples;       /* time samples per work-group of the fused TD-apply + FD pass */
    int32_t tile_pitch;         /* LDS elements per time sample of that tile */
    int64_t lds_bytes;          /* dynamic LDS of the fused launch that holds the beam */
    int32_t td_threads;         /* float32 TD kernel: work-group size (0: rows go to the wide kernel); uint8: 0 */
    int32_t td_values_per_lane; /* float32 TD kernel: row values per lane; uint8: 0 */
    int32_t fd_bin;             /* float32 fast FD path: bin size (0: none); uint8: 0 */
    int32_t fd_bins_per_lane;   /* float32 fast FD path: bins per lane; uint8: 0 */
} rfim_plan_beam_info;

/* Launch configuration a plan chose for beam `beam` in run `run` (the step
 * list split into runs of consecutive TD steps followed by consecutive FD
 * steps, in order), written to *out.  Host only, no device work.
 * RFIM_ERR_INVALID_ARG for an index out of range. */
rfim_status rfim_plan_describe(const rfim_plan* plan, int32_t beam, int32_t run, rfim_plan_beam_info* out);

/* Kernels the library launches, for per-kernel timing. */
typedef enum {
    RFIM_KERNEL_TD_ROWS_U8 = 0,  /* uint8 row statistics + TD decisions */
    RFIM_KERNEL_FUSED_U8 = 1,    /* uint8 TD apply + FD steps + write-back */
    RFIM_KERNEL_TD_ROWS_F32 = 2, /* float32 register-resident rows: TD steps */
    RFIM_KERNEL_FUSED_F32 = 3,   /* float32 TD apply + FD steps + write-back */
    RFIM_KERNEL_TD_WIDE_F32 = 4, /* float32 rows outside the fast window */
    RFIM_KERNEL_FD_WIDE_F32 = 5, /* float32 time samples outside the fast window */
    RFIM_KERNEL_TD_TWO_F32 = 6,  /* float32 rows needing a second fixed-point window */
    RFIM_KERNEL_FD_TWO_F32 = 7,  /* float32 time samples needing a second window */
    RFIM_KERNEL_PERSIST_U8 = 8,  /* uint8 persistent beam-major launch: TD pass + fused pass */
    RFIM_KERNEL_KINDS = 9
} rfim_kernel_kind;

/* Per-kernel timing of a plan (Section V-B reports execution time averaged
 * over many runs).  enable != 0 brackets every kernel the plan launches with
 * HIP events on the launch stream and clears the accumulated record; 0 stops
 * timing.  rfim_plan_kernel_times waits for the plan's last run and returns,
 * for one kernel kind, the number of timed launches and their summed duration
 * in milliseconds. */
rfim_status rfim_plan_set_timing(rfim_plan* plan, int32_t enable);
rfim_status rfim_plan_kernel_times(rfim_plan* plan, int32_t kind, uint64_t* launches,
                                   double* total_ms);

/* ---- Streaming serve loop ------------------------------------------------
 * Beams deliver batches of one shape (Section IV: mitigation runs per AMBER
 * batch; at the real-time rate one batch per batch period per beam).  The
 * loop is driven by the caller on one clock (seconds; rfim_serve_now gives
 * the loop's own steady clock, which GPU completions are measured on):
 *   rfim_serve_submit   admits one arrival: its data (host or device memory,
 *                       one contiguous [nchan][nsamp] batch of the loop's dtype)
 *                       is copied into a slot of the loop's device pool; refused
 *                       with RFIM_ERR_BUDGET when the pool (hbm_budget bytes) is
 *                       full or the beam already has ring_depth arrivals in
 *                       flight.  A device src produced on stream src_stream
 *                       (may be NULL: src is complete already) is copied after
 *                       the work queued there so far; a host src must stay
 *                       unchanged until the arrival completes.  The mitigated
 *                       batch goes to dst (device, contiguous [nchan][nsamp],
 *                       not overlapping the pool; must stay valid until the
 *                       arrival completes) or, with dst NULL, stays in the slot;
 *   rfim_serve_poll     harvests finished launches (latency = completion -
 *                       arrival) and launches batches of ready arrivals: a
 *                       batch goes when it holds max_batch arrivals or its
 *                       oldest arrival has waited max_wait_s;
 *   rfim_serve_drain    launches what is pending and waits for everything;
 *   rfim_serve_get_stats counts, latency percentiles (nearest rank) and
 *                       misses of deadline_s.
 * mode: RFIM_SERVE_PER_CALL (one pipeline run per arrival, then a stream
 * synchronise), RFIM_SERVE_BATCHED (plans of up to max_batch beams),
 * RFIM_SERVE_GRAPH (as BATCHED through one HIP graph per batch size).
 * mock = 1 runs no GPU work: a launch of k arrivals then takes
 * mock_launch_s + k * mock_beam_s on one in-order device (scheduler tests).
 * Mitigation is in place in the pool slot; the loop is single-threaded (one
 * caller thread per loop). */
typedef enum { RFIM_SERVE_PER_CALL = 0, RFIM_SERVE_BATCHED = 1, RFIM_SERVE_GRAPH = 2 } rfim_serve_mode;

typedef struct {
    int32_t dtype;      /* rfim_dtype of every arrival */
    int32_t reserved;   /* must be 0 */
    int64_t nchan, nsamp;
    int32_t ring_depth; /* arrivals in flight per beam, >= 1 */
    int32_t max_batch;  /* arrivals per launch, 1..4096 */
    int64_t hbm_budget; /* bytes of the device slot pool */
    double max_wait_s;  /* >= 0 */
    double deadline_s;  /* > 0 */
    int32_t mode;       /* rfim_serve_mode */
    int32_t mock;       /* 0 or 1 */
    double mock_launch_s, mock_beam_s;
} rfim_serve_config;

typedef struct {
    uint64_t submitted, admitted, rejected_budget, rejected_ring, completed, launches;
    uint64_t deadline_misses, max_backlog, slots, in_flight;
    double p50_s, p99_s, max_s, mean_batch;
} rfim_serve_stats;

typedef struct rfim_serve rfim_serve; /* opaque */

rfim_status rfim_serve_create(const rfim_serve_config* cfg, const rfim_step* steps, int32_t nsteps,
                              rfim_serve** out);
double rfim_serve_now(const rfim_serve* srv);
rfim_status rfim_serve_submit(rfim_serve* srv, int32_t beam, const void* src, int32_t src_on_host,
                              void* src_stream, void* dst, double arrival_s);
rfim_status rfim_serve_poll(rfim_serve* srv, double now_s, uint64_t* completed_total);
rfim_status rfim_serve_drain(rfim_serve* srv, double now_s);
rfim_status rfim_serve_get_stats(rfim_serve* srv, rfim_serve_stats* out);
rfim_status rfim_serve_destroy(rfim_serve* srv);

/* Human-readable text for a status code (static storage). */
const char* rfim_status_string(rfim_status s);

/* Library version as "major.minor.patch" (static storage). */
const char* rfim_version(void);

/* ---- Dedispersion and detection (the stage after RFI mitigation) ------------
 * Section I and Eq. 2: a dispersed pulse reaches channel c, centred at
 * f_c = f_low + (c + 1/2) * chan_bw (MHz, channel 0 lowest), later than the
 * top channel's centre f_top by k_DM * DM * (f_c^-2 - f_top^-2) seconds with
 * k_DM = 4.15e3 MHz^2 pc^-1 cm^3 s; incoherent dedispersion shifts every
 * channel back by its delay (in samples: the delay over tsamp, rounded to the
 * nearest integer, ties to even, evaluated in FP64) and sums the channels.
 * Section V-A uses the dedispersed series to show that mitigation keeps a
 * dispersed pulse detectable. */
typedef struct rfim_dedisp rfim_dedisp; /* opaque: delay tables of one band and DM list */

/* Computes the delays of every trial DM (dms[0..ndm), 1 <= ndm <= 65535,
 * each finite and >= 0) for nchan channels (1 <= nchan < 2^23) and uploads the library's device
 * tables (allocates).  INVALID_ARG for arguments outside these domains or a
 * delay beyond 2^31 - 1 samples. */
rfim_status rfim_dedisp_create(int64_t nchan, double f_low_mhz, double chan_bw_mhz, double tsamp_s,
                               const double* dms, int32_t ndm, rfim_dedisp** out);
rfim_status rfim_dedisp_destroy(rfim_dedisp* dd);

/* Host copy of the delays, [ndm][nchan] samples (host_delays may be NULL),
 * and the largest of them (max_delay may be NULL). */
rfim_status rfim_dedisp_delays(const rfim_dedisp* dd, int32_t* host_delays, int32_t* max_delay);

/* series[d][t] = sum over channels c in ascending order of beam[c][t +
 * delay_d(c)] for t in [0, nout), every trial d: device output [ndm][nout],
 * int32 for uint8 beams (exact) or double for float32 beams (FP64 sums added
 * in channel order).  Reads beam->in only ([nchan][row_stride], nchan as at
 * creation); requires 1 <= nout <= nsamp - max_delay, else INVALID_ARG.
 * Asynchronous on `stream`; the current device must be the creation device. */
rfim_status rfim_dedisperse(const rfim_dedisp* dd, const rfim_beam* beam, int64_t nout, void* series,
                            void* stream);

/* Detection statistics of nseries device series of n values each, stored
 * contiguously ([nseries][n]); dtype RFIM_U8 names int32 series (as
 * rfim_dedisperse writes for uint8 beams), RFIM_F32 double series.  Device
 * output stats[i][0..5) = SNR = (peak - mean) / std (0 when std = 0), peak
 * (the largest value), its first index, mean, population standard deviation.
 * int32 series: exact integer sums, then FP64; double series: two FP64
 * passes.  1 <= n < 2^32. */
rfim_status rfim_series_stats(int32_t dtype, const void* series, int32_t nseries, int64_t n, double* stats,
                              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RFIM_H */
