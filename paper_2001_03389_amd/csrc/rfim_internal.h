// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rfim.h"

namespace rfim {

constexpr int kMaxSteps = 16;   // steps per pipeline (flags need <= 8)
constexpr int kCountStride = kMaxSteps;   // flag counters per beam: one per step
constexpr int kBlock = 256;     // work-group size of every kernel
constexpr int kB32MaxBins = 7;  // bins per lane in the uint8 32-channel FD path

// Threshold k as an exact binary fraction k = mk * 2^ek (mk odd).  mode:
//  0 = exact comparison with mk^2 = (mk2_hi:mk2_lo) and ek,
//  1 = k so small that only exact equality with the centre passes (k = 0),
//  2 = k so large that no sample can be an outlier (Samuelson's bound:
//      |x - mu| <= sigma * sqrt(n - 1), and n < 2^31 <= k^2).
struct KExact {
    uint64_t mk2_lo, mk2_hi;
    int32_t ek;
    int32_t mode;
    int32_t mk2_bits;  // bit length of mk^2
    int32_t pad;
    double k;  // the double itself, for estimates only
};

struct SegStep {
    KExact kx;
    int32_t replace;   // rfim_replace
    int32_t bit;       // flag bit (step index in the caller's list), -1 = none
    int64_t bin;       // FD bin size (resolved per beam when 0: see DevBeam)
    int32_t ci;        // step index in the caller's list: the flag counter of this step
    int32_t pad;
};

// One run of consecutive TD steps followed by consecutive FD steps.
struct Segment {
    int32_t n_td, n_fd;
    int32_t flags_mode;  // 0 = no flags, 1 = write fresh, 2 = OR into existing
    int32_t td_masked;   // 1: the TD steps are one run of masked steps
    SegStep td[kMaxSteps];
    SegStep fd[kMaxSteps];
};

// Device-side beam record of one launch.
struct DevBeam {
    const void* in;
    void* out;
    uint8_t* flags;
    int64_t C, T, stride;
    int64_t row0;    // first row of this beam in the launch (work-group mapping)
    int64_t tile0;   // first tile of this beam in the launch
    int64_t rec0;    // first row of this beam in the TD record array
    int32_t Tt;      // samples per tile of the fused kernel
    int32_t Cp;      // LDS elements per time sample of a tile (>= C, padded)
    int32_t cidx;    // index of the beam in the caller's list (flag counters)
    int32_t pad;     // float32: index in the call's float32 beam table (wide lists)
    int32_t path;    // uint8: FD path of the fused kernel (rfim_fd_path), chosen on the host
    int32_t pad2;
    int64_t item0;   // uint8 persistent schedule: first work item of this beam
};

// Host launchers (defined in the .hip files).  counts (nullable) receives, per
// beam, the number of samples each step replaced: counts[beam * count_stride + bit].
// rows_per_wg: 2, 4 or 8 rows (waves) per work-group
hipError_t launch_td_rows_u8(const DevBeam* d_beams, int nbeams, int64_t total_rows, int rows_per_wg,
                             const Segment& seg, uint32_t* d_rec, unsigned long long* d_counts,
                             int count_stride, hipStream_t s);
// vec: every FD step's per-lane bin share is a multiple of 16 bytes (see
// fd_vec_ok) so the 16-byte LDS path applies
hipError_t launch_fused_u8(const DevBeam* d_beams, int nbeams, int64_t total_tiles,
                           const Segment& seg, const uint32_t* d_rec, size_t lds_bytes, bool vec,
                           unsigned long long* d_counts, int count_stride, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
// The whole run in one persistent launch (beam-major work items: each beam's
// TD row groups, then its tiles; a tile waits for its beam's row groups).
// The launch table lists the beams queue by queue; queue q owns the items
// [base[q], base[q + 1]).  ctl: zeroed [kPersistQueues + 1 + nbeams] words
// (next item per queue, error flag, per-beam row groups done); a wait longer
// than spin_limit polls sets the error flag and stops the work-group;
// wait_extra (0 in use) raises the count a tile waits for (a test makes the
// waits run out with it).  grid: work-groups of the launch.
constexpr int kPersistQueues = 8;   // one per XCD
struct PersistQueues {
    int64_t base[kPersistQueues + 1];
};
hipError_t launch_persist_u8(const DevBeam* d_beams, int nbeams, const PersistQueues& qs, const Segment& seg,
                             uint32_t* d_rec, size_t lds_bytes, bool vec, unsigned long long* d_counts,
                             int count_stride, unsigned* ctl, uint32_t spin_limit, uint32_t wait_extra, int grid,
                             hipStream_t s);
// work-groups of the persistent launch that fit the device at once
int persist_u8_grid(size_t lds_bytes, bool vec);
size_t td_group_lds_bytes();

// float32 launchers.  TD kernels write float4 records (Lo, H, r, 0) per row
// and step, which launch_td_compose_f32 turns into composite ones;
// wide lists hold (float32 beam index, row or time sample) pairs after a
// counter.  nt x vpt: work-group size and values per lane of the TD kernel
// (nt * vpt >= T).  B, bpl: fast FD bin size (0 = none) and bins per lane.
hipError_t launch_td_rows_f32(const DevBeam* d_beams, int nbeams, int64_t total_rows, int nt, int vpt,
                              const Segment& seg, float4* rec, unsigned* tiny_n, int2* tiny_items, unsigned* wide_n,
                              int2* wide_items, unsigned long long* counts, int count_stride, hipStream_t s);
hipError_t launch_td_two_f32(const DevBeam* d_all, const unsigned* tiny_n, const int2* tiny_items, int grid,
                             const Segment& seg, float4* rec, unsigned* wide_n, int2* wide_items,
                             unsigned long long* counts, int count_stride, hipStream_t s);
// composite TD records (in place) and each row's innermost kept interval
// (fast), after every TD kernel of the run
hipError_t launch_td_compose_f32(float4* rec, float2* fast, int64_t rows, const Segment& seg, hipStream_t s);
hipError_t launch_fused_f32(const DevBeam* d_beams, int nbeams, int64_t total_tiles, int B, int bpl,
                            const Segment& seg, const float4* rec, const float2* fast, size_t lds_bytes,
                            unsigned* tiny_n,
                            int2* tiny_items, unsigned* wide_n, int2* wide_items, unsigned long long* counts,
                            int count_stride, hipStream_t s);
// time samples listed by the fused kernel for both windows; the all-beam
// table carries each beam's fast bin shape in Tt (B) and Cp (bins per lane)
hipError_t launch_fd_two_f32(const DevBeam* d_all, const unsigned* tiny_n, const int2* tiny_items, int grid, int B,
                             int bpl, const Segment& seg, unsigned* wide_n, int2* wide_items,
                             unsigned long long* counts, int count_stride, hipStream_t s);
hipError_t launch_td_wide_f32(const DevBeam* d_all, const unsigned* wide_n, const int2* items, int grid,
                              const Segment& seg, float4* rec, unsigned long long* counts, int count_stride,
                              hipStream_t s);
hipError_t launch_fd_wide_f32(const DevBeam* d_all, const unsigned* wide_n, const int2* items, int grid,
                              int64_t max_C, const Segment& seg, unsigned long long* counts, int count_stride,
                              hipStream_t s);
hipError_t launch_list_all(unsigned* wide_n, int2* items, int gidx, int64_t n, hipStream_t s);

}  // namespace rfim
