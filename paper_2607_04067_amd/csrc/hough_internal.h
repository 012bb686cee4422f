// Internal declarations of libhough.so shared by its host API and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hough.h"

namespace hough {

// Lanes of a CDNA wavefront; every tile is a whole number of 64-column groups so that one
// lane owns one theta column.
constexpr int kWave = 64;
// Largest event of the fused batch kernel: a count then fits a packed 16-bit LDS counter, and
// each wave's keep flags fit a few registers (at most 8192 hits per wave, 64 per lane).
constexpr uint32_t kMaxBatchHits = 32767;
// Largest event whose duplicate hits the batch path suppresses: its hash table (twice as many
// 32-bit slots as hits, rounded up to a power of two) fits 64 KB of LDS.
constexpr uint32_t kDedupMaxHits = 8192;
constexpr uint32_t kDedupSlots = 2 * kDedupMaxHits;
// Under duplicate suppression a keep byte carries two bits until its event is finished: bit 0
// is the kept flag, bit 1 (this value) marks a later copy of a hit (set by the duplicate pass).
constexpr uint8_t kKeepDuplicate = 2;

// Grid constants as the kernels see them.
struct GridArgs {
    const float *C;      // [n_theta] (float)(A cos theta_j)
    const float *S;      // [n_theta] (float)(A sin theta_j)
    int32_t n_theta;
    int32_t n_rho;
    float Bf;            // (float)(-rho_min * A)
    float nrho_f;        // (float)n_rho
    float safe_r2;       // u^2 + v^2 below this: every vote of the hit is in range
    uint32_t threshold;
    int32_t rho_window;
    int32_t periodic;    // theta-periodic 3x3 test (HOUGH_FLAG_THETA_PERIODIC)
    int32_t dedup;       // later copies of a hit do not vote (HOUGH_FLAG_DEDUP)
    int32_t vote_rows;   // rho rows per LDS slab of hough_vote (n_rho when the column fits)
    int32_t peak_waves;  // theta rows per workgroup of hough_peaks (16, 8, 4 or 2)
    double wA, wB;       // A and B in double: the rho window of an event's hits (fused kernel)
};

// Launch shape of the fused batch kernel (chosen by the host; see plan_batch()).
struct BatchPlan {
    int waves;           // waves per workgroup
    int groups;          // 64-column groups per theta tile
    int tile_cols;       // 64 * groups, including one halo column on each side
    int out_cols;        // tile_cols - 2 output columns per tile
    int n_tiles;         // ceil(n_theta / out_cols)
    size_t lds_bytes;    // dynamic LDS per workgroup
    int per_cu;          // resident workgroups per CU (occupancy API)
    int grid;            // persistent workgroups
    int sparse;          // retention by peak list on tiles with few peaks (see kSparseRhoRows)
    int win;             // rows of a windowed tile (0: the tile holds the whole rho column)
    size_t split_lds_bytes;   // the split form's LDS (it always holds the whole column)
    int split_per_cu;    // its resident workgroups per CU
};
// Status bit of an event the fused (or split) kernel leaves to the spill kernel launched after
// it: more than kMaxBatchHits hits, or hits that reach beyond the rows of a windowed tile.  The
// spill kernel replaces the event's status.
constexpr uint32_t kStatusSpill = 0x80000000u;
// Grids with at least this many rho rows take the fused kernel's peak-list retention on tiles
// with few peaks (their votes spread over many rows, so a tile rarely has many peaks); so does
// every relative-threshold launch.  Other launches run the kernel compiled without it, which
// measured about 2% faster on grids whose tiles hold hundreds of peaks.
constexpr int kSparseRhoRows = 768;

struct BatchArgs {
    const float *x;
    const float *y;
    const uint32_t *offsets;
    const uint32_t *ids;            // null, or the pool event of each batch event (gather form)
    const uint32_t *keep_offsets;   // gather form: first keep byte of each batch event
    uint32_t n_events;
    hough_peak *peaks;
    uint32_t *n_peaks;
    uint8_t *keep;
    uint32_t *status;
    uint32_t max_peaks;
    const uint32_t *order;          // null, or the batch event taken at each queue position
    uint32_t *queue;     // [2] work counter and exit counter (device, zero between launches)
    uint32_t frac_num;   // fused kernel: frac_den != 0 takes each event's threshold as
    uint32_t frac_den;   // max(threshold, ceil(event maximum * frac_num / frac_den))
    uint32_t *spill_count;   // null, or a counter of the events left to the spill kernel
                             // (zero between launches; the spill kernel clears it)
};

// Workspace of the split form (one workgroup per theta tile of an event), laid out by
// split_layout() in the caller's buffer.  Everything in it is zero between launches.
struct SplitArgs {
    uint32_t n_tiles;
    uint32_t tile_cap;       // most peaks one tile can hold (no two peaks are 8-adjacent)
    uint32_t *counts;        // [n_events * n_tiles] peaks listed by each tile
    hough_peak *staged;      // [n_events * n_tiles * tile_cap] each tile's list, raster order
    uint32_t *kept;          // [n_events * kSplitKeepWords] keep bits of each event's hits
    uint32_t *done;          // [n_events] tiles finished; the last one merges
    uint32_t *flags;         // [n_events] HOUGH_EV_* bits seen by the tiles
};
constexpr uint32_t kSplitKeepWords = (kMaxBatchHits + 31) / 32 + 1;
size_t split_workspace_bytes(int n_theta, int n_rho, int groups, uint32_t n_events);
bool split_layout(int n_theta, int n_rho, int groups, uint32_t n_events, void *ws, size_t bytes,
                  SplitArgs *out);

// Spill path of the batch entry points (k_spill): events processed one per workgroup, the
// accumulator swept through rho slabs in LDS.  all = 1: every event (no fused kernel for the
// grid, or the split form on a grid whose column does not fit its tile); all = 0: the events
// the fused or split kernel flagged (kStatusSpill: above kMaxBatchHits hits, or beyond a
// windowed tile) and skipped.  Each workgroup owns `stride` 32-bit words of `work`: dilated
// retention bits (ceil(n_rho / 32) * n_theta), per (column, 32-row block) a peak-row mask and
// a place, per column a first place (n_theta + 1), and per block 16 peak counts.
struct SpillArgs {
    uint32_t *work;      // one slice of `stride` words per workgroup (spill_stride)
    size_t stride;
    uint32_t *queue;     // [3], zero between launches: all = 1: work and exit counters; all = 0:
                         // the count of events left to it, the exit counter, the block counter
    uint32_t all;
};
size_t spill_stride(int n_theta, int n_rho);
hipError_t launch_spill(const GridArgs &g, const BatchArgs &a, const SpillArgs &sp, int n_wg, hipStream_t s);

// Library-held scratch of hough_run_batch_split_static (hough_scratch.hip): one device array
// per device, its address taken once per device by scratch_init (called from hough_config
// with that device current).  Zero between calls, as the split form's workspace.
constexpr size_t kStaticScratchBytes = HOUGH_STATIC_SCRATCH_BYTES;
int scratch_init(int device);
void *scratch_ptr(int device);

// Phase slots of the instrumented build (HOUGH_PHASE_TIMING): clock ticks each workgroup of
// the fused kernel spent per phase, summed over workgroups, plus two counts.
enum PhaseSlot {
    kPhasePop = 0,       // taking the next event (work counter, barrier)
    kPhaseSetup,         // event set-up: keep bytes cleared, relative-threshold pass
    kPhaseVote,          // steps 1-3 of a tile
    kPhasePeaks,         // step 4: 3x3 test into peak bits
    kPhaseList,          // listing and dilation
    kPhaseRetain,        // step 5, and the tile cleared for the next one
    kPhaseFinish,        // flags, n_peaks and status of the event
    kPhaseEvents,        // count: events processed
    kPhaseStagedHits,    // count: valid hits x theta tiles (each staged hit votes every tile column)
    kPhaseSlots
};

// Largest-first schedule of the fused kernel: for batches of more events than resident
// workgroups (and at most kOrderMaxEvents of them) a one-workgroup pass sorts the events by
// hit count, largest first, in size classes of 1/64 of an octave, so that the last events
// taken from the work queue are the small ones.  Which workgroup runs an event never changes
// its results.
constexpr uint32_t kOrderMaxEvents = 1u << 16;

// Launchers (hough_kernels.hip).  All return a hipError_t from the launch.
// order[0 .. n_events) := the events of offsets (CSR, n_events + 1 entries) largest first.
hipError_t launch_order(const uint32_t *offsets, uint32_t n_events, uint32_t *order, hipStream_t s);
// Duplicate pass of the batch path: writes every keep byte of each well-formed event of at
// most kMaxBatchHits hits, kKeepDuplicate for a later copy of a hit and 0 otherwise (all 0 for
// events above kDedupMaxHits).
hipError_t launch_dedup(const BatchArgs &a, hipStream_t s);
// Launch shape of the iterative finder: `keys` candidate keys per chunk in LDS, and its
// suppression bitmap (bm_bytes per event) in LDS after them (gbm 0) or in device memory (gbm 1).
struct IterPlan {
    uint32_t keys;
    int gbm;
    size_t lds_bytes;    // dynamic LDS per workgroup
    size_t bm_bytes;     // bitmap bytes of one event (one bit per cell, whole 32-bit words)
};
// per_cu: workgroups per CU the plan should leave room for (the batch form runs one per event).
IterPlan plan_iterative(int n_theta, int n_rho, size_t lds_limit, int per_cu);
// The iterative finder over a CSR batch (a.ids must be null): acc holds n_events accumulators
// of n_theta * n_rho 16-bit cells; gbm (ip.gbm): n_events bitmaps of ip.bm_bytes.
hipError_t launch_batch_iterative(const GridArgs &g, const BatchArgs &a, uint16_t *acc, uint32_t frac_num,
                                  uint32_t frac_den, int r_theta, int r_rho, const IterPlan &ip, uint32_t *gbm,
                                  hipStream_t s);
hipError_t launch_vote(const GridArgs &g, const float *x, const float *y, uint32_t n_hits,
                       void *acc, int acc_type, hipStream_t s);
// counts: ceil(n_theta / kPeakRowsPerBlock) counters of device scratch (the context's).
constexpr int kPeakRowsPerBlock = 16;
hipError_t launch_peaks(const GridArgs &g, const void *acc, int acc_type, hough_peak *peaks,
                        uint32_t cap, uint32_t *n_peaks, uint32_t *counts, hipStream_t s);
hipError_t launch_retain(const GridArgs &g, const float *x, const float *y, uint32_t n_hits,
                         const hough_peak *peaks, const uint32_t *n_peaks, uint32_t cap,
                         uint8_t *keep, hipStream_t s);
hipError_t launch_batch(const GridArgs &g, const BatchPlan &p, const BatchArgs &a, hipStream_t s);
hipError_t launch_batch_split(const GridArgs &g, const BatchPlan &p, const BatchArgs &a,
                              const SplitArgs &sp, hipStream_t s);

// LDS needs and plans (hough_kernels.hip).
// LDS of hough_vote's workgroup for a slab of `rows` rho rows, and the tallest slab that fits.
size_t vote_lds_bytes(int rows);
int vote_slab_rows(int n_rho, size_t lds_limit);
// LDS of hough_peaks' workgroup of `waves` theta rows, and the most rows that fit (0: none).
size_t peaks_lds_bytes(int n_rho, int waves);
int peak_block_waves(int n_rho, size_t lds_limit);
hipError_t launch_track_params(const GridArgs &g, const float *x, const float *y, uint32_t n_hits,
                               const hough_peak *peaks, const uint32_t *n_peaks, uint32_t cap,
                               double rho_min, double rho_max, double b_tesla, hough_track *out,
                               hipStream_t s);
hipError_t launch_peaks_iterative(const GridArgs &g, const void *acc, int acc_type, uint32_t frac_num,
                                  uint32_t frac_den, int r_theta, int r_rho, hough_peak *peaks,
                                  uint32_t cap, uint32_t *n_peaks, uint32_t *status, const IterPlan &ip,
                                  uint32_t *gbm, hipStream_t s);
// LDS of the fused kernel's workgroup: the whole column (win 0) or a window of win rows.
size_t batch_lds_bytes(int n_rho, int waves, int groups, int win = 0);
int plan_batch(int n_theta, int n_rho, int waves, int groups, size_t lds_limit, BatchPlan *out, int win = 0,
               bool need_split = true);
int prepare_batch(BatchPlan *p);

}  // namespace hough
