/*
 * hough.h -- C ABI of libhough.so, the MI355X (gfx950) conformal Hough transform for
 * drift-chamber hits.
 *
 * The library runs the data-parallel hot path of the matrix-based conformal Hough transform:
 *   1. conformal map of each hit (x, y) -> (u, v) = (x, y) / (x^2 + y^2)          [Eq. (1)]
 *   2. theta sweep: rho_ij = u_i cos(theta_j) + v_i sin(theta_j) for every hit and every
 *      theta column, binned on a uniform (theta, rho) grid                       [Sec. II, Sec. III]
 *   3. voting into a per-event integer accumulator acc[theta][rho]              [Sec. II, Sec. III]
 *   4. threshold + 3x3 local-maximum peaks, returned in raster order            [Sec. II]
 *   5. the retention mask: a hit is kept when it lies within rho_window rho bins
 *      of a peak at the peak's own theta                                       [Sec. I, Sec. II]
 * An event is the point set of hit wire positions {(x_i, y_i)} of Sec. II.  Beside them:
 * the paper's own peak finder (relative threshold and iterative extraction, Sec. II) and the
 * candidate circles / track parameters of a peak list (Eq. (2)).
 *
 * Exact rules (every result is an integer and is reproduced bit for bit by the CPU oracle):
 *   - theta_j = (j * pi) / n_theta in double (lower bin edge), j = 0 .. n_theta-1.
 *   - A = n_rho / (rho_max - rho_min), B = -rho_min * A in double; per column
 *     C_j = (float)(A cos theta_j), S_j = (float)(A sin theta_j); Bf = (float)B.
 *   - a hit is valid iff r2 = fmaf(x, x, y*y) satisfies 0 < r2 <= FLT_MAX; then u = x/r2 and
 *     v = y/r2 (IEEE single-precision division).  Invalid hits vote nowhere and are never kept.
 *   - bin of hit i in column j: w = fmaf(v, S_j, Bf); t = fmaf(u, C_j, w); in range iff
 *     0 <= t < n_rho, and then k = (int)t.  Out-of-range votes are dropped.
 *   - acc[j][k] = number of valid hits whose bin in column j is k.
 *   - (j, k) is a peak iff acc[j][k] >= threshold and, for each of its 8 neighbours inside the
 *     grid, acc[j][k] > neighbour when the neighbour comes first in raster order (smaller j,
 *     or equal j and smaller k) and acc[j][k] >= neighbour otherwise.  theta does not wrap
 *     unless the context asks for it (HOUGH_FLAG_THETA_PERIODIC).
 *   - keep_i = 1 iff hit i is valid and some peak (jp, kp) has hit i's bin in column jp in
 *     range with |bin - kp| <= rho_window.
 *
 * Memory and streams: every array argument is a DEVICE pointer owned by the caller (for
 * instance torch tensors' data pointers).  `stream` is a hipStream_t (NULL = the default
 * stream).  Calls are asynchronous: HOUGH_OK means "validated and enqueued".  A context owns its
 * constant tables and a small device workspace on the device that was current when it was
 * configured; calls must be made with that device current (HOUGH_EINVAL otherwise), calls
 * that share a context must be ordered on one stream (they share the workspace) and one host
 * thread at a time may use a context.
 * No call allocates device memory after hough_config, and none synchronises the device, so
 * the calls may be captured into a HIP graph.
 *
 * Errors: host-detectable problems return a negative status synchronously and enqueue nothing.
 * Conditions only the device sees (a truncated peak list, an event too large for the fused
 * kernel) are reported through the n_peaks / status outputs.
 */
#ifndef HOUGH_H
#define HOUGH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOUGH_OK          0
#define HOUGH_EINVAL    (-1)   /* bad argument: null pointer, bad grid or parameter          */
#define HOUGH_ENOMEM    (-2)   /* device or host allocation failed in hough_config            */
#define HOUGH_EOVERFLOW (-3)   /* a count could exceed the output type (u16 accumulator)      */
#define HOUGH_EDEVICE   (-4)   /* a HIP runtime call or kernel launch failed                  */
#define HOUGH_ETOOLARGE (-5)   /* the batch needs more than the library's static scratch      */

#define HOUGH_ACC_U16 1        /* accumulator cells are uint16_t (needs n_hits <= 65535)     */
#define HOUGH_ACC_I32 2        /* accumulator cells are int32_t                               */

/* Per-event status bits written by hough_run_batch. */
#define HOUGH_EV_PEAKS_TRUNCATED 1u  /* more peaks than max_peaks; n_peaks holds the true count */
#define HOUGH_EV_INVALID_HITS    2u  /* the event contains invalid hits (they were ignored)     */
#define HOUGH_EV_TOO_MANY_HITS   4u  /* the event's offsets decrease (n_peaks written as zero,
                                        nothing else touched), or (hough_run_batch_iterative
                                        only) it has more than HOUGH_MAX_ITERATIVE_BATCH_HITS
                                        hits: skipped, n_peaks and keep written as zero        */
/* Largest event hough_run_batch_iterative processes (its accumulators hold 16-bit counts). */
#define HOUGH_MAX_ITERATIVE_BATCH_HITS 32767u
/* 8u: unused */
#define HOUGH_EV_DEDUP_SKIPPED   16u /* HOUGH_FLAG_DEDUP: the event has more hits than
                                        hough_max_dedup_hits(), so every hit voted            */

/* The (theta, rho) grid and the peak / retention parameters (Sec. II). */
typedef struct hough_params {
    int32_t n_theta;     /* theta bins on [0, pi), 1 .. 65535                                */
    int32_t n_rho;       /* rho bins on [rho_min, rho_max), 1 .. hough_max_n_rho() (8192)    */
    double  rho_min;     /* lower rho edge (inverse length units of the hit coordinates)     */
    double  rho_max;     /* upper rho edge, > rho_min                                         */
    int32_t acc_type;    /* HOUGH_ACC_U16 or HOUGH_ACC_I32: element type of hough_vote's acc */
    int32_t threshold;   /* minimum peak count, >= 1                                          */
    int32_t rho_window;  /* retention half-width in rho bins, >= 0                            */
    int32_t max_peaks;   /* per-event capacity of hough_run_batch's peak list, >= 0           */
    int32_t flags;       /* HOUGH_FLAG_* bits, 0 for the plain grid                          */
    int32_t reserved;    /* must be 0                                                         */
} hough_params;

/* hough_params.flags: treat theta as periodic in the 3x3 peak test (hough_peaks and the fused
 * batch kernel): with a symmetric rho range (rho_min == -rho_max) the line (theta + pi, rho) is
 * (theta, -rho), so column n_theta - 1 borders column 0 with rho reversed (a step across the
 * border from row k + dk lands on row n_rho - 1 - (k + dk)); raster order still decides ties.
 * Needs n_theta >= 2.  The iterative finder's suppression window does not wrap. */
#define HOUGH_FLAG_THETA_PERIODIC 1

/* hough_params.flags: duplicate suppression on the batch path (hough_run_batch,
 * hough_run_batch_gather, hough_run_batch_split).  A track that curls through the chamber
 * several times fires the same wires on every turn, so an event can hold the same wire
 * position more than once.  With this flag a hit whose (x, y) is bit-identical to an earlier
 * hit of its event casts no votes; every copy is still retained, or not, by its coordinates
 * (so all copies get the same keep byte).  Events with more than hough_max_dedup_hits() hits
 * vote every hit and get HOUGH_EV_DEDUP_SKIPPED.  A batch call then makes one more kernel
 * launch before the fused one, and it writes the events' keep bytes in both.  hough_vote
 * rejects a context with this flag (HOUGH_EINVAL): the per-event path has no such pass. */
#define HOUGH_FLAG_DEDUP 2

/* One peak: grid cell and its count.  8 bytes, no padding. */
typedef struct hough_peak {
    uint16_t theta_bin;
    uint16_t rho_bin;
    uint32_t count;
} hough_peak;

typedef struct hough_ctx hough_ctx;   /* opaque; owned by the library */

/* Validate `p`, build the per-column constants C_j, S_j on the host (double libm cos/sin, each
 * rounded once to float) and upload them, and allocate the workspace on the current device.
 * On success *out receives a new context.  Returns HOUGH_EINVAL for a bad grid or parameter
 * (including n_rho above hough_max_n_rho()), HOUGH_ENOMEM / HOUGH_EDEVICE on allocation or
 * copy failure.  The workspace includes the spill path's per-event slices (peak counts, peak
 * masks and places, dilated bits: about 2.4 bytes per grid cell; see hough_run_batch): a few
 * events' worth, or for a grid taller than the fused kernel's tile one event's worth per CU up
 * to 2 GiB (fewer where the device has not that much free). */
int hough_config(const hough_params *p, hough_ctx **out);

/* Release a context (waits for nothing: the caller must have finished its work on it). */
void hough_destroy(hough_ctx *ctx);

/* Copy the parameters a context was configured with. */
int hough_get_params(const hough_ctx *ctx, hough_params *out);

/* Steps 1-3 for one event (Eq. (1), Sec. II, Sec. III).
 * x, y: n_hits floats each (hit coordinates, SoA).  acc: n_theta * n_rho cells of the
 * configured acc_type, row-major acc[j * n_rho + k]; every cell is written (no pre-zeroing).
 * n_hits == 0 is valid (acc becomes all zero; x and y may then be NULL).
 * HOUGH_EOVERFLOW if acc_type is HOUGH_ACC_U16 and n_hits > 65535. */
int hough_vote(hough_ctx *ctx, const float *x, const float *y, uint32_t n_hits,
               void *acc, void *stream);

/* Step 4 for one event (Sec. II): peaks of `acc` (as written by hough_vote, same acc_type).
 * The first min(count, cap) peaks in raster order go to peaks[0 .. cap-1]; *n_peaks (device)
 * receives the true count, which may exceed cap.  cap == 0 is valid (count only). */
int hough_peaks(hough_ctx *ctx, const void *acc, hough_peak *peaks, uint32_t cap,
                uint32_t *n_peaks, void *stream);

/* Step 4 for one event with the peak finder the paper describes for multi-track events
 * (Sec. II): a threshold relative to the accumulator's global maximum,
 *     thr = max(threshold of the context, ceil(max * frac_num / frac_den)),
 * then iterative extraction: the largest remaining cell at or above thr (the first in raster
 * order among equal counts) becomes a peak and every cell within r_theta theta bins and r_rho
 * rho bins of it (clipped at the grid edges, theta does not wrap) is suppressed; repeat until
 * no cell reaches thr.  Every cell at or above thr takes part, however many there are (the
 * kernel walks them in chunks of its LDS key buffer).  acc as written by hough_vote.  The first
 * min(count, cap) peaks, in extraction order, go to peaks; *n_peaks (device) receives the
 * count; *status (device) receives 0, or HOUGH_EV_PEAKS_TRUNCATED when the count exceeds cap.
 * HOUGH_EINVAL for frac_den == 0 or a negative radius. */
int hough_peaks_iterative(hough_ctx *ctx, const void *acc, uint32_t frac_num, uint32_t frac_den,
                          int32_t r_theta, int32_t r_rho, hough_peak *peaks, uint32_t cap,
                          uint32_t *n_peaks, uint32_t *status, void *stream);

/* A peak read as a candidate track (Sec. II, Eq. (2) with the factor two of Eq. (1)): the
 * circle through the origin whose conformal line is u cos(theta) + v sin(theta) = rho, with
 * theta = theta_bin * pi / n_theta and rho the centre of rho_bin.  48 bytes. */
typedef struct hough_track {
    double a, b;         /* circle centre, (cos theta, sin theta) / (2 rho), hit units       */
    double radius;       /* 1 / (2 |rho|)                                                    */
    double pt;           /* 0.299792458 * b_tesla * radius * 1e-3 (GeV/c for mm and tesla)   */
    double phi_c;        /* atan2(b, a); the direction at the origin is phi_c + charge*pi/2   */
    int32_t charge;      /* +1 when more of the peak's hits lie counter-clockwise of the line
                            from the origin through the centre than clockwise, -1 for the
                            opposite, 0 on a tie (side test sign(rho) (C_j y - S_j x) in float) */
    uint32_t n_hits;     /* hits the retention rule associates with this peak alone          */
} hough_track;

/* Candidate circles and track parameters of the peaks peaks[0 .. min(*n_peaks, cap)-1] of one
 * event (peaks and n_peaks as written by hough_peaks / hough_peaks_iterative; device
 * pointers): tracks[p] for each of them.  x, y: the event's n_hits hits.  A peak outside the
 * grid gets charge 0 and n_hits 0. */
int hough_track_params(hough_ctx *ctx, const float *x, const float *y, uint32_t n_hits,
                       const hough_peak *peaks, const uint32_t *n_peaks, uint32_t cap,
                       double b_tesla, hough_track *tracks, void *stream);

/* Step 5 for one event (Sec. I, Sec. II): keep[i] = 1 iff hit i is within rho_window rho bins
 * of one of the peaks peaks[0 .. min(*n_peaks, cap)-1] (n_peaks is a device pointer, as
 * written by hough_peaks), else 0.  Peak cells outside the grid are ignored. */
int hough_retain(hough_ctx *ctx, const float *x, const float *y, uint32_t n_hits,
                 const hough_peak *peaks, const uint32_t *n_peaks, uint32_t cap,
                 uint8_t *keep, void *stream);

/* Steps 1-5 for a batch of events packed CSR (Sec. III: events are independent and are
 * processed in batches), in one persistent fused kernel that never writes an accumulator.
 * x, y: offsets[n_events] floats; hits of event e are [offsets[e], offsets[e+1]).
 * offsets: n_events + 1 uint32 (device), non-decreasing, offsets[0] may be non-zero.
 * peaks: n_events * max_peaks entries; event e's peaks go to peaks[e * max_peaks ...] in raster
 * order, truncated at max_peaks.  n_peaks[e]: the true peak count.  keep: offsets[n_events]
 * bytes (indexed like x), computed from ALL peaks of the event even when the list is
 * truncated.  status[e]: HOUGH_EV_* bits.  n_events == 0 is valid.  A batch of more events
 * than the kernel has resident workgroups (and at most 65,536 events) is preceded by a small
 * launch that schedules the events largest first; no result depends on the schedule.
 * The fused kernel keeps an event's theta tile on chip, with 16-bit counts.  What it cannot
 * hold -- events above 32,767 hits, events whose hits reach beyond a windowed tile, and every
 * event of a theta-periodic grid whose rho column is taller than its tile (hough_get_batch_plan
 * then reports an all-zero shape) -- is computed by a spill launch after it, one event per
 * workgroup, its accumulator swept through on-chip rho slabs (Sec. II, Sec. III), with the
 * same results; when the fused kernel leaves it nothing, that launch returns at once. */
int hough_run_batch(hough_ctx *ctx, const float *x, const float *y, const uint32_t *offsets,
                    uint32_t n_events, hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep,
                    uint32_t *status, void *stream);

/* hough_run_batch with a per-event threshold relative to the event's largest count, the form
 * of threshold the paper gives its peak finder (Sec. II):
 *     thr_e = max(threshold of the context, ceil(max_e * frac_num / frac_den)),
 * with max_e the largest cell of event e's accumulator (integer arithmetic), then the same 3x3
 * test, listing and retention.  The fused kernel votes every tile twice (once for max_e), so a
 * call costs up to about 1.5 launches of hough_run_batch.  frac_den == 0: HOUGH_EINVAL. */
int hough_run_batch_relative(hough_ctx *ctx, const float *x, const float *y, const uint32_t *offsets,
                             uint32_t n_events, uint32_t frac_num, uint32_t frac_den, hough_peak *peaks,
                             uint32_t *n_peaks, uint8_t *keep, uint32_t *status, void *stream);

/* hough_run_batch over a chosen subset of a resident event pool (Sec. III batches, as formed by
 * a server from arriving events).  x, y, offsets describe the pool exactly as for
 * hough_run_batch; batch event e is pool event event_ids[e] (device array of n_events pool
 * indices, repeats allowed).  Outputs are indexed by batch position: peaks[e * max_peaks ...],
 * n_peaks[e], status[e], and event e's keep bytes are keep[keep_offsets[e] ...] (device array,
 * one entry per batch event; the caller lays the events' keep ranges out without overlap).
 * Same semantics, errors and asynchrony as hough_run_batch. */
int hough_run_batch_gather(hough_ctx *ctx, const float *x, const float *y, const uint32_t *offsets,
                           const uint32_t *event_ids, const uint32_t *keep_offsets,
                           uint32_t n_events, hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep,
                           uint32_t *status, void *stream);

/* The latency form of hough_run_batch / hough_run_batch_gather: the same outputs (bit for bit),
 * but each (event, theta tile) pair is a work item of its own, so the tiles of one event run on
 * different workgroups at once and a small batch finishes sooner (each tile examines the hits
 * the others have not kept yet, so a large batch finishes later than with hough_run_batch).
 * event_ids and keep_offsets are both NULL (events are offsets' own, keep indexed like x) or
 * both given (gather form).  workspace: device buffer of at least
 * hough_split_workspace_bytes(ctx, n_events) bytes, 256-byte aligned, filled with zeros before
 * its first use (NULL when that size is 0); every call leaves it zero again.  Calls sharing a
 * workspace must be ordered. */
int hough_run_batch_split(hough_ctx *ctx, const float *x, const float *y, const uint32_t *offsets,
                          const uint32_t *event_ids, const uint32_t *keep_offsets, uint32_t n_events,
                          hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep, uint32_t *status,
                          void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): hough_run_batch_split with the library's own scratch
 * in place of a caller workspace.  Same arguments (minus the workspace), outputs, asynchrony and
 * errors; the call itself allocates nothing.  The scratch is one device array of
 * HOUGH_STATIC_SCRATCH_BYTES per device, set up by hough_config on that device and held until
 * the process ends; a batch whose hough_split_workspace_bytes exceeds it is refused with
 * HOUGH_ETOOLARGE before anything is enqueued.  Every call on a device shares that device's
 * array (each call leaves it zero), so calls that may overlap on one device -- on different
 * streams, or from different host threads -- race and must be ordered by the caller. */
#define HOUGH_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
int hough_run_batch_split_static(hough_ctx *ctx, const float *x, const float *y, const uint32_t *offsets,
                                 const uint32_t *event_ids, const uint32_t *keep_offsets, uint32_t n_events,
                                 hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep, uint32_t *status,
                                 void *stream);

/* The paper's peak finder over a batch of CSR events (as hough_run_batch takes them): steps
 * 1-3 into one 16-bit accumulator per event in `workspace` (device, 256-byte aligned, at least
 * hough_iterative_workspace_bytes(ctx, n_events) bytes, contents not preserved), then
 * hough_peaks_iterative's finder per event (same frac, r_theta, r_rho and threshold floor),
 * then retention (as hough_retain) with each event's first min(n_peaks, max_peaks) peaks.
 * peaks (device): max_peaks records per event, in extraction order; n_peaks[e] the true count;
 * keep[offsets[0] .. offsets[n_events]] one byte per hit; status[e] the HOUGH_EV_* bits.
 * Events above HOUGH_MAX_ITERATIVE_BATCH_HITS hits are skipped (HOUGH_EV_TOO_MANY_HITS);
 * HOUGH_FLAG_DEDUP applies.
 * Four kernel launches per call.  Accumulators go through HBM (n_theta * n_rho * 2 bytes per
 * event), so this is the per-event path's work done for the whole batch at once, not the fused
 * kernel. */
int hough_run_batch_iterative(hough_ctx *ctx, const float *x, const float *y, const uint32_t *offsets,
                              uint32_t n_events, uint32_t frac_num, uint32_t frac_den, int32_t r_theta,
                              int32_t r_rho, hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep,
                              uint32_t *status, void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes hough_run_batch_iterative needs for n_events events: the 16-bit accumulators
 * and, on grids whose suppression bitmap does not fit on chip beside the finder's key buffer,
 * one bitmap (one bit per cell) per event (0 for a NULL context). */
size_t hough_iterative_workspace_bytes(const hough_ctx *ctx, uint32_t n_events);

/* Largest event (hits) whose duplicates HOUGH_FLAG_DEDUP suppresses. */
uint32_t hough_max_dedup_hits(void);

/* Workspace bytes hough_run_batch_split needs for n_events events with the context's current
 * launch shape (0 for a NULL context, and for a grid without a fused kernel, whose batches need
 * no workspace). */
size_t hough_split_workspace_bytes(const hough_ctx *ctx, uint32_t n_events);

/* Launch shape of hough_run_batch's fused kernel.  A theta tile is 64 * column_groups columns
 * (two of them halo columns shared with the neighbouring tiles); the hits of an event are split
 * over waves_per_group waves of a workgroup; groups_per_cu workgroups run on each compute unit.
 * The schedule changes speed only, never results. */
typedef struct hough_batch_plan {
    int32_t waves_per_group;   /* 4, 6, 8, 12 or 16                                    */
    int32_t column_groups;     /* 1 or 2                                               */
    int32_t groups_per_cu;     /* workgroups launched per CU (<= what fits)            */
    int32_t lds_bytes;         /* LDS per workgroup (read-only)                        */
    int32_t window_rows;       /* rho rows of a windowed tile, 0 = whole column (read-only) */
} hough_batch_plan;

/* The launch shape hough_run_batch currently uses (the library picks one at hough_config).  A
 * grid whose whole rho column does not fit the fused kernel's tile gets a windowed tile (theta
 * not periodic; window_rows > 0): each event whose hits reach only that many rows runs in the
 * fused kernel, the others, and every event of the split forms, through the spill path.  All
 * zero when there is no fused kernel for the grid (a periodic grid taller than the tile: every
 * event spills). */
int hough_get_batch_plan(const hough_ctx *ctx, hough_batch_plan *out);

/* Select a launch shape (for autotuning).  groups_per_cu = 0 launches as many workgroups per CU
 * as fit; a positive value launches at most that many.  A groups_per_cu above what a tile of the
 * whole rho column allows selects a windowed tile (one column group, theta not periodic): the
 * tallest whole number of 32-row words that lets that many workgroups share a CU.  Each event
 * then gets the window of rows its hits can reach (they are bounded by the event's smallest
 * x^2 + y^2, Eq. (1)); an event whose rows do not fit goes through the spill path, as do
 * events above the fused kernel's hit limit.  The split forms always hold the whole column.
 * HOUGH_EINVAL if the combination is not supported or does not fit the device, or the grid has
 * no fused kernel; the context keeps its previous shape then. */
int hough_set_batch_plan(hough_ctx *ctx, int32_t waves_per_group, int32_t column_groups,
                         int32_t groups_per_cu);

/* Largest number of hits per event hough_run_batch processes for this context: every event
 * (UINT32_MAX; larger events go through the spill path), 0 for a NULL context. */
uint32_t hough_max_batch_hits(const hough_ctx *ctx);

/* Largest n_rho hough_config accepts on the current device (8192 on MI355X). */
int32_t hough_max_n_rho(void);

/* Static description of a status code. */
const char *hough_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* HOUGH_H */
