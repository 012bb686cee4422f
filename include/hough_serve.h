/*
 * hough_serve.h -- C ABI of the serving loop in libhough.so: an online (trigger-like) request
 * loop around the batch entry points of hough.h.
 *
 * Sec. III processes events in batches and states that host-to-device transfer, kernel
 * execution and device-to-host transfer can overlap; Sec. V names streams and asynchronous
 * transfers as the way to feed continuous event streams.  hough_serve_run is that loop: events
 * arrive at scheduled times (open loop), wait in a per-grid queue, are admitted into a batch as
 * long as the batch's device arena has room for their hits (memory-based admission), and a batch
 * is launched on a free stream as soon as one exists (continuous batching: events that arrive
 * while other batches are on the GPU form the next batch, and up to n_streams batches overlap
 * on the device).  A request is complete when its results are in host memory.
 *
 * A pool's events reach the device in one of two ways.  Resident pools (x, y given) keep every
 * event's hits in device memory (e.g. a readout buffer filled by DMA): admitting an event sends
 * its 4-byte pool index and keep offset to the device.  Host pools (host_x, host_y given) keep the
 * hits in host memory: admitting a batch packs its events' hits and CSR offsets into the stream
 * slot's pinned staging buffer and sends them in one asynchronous host-to-device copy into the
 * slot's device arena (max_batch_hits hits), on the slot's stream, ahead of the kernels, so a
 * request's latency includes its transfer.  Completion brings back n_peaks, status, keep and,
 * on request, the peak list.  Results are identical to processing each event alone (every
 * output is an integer and events are independent).
 *
 * Batches on different streams run concurrently; each stream slot therefore launches through
 * private copies of the pools' contexts (same parameters and launch shape), made on entry.
 * Inside a batch the events are ordered largest first (the smallest fill the kernel's tail);
 * a batch's inputs (resident: ids and keep offsets; host: offsets and hits) go to the device in
 * one copy and its n_peaks, status and keep bytes come back in one.  Small batches can take the split form (each stream slot then
 * holds a zero-filled workspace for split_batch_events events), which trades total work for a
 * shorter time per batch.
 *
 * With `plain` set, each request is instead processed alone by hough_vote, hough_peaks and
 * hough_retain (three launches, accumulator through HBM), one request per stream slot, under
 * the same arrivals: the per-event launch it is compared against.
 */
#ifndef HOUGH_SERVE_H
#define HOUGH_SERVE_H

#include <stdint.h>

#include "hough.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One event pool and the grid its events are processed on.  Either x, y and offsets (resident
 * pool, device memory) or host_x and host_y (host pool, sent per batch) are given. */
typedef struct hough_serve_pool {
    hough_ctx *ctx;                 /* grid, thresholds, max_peaks                          */
    const float *x;                 /* device, pool hits (as for hough_run_batch), or NULL  */
    const float *y;                 /* device, or NULL                                      */
    const uint32_t *offsets;        /* device, [n_events + 1], or NULL                      */
    const uint32_t *host_offsets;   /* host, [n_events + 1] (hit counts for admission)      */
    uint32_t n_events;
    uint32_t reserved;              /* 0                                                     */
    const float *host_x;            /* host, pool hits indexed like host_offsets, or NULL   */
    const float *host_y;            /* host, or NULL                                        */
} hough_serve_pool;

typedef struct hough_serve_config {
    int32_t n_streams;              /* batches (plain: events) in flight, 1 .. 32            */
    int32_t max_batch_events;       /* events per batch, >= 1                                */
    int32_t max_batch_hits;         /* device arena per stream slot, in hits, >= 1           */
    int32_t plain;                  /* 0: batches (resident pools: hough_run_batch_gather;
                                       host pools: hough_run_batch on the slot's arena);
                                       1: per event                                           */
    int32_t copy_peaks;             /* 1: bring the peak lists back as part of completion    */
    int32_t small_batch_events;     /* batches of at most this many events run with 16-wave
                                       workgroups (one event per CU finishes sooner); 0: never */
    int32_t split_batch_events;     /* batches of at most this many events run through
                                       hough_run_batch_split on the 16-wave shape (an event's
                                       theta tiles on separate workgroups); 0: never          */
    int32_t reserved;               /* 0                                                     */
    double max_wait_us;             /* hold a partial batch until its oldest event waited this
                                       long while a slot is free (0: launch at once)          */
} hough_serve_config;

typedef struct hough_serve_request {
    double arrival_us;              /* scheduled arrival, microseconds from the run's start  */
    int32_t kind;                   /* pool index                                            */
    uint32_t event;                 /* event index in that pool                              */
} hough_serve_request;

typedef struct hough_serve_result {
    double launch_us;               /* its batch (or its first kernel) was enqueued          */
    double done_us;                 /* its results were observed in host memory              */
    uint32_t n_peaks;               /* true peak count                                       */
    uint32_t status;                /* HOUGH_EV_* bits                                       */
    uint32_t batch_events;          /* events in the batch that carried it (plain: 1)        */
    uint32_t slot;                  /* stream slot that ran it                               */
} hough_serve_result;

/* Run the request trace `reqs` (non-decreasing arrival_us) to completion on the current device.
 * res[i] receives request i's timing and counts.  keep_out (host, optional): request i's keep
 * bytes are written at keep_out[sum of the hit counts of requests 0 .. i-1].  peaks_out (host,
 * optional, needs copy_peaks): request i's first min(n_peaks, max_peaks of its pool) peaks are
 * written at peaks_out[i * peaks_stride].  The call blocks until every request completed; it
 * allocates its stream slots' buffers on entry and frees them on return.
 * Returns HOUGH_EINVAL for a bad argument or a request whose event does not fit a slot's arena,
 * HOUGH_ENOMEM, or HOUGH_EDEVICE. */
int hough_serve_run(const hough_serve_pool *pools, int32_t n_kinds, const hough_serve_config *cfg,
                    const hough_serve_request *reqs, uint32_t n_reqs, hough_serve_result *res,
                    uint8_t *keep_out, hough_peak *peaks_out, uint32_t peaks_stride);

/* Cost of one batch of a kind in hough_serve_simulate: a batch of n events and h hits occupies
 * its stream slot for fixed_us + per_event_us * n + per_hit_us * h microseconds. */
typedef struct hough_serve_model {
    double fixed_us;
    double per_event_us;
    double per_hit_us;
} hough_serve_model;

/* The scheduling of hough_serve_run (admission, queues, batching, slot choice) replayed on a
 * simulated clock against a cost model instead of the GPU, for capacity planning and for testing
 * the scheduler on a host without a device.  hits[i] is request i's event size (events are not
 * read); models[kind] gives each kind's batch cost; slots run their batches concurrently and
 * independently.  res[i] receives launch_us, done_us, batch_events and slot (n_peaks and status
 * are 0).  The plain, small_batch_events and split_batch_events settings only change the model's
 * inputs as they change batch formation (plain: one event per slot).  Same argument checks as
 * hough_serve_run; touches no device. */
int hough_serve_simulate(int32_t n_kinds, const hough_serve_config *cfg, const hough_serve_request *reqs,
                         const uint32_t *hits, uint32_t n_reqs, const hough_serve_model *models,
                         hough_serve_result *res);

#ifdef __cplusplus
}
#endif

#endif /* HOUGH_SERVE_H */
