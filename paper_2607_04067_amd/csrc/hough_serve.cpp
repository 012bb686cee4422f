// Serving loop of libhough.so (include/hough_serve.h): open-loop arrivals, per-grid queues,
// memory-based admission into stream-slot arenas, continuous batching over HIP streams.
// The loop runs on the calling host thread and does O(1) work per event plus the copies of
// its results; all per-event compute runs in the library's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/hough_serve.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Kind {
    hough_serve_pool pool;
    hough_params p;
    size_t acc_bytes;
};

// One stream and the device/pinned buffers of one batch (or one plain event) in flight.
// A batch of n events moves in one copy each way: in = [ids (n) | keep offsets (n)] and
// out = [n_peaks (n) | status (n) | keep bytes], packed for the batch's own n.
struct Slot {
    hipStream_t stream = nullptr;
    std::vector<hough_ctx *> ctx;      // one private context per kind: its own work counter
    std::vector<hough_ctx *> ctx_small;  // the same grid with 16-wave workgroups, for small batches
    hipEvent_t done = nullptr;
    uint32_t *d_in = nullptr;
    uint8_t *d_out = nullptr;
    hough_peak *d_peaks = nullptr;
    void *d_acc = nullptr;
    void *d_ws = nullptr;              // split-form workspace (zero between launches)
    size_t ws_bytes = 0;
    uint32_t *h_in = nullptr;
    uint8_t *h_out = nullptr;
    hough_peak *h_peaks = nullptr;
    uint32_t n = 0;                    // events of the batch in flight
    bool busy = false;
    int kind = 0;
    double t_launch = 0.0;
    std::vector<uint32_t> reqs;
};

struct Server {
    std::vector<Kind> kinds;
    std::vector<Slot> slots;
    hough_serve_config cfg{};
    size_t cap_max = 0, acc_max = 0;

    ~Server() {
        for (Slot &s : slots) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            (void)hipFree(s.d_in); (void)hipFree(s.d_out); (void)hipFree(s.d_peaks); (void)hipFree(s.d_acc);
            (void)hipFree(s.d_ws);
            (void)hipHostFree(s.h_in); (void)hipHostFree(s.h_out); (void)hipHostFree(s.h_peaks);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            for (hough_ctx *c : s.ctx) hough_destroy(c);
            for (hough_ctx *c : s.ctx_small) hough_destroy(c);
        }
    }

    int setup() {
        const size_t E = cfg.plain ? 1u : (size_t)cfg.max_batch_events;
        const size_t H = (size_t)cfg.max_batch_hits;
        slots.resize((size_t)cfg.n_streams);
        for (Slot &s : slots) {
            bool ok = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
                      hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess;
            ok = ok && hipMalloc(&s.d_in, E * 8) == hipSuccess && hipMalloc(&s.d_out, E * 8 + H) == hipSuccess &&
                 hipMalloc(&s.d_peaks, E * (cap_max ? cap_max : 1) * sizeof(hough_peak)) == hipSuccess;
            if (ok && cfg.plain) ok = hipMalloc(&s.d_acc, acc_max) == hipSuccess;
            ok = ok && hipHostMalloc(&s.h_in, E * 8) == hipSuccess && hipHostMalloc(&s.h_out, E * 8 + H) == hipSuccess &&
                 hipHostMalloc(&s.h_peaks, (cfg.copy_peaks ? E * (cap_max ? cap_max : 1) : 1) * sizeof(hough_peak)) == hipSuccess;
            if (!ok) return HOUGH_ENOMEM;
            s.reqs.reserve(E);
            // batches on different streams run at the same time, so each slot launches through
            // its own copy of every kind's context (same grid, parameters and launch shape)
            for (const Kind &k : kinds) {
                hough_ctx *c = nullptr;
                const int rc = hough_config(&k.p, &c);
                if (rc != HOUGH_OK) return rc;
                s.ctx.push_back(c);
                hough_batch_plan bp;
                if (hough_get_batch_plan(k.pool.ctx, &bp) != HOUGH_OK ||
                    hough_set_batch_plan(c, bp.waves_per_group, bp.column_groups, bp.groups_per_cu) != HOUGH_OK)
                    return HOUGH_EINVAL;
                // a batch of fewer events than workgroup slots runs each event on one workgroup:
                // 16 waves finish it sooner than 8 (when that shape fits; else the pool's shape)
                hough_ctx *cs = nullptr;
                const int rs = hough_config(&k.p, &cs);
                if (rs != HOUGH_OK) return rs;
                s.ctx_small.push_back(cs);
                if (hough_set_batch_plan(cs, 16, 1, 0) != HOUGH_OK &&
                    hough_set_batch_plan(cs, bp.waves_per_group, bp.column_groups, bp.groups_per_cu) != HOUGH_OK)
                    return HOUGH_EINVAL;
                // every split launch leaves the workspace zero, so the kinds can share it
                if (!cfg.plain && cfg.split_batch_events > 0)
                    s.ws_bytes = std::max(s.ws_bytes,
                                          hough_split_workspace_bytes(cs, (uint32_t)cfg.split_batch_events));
            }
            if (s.ws_bytes && (hipMalloc(&s.d_ws, s.ws_bytes) != hipSuccess ||
                               hipMemset(s.d_ws, 0, s.ws_bytes) != hipSuccess))
                return HOUGH_ENOMEM;
        }
        return HOUGH_OK;
    }
};

inline uint32_t hits_of(const Kind &k, uint32_t ev) {
    return k.pool.host_offsets[ev + 1] - k.pool.host_offsets[ev];
}

}  // namespace

extern "C" int hough_serve_run(const hough_serve_pool *pools, int32_t n_kinds, const hough_serve_config *cfg,
                               const hough_serve_request *reqs, uint32_t n_reqs, hough_serve_result *res,
                               uint8_t *keep_out, hough_peak *peaks_out, uint32_t peaks_stride) {
    if (!pools || n_kinds < 1 || !cfg || (n_reqs && (!reqs || !res))) return HOUGH_EINVAL;
    if (cfg->n_streams < 1 || cfg->n_streams > 32 || cfg->max_batch_events < 1 || cfg->max_batch_hits < 1 ||
        cfg->small_batch_events < 0 || cfg->split_batch_events < 0 || cfg->reserved != 0 ||
        !(cfg->max_wait_us >= 0.0))
        return HOUGH_EINVAL;
    if (peaks_out && !cfg->copy_peaks) return HOUGH_EINVAL;

    Server *srv = new (std::nothrow) Server();
    if (!srv) return HOUGH_ENOMEM;
    srv->cfg = *cfg;
    for (int k = 0; k < n_kinds; ++k) {
        const hough_serve_pool &pl = pools[k];
        Kind kd;
        kd.pool = pl;
        if (!pl.ctx || !pl.x || !pl.y || !pl.offsets || !pl.host_offsets || pl.n_events < 1 ||
            hough_get_params(pl.ctx, &kd.p) != HOUGH_OK) {
            delete srv;
            return HOUGH_EINVAL;
        }
        kd.acc_bytes = (size_t)kd.p.n_theta * kd.p.n_rho * (kd.p.acc_type == HOUGH_ACC_U16 ? 2 : 4);
        if ((size_t)kd.p.max_peaks > srv->cap_max) srv->cap_max = (size_t)kd.p.max_peaks;
        if (kd.acc_bytes > srv->acc_max) srv->acc_max = kd.acc_bytes;
        srv->kinds.push_back(kd);
    }
    // every request must name a pool event that fits one slot's arena; arrivals are ordered
    std::vector<uint64_t> keep_off(n_reqs ? n_reqs : 1);
    uint64_t acc_hits = 0;
    for (uint32_t i = 0; i < n_reqs; ++i) {
        const hough_serve_request &r = reqs[i];
        if (r.kind < 0 || r.kind >= n_kinds || r.event >= srv->kinds[r.kind].pool.n_events ||
            hits_of(srv->kinds[r.kind], r.event) > (uint32_t)cfg->max_batch_hits ||
            (i && r.arrival_us < reqs[i - 1].arrival_us) || !(r.arrival_us >= 0.0)) {
            delete srv;
            return HOUGH_EINVAL;
        }
        keep_off[i] = acc_hits;
        acc_hits += hits_of(srv->kinds[r.kind], r.event);
    }
    int rc = srv->setup();
    if (rc != HOUGH_OK) {
        delete srv;
        return rc;
    }

    // per-kind FIFO of arrived, not yet admitted requests (requests arrive in order)
    std::vector<std::vector<uint32_t>> pend((size_t)n_kinds);
    std::vector<size_t> head((size_t)n_kinds, 0);
    for (auto &q : pend) q.reserve(n_reqs);

    const Clock::time_point t0 = Clock::now();
    auto now_us = [&]() { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); };

    auto finish = [&](Slot &sl, double t) {
        const Kind &kd = srv->kinds[(size_t)sl.kind];
        const uint32_t n = (uint32_t)sl.reqs.size();
        const uint32_t *h_npk = reinterpret_cast<const uint32_t *>(sl.h_out);
        const uint32_t *h_status = h_npk + n;
        const uint8_t *h_keep = sl.h_out + 8u * n;
        const uint32_t *h_koff = sl.h_in + n;
        for (uint32_t j = 0; j < n; ++j) {
            const uint32_t r = sl.reqs[j];
            hough_serve_result &o = res[r];
            o.launch_us = sl.t_launch;
            o.done_us = t;
            o.n_peaks = h_npk[j];
            o.status = cfg->plain ? (o.n_peaks > (uint32_t)kd.p.max_peaks ? HOUGH_EV_PEAKS_TRUNCATED : 0u)
                                  : h_status[j];
            o.batch_events = n;
            o.pad = 0;
            const uint32_t H = hits_of(kd, reqs[r].event);
            if (keep_out) std::memcpy(keep_out + keep_off[r], h_keep + h_koff[j], H);
            if (peaks_out) {
                uint32_t m = o.n_peaks < (uint32_t)kd.p.max_peaks ? o.n_peaks : (uint32_t)kd.p.max_peaks;
                if (m > peaks_stride) m = peaks_stride;
                std::memcpy(peaks_out + (size_t)r * peaks_stride, sl.h_peaks + (size_t)j * kd.p.max_peaks,
                            (size_t)m * sizeof(hough_peak));
            }
        }
        sl.reqs.clear();
        sl.busy = false;
        return n;
    };

    auto launch = [&](Slot &sl, int k, double t) -> int {
        const Kind &kd = srv->kinds[(size_t)k];
        std::vector<uint32_t> &q = pend[(size_t)k];
        size_t &h = head[(size_t)k];
        const uint32_t E = cfg->plain ? 1u : (uint32_t)cfg->max_batch_events;
        uint32_t n = 0, hits = 0;
        while (h < q.size() && n < E) {                       // memory-based admission
            const uint32_t H = hits_of(kd, reqs[q[h]].event);
            if (hits + H > (uint32_t)cfg->max_batch_hits) break;
            sl.reqs.push_back(q[h]);
            hits += H;
            ++n;
            ++h;
        }
        // the batch's events go largest first, so that the smallest ones fill the tail of the
        // kernel; request order inside the slot follows
        std::sort(sl.reqs.begin(), sl.reqs.end(), [&](uint32_t a, uint32_t b) {
            const uint32_t ha = hits_of(kd, reqs[a].event), hb = hits_of(kd, reqs[b].event);
            return ha != hb ? ha > hb : a < b;
        });
        uint32_t *h_ids = sl.h_in, *h_koff = sl.h_in + n;
        uint32_t koff = 0;
        for (uint32_t j = 0; j < n; ++j) {
            h_ids[j] = reqs[sl.reqs[j]].event;
            h_koff[j] = koff;
            koff += hits_of(kd, h_ids[j]);
        }
        sl.n = n;
        uint32_t *d_ids = sl.d_in, *d_koff = sl.d_in + n;
        uint32_t *d_npk = reinterpret_cast<uint32_t *>(sl.d_out), *d_status = d_npk + n;
        uint8_t *d_keep = sl.d_out + 8u * n;
        sl.kind = k;
        sl.busy = true;
        sl.t_launch = t;
        const hipStream_t s = sl.stream;
        const size_t cap = (size_t)kd.p.max_peaks;
        int st = HOUGH_OK;
        if (!cfg->plain) {
            if (hipMemcpyAsync(sl.d_in, sl.h_in, n * 8u, hipMemcpyHostToDevice, s) != hipSuccess)
                return HOUGH_EDEVICE;
            if (n <= (uint32_t)cfg->split_batch_events) {
                st = hough_run_batch_split(sl.ctx_small[(size_t)k], kd.pool.x, kd.pool.y, kd.pool.offsets, d_ids,
                                           d_koff, n, sl.d_peaks, d_npk, d_keep, d_status, sl.d_ws, sl.ws_bytes, s);
            } else {
                hough_ctx *c = n <= (uint32_t)cfg->small_batch_events ? sl.ctx_small[(size_t)k] : sl.ctx[(size_t)k];
                st = hough_run_batch_gather(c, kd.pool.x, kd.pool.y, kd.pool.offsets, d_ids, d_koff,
                                            n, sl.d_peaks, d_npk, d_keep, d_status, s);
            }
        } else {
            const uint32_t h0 = kd.pool.host_offsets[h_ids[0]];
            st = hough_vote(sl.ctx[(size_t)k], kd.pool.x + h0, kd.pool.y + h0, hits, sl.d_acc, s);
            if (st == HOUGH_OK) st = hough_peaks(sl.ctx[(size_t)k], sl.d_acc, sl.d_peaks, (uint32_t)cap, d_npk, s);
            if (st == HOUGH_OK)
                st = hough_retain(sl.ctx[(size_t)k], kd.pool.x + h0, kd.pool.y + h0, hits, sl.d_peaks, d_npk,
                                  (uint32_t)cap, d_keep, s);
        }
        if (st != HOUGH_OK) return st;
        if (hipMemcpyAsync(sl.h_out, sl.d_out, 8u * n + hits, hipMemcpyDeviceToHost, s) != hipSuccess ||
            (cfg->copy_peaks && cap &&
             hipMemcpyAsync(sl.h_peaks, sl.d_peaks, n * cap * sizeof(hough_peak), hipMemcpyDeviceToHost, s) != hipSuccess) ||
            hipEventRecord(sl.done, s) != hipSuccess)
            return HOUGH_EDEVICE;
        return HOUGH_OK;
    };

    uint32_t next = 0, completed = 0;
    rc = HOUGH_OK;
    while (completed < n_reqs && rc == HOUGH_OK) {
        double t = now_us();
        while (next < n_reqs && reqs[next].arrival_us <= t) {
            pend[(size_t)reqs[next].kind].push_back(next);
            ++next;
        }
        for (Slot &sl : srv->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) completed += finish(sl, now_us());
            else if (q != hipErrorNotReady) { rc = HOUGH_EDEVICE; break; }
        }
        if (rc != HOUGH_OK) break;
        t = now_us();
        for (Slot &sl : srv->slots) {
            if (sl.busy) continue;
            // the kind whose oldest waiting request arrived first
            int k = -1;
            double oldest = 0.0;
            for (int kk = 0; kk < n_kinds; ++kk) {
                if (head[(size_t)kk] >= pend[(size_t)kk].size()) continue;
                const double a = reqs[pend[(size_t)kk][head[(size_t)kk]]].arrival_us;
                if (k < 0 || a < oldest) { k = kk; oldest = a; }
            }
            if (k < 0) break;
            if (!cfg->plain && cfg->max_wait_us > 0.0) {
                const size_t waiting = pend[(size_t)k].size() - head[(size_t)k];
                if (waiting < (size_t)cfg->max_batch_events && t - oldest < cfg->max_wait_us) break;
            }
            rc = launch(sl, k, t);
            if (rc != HOUGH_OK) break;
        }
    }
    delete srv;   // waits for its streams, frees its buffers
    return rc;
}
