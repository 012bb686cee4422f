// Serving loop of libhough.so (include/hough_serve.h): the scheduling core of serve_sched.h run
// over HIP streams (hough_serve_run) or over a cost model on a simulated clock
// (hough_serve_simulate).  The loop runs on the calling host thread and does O(1) work per event
// plus the copies of its hits and results; all per-event compute runs in the library's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "serve_sched.h"

namespace {

using Clock = std::chrono::steady_clock;
using hough_serve::Batch;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Kind {
    hough_serve_pool pool;
    hough_params p;
    size_t acc_bytes;
    bool host;                        // hits in host memory, sent with each batch
};

// One stream and the buffers of one batch (or one plain event) in flight.
//   resident pools: in = [ids (n) | keep offsets (n)] (device copy d_in), launched as a gather;
//   host pools:     arena = [offsets (n + 1) | x (hits) | y (hits)], each section 256-byte
//                   aligned, packed in pinned h_arena and sent in one copy to d_arena.
// out = [n_peaks (n) | status (n) | keep bytes (hits)] comes back in one copy.
struct Slot {
    hipStream_t stream = nullptr;
    std::vector<hough_ctx *> ctx;        // one private context per kind: its own work counter
    std::vector<hough_ctx *> ctx_small;  // the same grid with 16-wave workgroups, for small batches
    hipEvent_t done = nullptr;
    uint32_t *d_in = nullptr;
    uint8_t *d_arena = nullptr;
    uint8_t *d_out = nullptr;
    hough_peak *d_peaks = nullptr;
    void *d_acc = nullptr;
    void *d_ws = nullptr;                // split-form workspace (zero between launches)
    size_t ws_bytes = 0;
    uint32_t *h_in = nullptr;
    uint8_t *h_arena = nullptr;
    uint8_t *h_out = nullptr;
    hough_peak *h_peaks = nullptr;
    std::vector<uint32_t> koff;          // keep offset of each batch event in out's keep bytes
};

struct HipServer {
    std::vector<Kind> kinds;
    std::vector<Slot> slots;
    hough_serve_config cfg{};
    const hough_serve_request *reqs = nullptr;
    std::vector<uint64_t> keep_off;      // request -> offset of its keep bytes in keep_out
    uint8_t *keep_out = nullptr;
    hough_peak *peaks_out = nullptr;
    uint32_t peaks_stride = 0;
    size_t cap_max = 0, acc_max = 0, arena_bytes = 0;
    bool any_host = false, any_resident = false;
    Clock::time_point t0;

    ~HipServer() {
        for (Slot &s : slots) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            (void)hipFree(s.d_in); (void)hipFree(s.d_arena); (void)hipFree(s.d_out); (void)hipFree(s.d_peaks);
            (void)hipFree(s.d_acc); (void)hipFree(s.d_ws);
            (void)hipHostFree(s.h_in); (void)hipHostFree(s.h_arena); (void)hipHostFree(s.h_out);
            (void)hipHostFree(s.h_peaks);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            for (hough_ctx *c : s.ctx) hough_destroy(c);
            for (hough_ctx *c : s.ctx_small) hough_destroy(c);
        }
    }

    uint32_t hits_of(int k, uint32_t ev) const {
        const uint32_t *o = kinds[(size_t)k].pool.host_offsets;
        return o[ev + 1] - o[ev];
    }

    int setup() {
        const size_t E = cfg.plain ? 1u : (size_t)cfg.max_batch_events;
        const size_t H = (size_t)cfg.max_batch_hits;
        arena_bytes = align256(4 * (E + 1)) + 2 * align256(4 * H);
        slots.resize((size_t)cfg.n_streams);
        for (Slot &s : slots) {
            bool ok = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
                      hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess;
            ok = ok && hipMalloc(&s.d_out, E * 8 + H) == hipSuccess &&
                 hipMalloc(&s.d_peaks, E * (cap_max ? cap_max : 1) * sizeof(hough_peak)) == hipSuccess &&
                 hipHostMalloc(&s.h_out, E * 8 + H) == hipSuccess &&
                 hipHostMalloc(&s.h_peaks, (cfg.copy_peaks ? E * (cap_max ? cap_max : 1) : 1) * sizeof(hough_peak)) ==
                     hipSuccess;
            if (ok && any_resident)
                ok = hipMalloc(&s.d_in, E * 8) == hipSuccess && hipHostMalloc(&s.h_in, E * 8) == hipSuccess;
            if (ok && any_host)
                ok = hipMalloc(&s.d_arena, arena_bytes) == hipSuccess &&
                     hipHostMalloc(&s.h_arena, arena_bytes) == hipSuccess;
            if (ok && cfg.plain) ok = hipMalloc(&s.d_acc, acc_max) == hipSuccess;
            if (!ok) return HOUGH_ENOMEM;
            s.koff.reserve(E);
            // batches on different streams run at the same time, so each slot launches through
            // its own copy of every kind's context (same grid, parameters and launch shape)
            for (const Kind &k : kinds) {
                hough_ctx *c = nullptr;
                const int rc = hough_config(&k.p, &c);
                if (rc != HOUGH_OK) return rc;
                s.ctx.push_back(c);
                hough_batch_plan bp;
                if (hough_get_batch_plan(k.pool.ctx, &bp) != HOUGH_OK) return HOUGH_EINVAL;
                const bool fused = bp.waves_per_group > 0;    // else every event spills: no shape to set
                if (fused &&
                    hough_set_batch_plan(c, bp.waves_per_group, bp.column_groups, bp.groups_per_cu) != HOUGH_OK)
                    return HOUGH_EINVAL;
                // a batch of fewer events than workgroup slots runs each event on one workgroup:
                // 16 waves finish it sooner than 8 (when that shape fits; else the pool's shape)
                hough_ctx *cs = nullptr;
                const int rs = hough_config(&k.p, &cs);
                if (rs != HOUGH_OK) return rs;
                s.ctx_small.push_back(cs);
                if (fused && hough_set_batch_plan(cs, 16, 1, 0) != HOUGH_OK &&
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

    // ------------------------------------------------------------ Backend of serve_sched.h
    double now() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }

    void idle(double) const {}           // the loop polls its streams' events

    int poll(int s, bool *done) {
        const hipError_t q = hipEventQuery(slots[(size_t)s].done);
        if (q == hipSuccess) { *done = true; return HOUGH_OK; }
        *done = false;
        return q == hipErrorNotReady ? HOUGH_OK : HOUGH_EDEVICE;
    }

    int launch(int si, const Batch &b) {
        Slot &sl = slots[(size_t)si];
        const Kind &kd = kinds[(size_t)b.kind];
        const uint32_t n = (uint32_t)b.reqs.size();
        const hipStream_t s = sl.stream;
        const size_t cap = (size_t)kd.p.max_peaks;
        uint32_t *d_npk = reinterpret_cast<uint32_t *>(sl.d_out), *d_status = d_npk + n;
        uint8_t *d_keep = sl.d_out + 8u * n;
        sl.koff.resize(n);
        uint32_t koff = 0;
        for (uint32_t j = 0; j < n; ++j) {
            sl.koff[j] = koff;
            koff += hits_of(b.kind, reqs[b.reqs[j]].event);
        }
        const float *x = kd.pool.x, *y = kd.pool.y;
        const uint32_t *off = kd.pool.offsets;
        uint32_t *d_ids = nullptr, *d_koff = nullptr;
        if (kd.host) {
            // pack the batch's CSR offsets and hits into pinned staging, then one copy to the arena
            const size_t xo = align256(4 * ((size_t)n + 1)), yo = xo + align256(4 * (size_t)b.hits);
            uint32_t *h_off = reinterpret_cast<uint32_t *>(sl.h_arena);
            float *hx = reinterpret_cast<float *>(sl.h_arena + xo), *hy = reinterpret_cast<float *>(sl.h_arena + yo);
            for (uint32_t j = 0; j < n; ++j) {
                const uint32_t ev = reqs[b.reqs[j]].event, h0 = kd.pool.host_offsets[ev];
                const uint32_t H = hits_of(b.kind, ev);
                h_off[j] = sl.koff[j];
                std::memcpy(hx + sl.koff[j], kd.pool.host_x + h0, (size_t)H * 4);
                std::memcpy(hy + sl.koff[j], kd.pool.host_y + h0, (size_t)H * 4);
            }
            h_off[n] = b.hits;
            if (hipMemcpyAsync(sl.d_arena, sl.h_arena, yo + 4 * (size_t)b.hits, hipMemcpyHostToDevice, s) != hipSuccess)
                return HOUGH_EDEVICE;
            off = reinterpret_cast<const uint32_t *>(sl.d_arena);
            x = reinterpret_cast<const float *>(sl.d_arena + xo);
            y = reinterpret_cast<const float *>(sl.d_arena + yo);
        } else if (!cfg.plain) {
            uint32_t *h_ids = sl.h_in, *h_koff = sl.h_in + n;
            for (uint32_t j = 0; j < n; ++j) {
                h_ids[j] = reqs[b.reqs[j]].event;
                h_koff[j] = sl.koff[j];
            }
            if (hipMemcpyAsync(sl.d_in, sl.h_in, n * 8u, hipMemcpyHostToDevice, s) != hipSuccess)
                return HOUGH_EDEVICE;
            d_ids = sl.d_in;
            d_koff = sl.d_in + n;
        }
        int st = HOUGH_OK;
        if (!cfg.plain) {
            if (n <= (uint32_t)cfg.split_batch_events) {
                st = hough_run_batch_split(sl.ctx_small[(size_t)b.kind], x, y, off, d_ids, d_koff, n, sl.d_peaks,
                                           d_npk, d_keep, d_status, sl.d_ws, sl.ws_bytes, s);
            } else {
                hough_ctx *c = n <= (uint32_t)cfg.small_batch_events ? sl.ctx_small[(size_t)b.kind]
                                                                      : sl.ctx[(size_t)b.kind];
                st = kd.host ? hough_run_batch(c, x, y, off, n, sl.d_peaks, d_npk, d_keep, d_status, s)
                             : hough_run_batch_gather(c, x, y, off, d_ids, d_koff, n, sl.d_peaks, d_npk, d_keep,
                                                      d_status, s);
            }
        } else {
            const uint32_t h0 = kd.host ? 0u : kd.pool.host_offsets[reqs[b.reqs[0]].event];
            hough_ctx *c = sl.ctx[(size_t)b.kind];
            st = hough_vote(c, x + h0, y + h0, b.hits, sl.d_acc, s);
            if (st == HOUGH_OK) st = hough_peaks(c, sl.d_acc, sl.d_peaks, (uint32_t)cap, d_npk, s);
            if (st == HOUGH_OK)
                st = hough_retain(c, x + h0, y + h0, b.hits, sl.d_peaks, d_npk, (uint32_t)cap, d_keep, s);
        }
        if (st != HOUGH_OK) return st;
        if (hipMemcpyAsync(sl.h_out, sl.d_out, 8u * n + b.hits, hipMemcpyDeviceToHost, s) != hipSuccess ||
            (cfg.copy_peaks && cap &&
             hipMemcpyAsync(sl.h_peaks, sl.d_peaks, n * cap * sizeof(hough_peak), hipMemcpyDeviceToHost, s) !=
                 hipSuccess) ||
            hipEventRecord(sl.done, s) != hipSuccess)
            return HOUGH_EDEVICE;
        return HOUGH_OK;
    }

    void complete(int si, const Batch &b, hough_serve_result *res) {
        const Slot &sl = slots[(size_t)si];
        const Kind &kd = kinds[(size_t)b.kind];
        const uint32_t n = (uint32_t)b.reqs.size();
        const uint32_t *h_npk = reinterpret_cast<const uint32_t *>(sl.h_out);
        const uint32_t *h_status = h_npk + n;
        const uint8_t *h_keep = sl.h_out + 8u * n;
        for (uint32_t j = 0; j < n; ++j) {
            const uint32_t r = b.reqs[j];
            hough_serve_result &o = res[r];
            o.n_peaks = h_npk[j];
            o.status = cfg.plain ? (o.n_peaks > (uint32_t)kd.p.max_peaks ? HOUGH_EV_PEAKS_TRUNCATED : 0u)
                                 : h_status[j];
            const uint32_t H = hits_of(b.kind, reqs[r].event);
            if (keep_out) std::memcpy(keep_out + keep_off[r], h_keep + sl.koff[j], H);
            if (peaks_out) {
                uint32_t m = o.n_peaks < (uint32_t)kd.p.max_peaks ? o.n_peaks : (uint32_t)kd.p.max_peaks;
                if (m > peaks_stride) m = peaks_stride;
                std::memcpy(peaks_out + (size_t)r * peaks_stride, sl.h_peaks + (size_t)j * kd.p.max_peaks,
                            (size_t)m * sizeof(hough_peak));
            }
        }
    }
};

// Cost-model backend: batches take the modelled time on their slot, the clock jumps to the next
// thing that happens.
struct ModelServer {
    const hough_serve_model *models = nullptr;
    std::vector<double> finish;          // per slot: completion time of its batch (+inf: idle)
    double t = 0.0;

    double now() const { return t; }
    void idle(double wake) {
        double next = wake;
        for (double f : finish) next = std::min(next, f);
        if (next < std::numeric_limits<double>::infinity() && next > t) t = next;
    }
    int poll(int s, bool *done) {
        *done = finish[(size_t)s] <= t;
        if (*done) finish[(size_t)s] = std::numeric_limits<double>::infinity();
        return HOUGH_OK;
    }
    int launch(int s, const Batch &b) {
        const hough_serve_model &m = models[b.kind];
        finish[(size_t)s] = t + m.fixed_us + m.per_event_us * (double)b.reqs.size() + m.per_hit_us * (double)b.hits;
        return HOUGH_OK;
    }
    void complete(int, const Batch &b, hough_serve_result *res) {
        for (uint32_t r : b.reqs) {
            res[r].n_peaks = 0;
            res[r].status = 0;
        }
    }
};

}  // namespace

extern "C" int hough_serve_run(const hough_serve_pool *pools, int32_t n_kinds, const hough_serve_config *cfg,
                               const hough_serve_request *reqs, uint32_t n_reqs, hough_serve_result *res,
                               uint8_t *keep_out, hough_peak *peaks_out, uint32_t peaks_stride) {
    if (!pools || n_kinds < 1 || !cfg || (n_reqs && (!reqs || !res))) return HOUGH_EINVAL;
    if (peaks_out && !cfg->copy_peaks) return HOUGH_EINVAL;
    HipServer *srv = new (std::nothrow) HipServer();
    if (!srv) return HOUGH_ENOMEM;
    srv->cfg = *cfg;
    srv->reqs = reqs;
    srv->keep_out = keep_out;
    srv->peaks_out = peaks_out;
    srv->peaks_stride = peaks_stride;
    for (int k = 0; k < n_kinds; ++k) {
        const hough_serve_pool &pl = pools[k];
        Kind kd;
        kd.pool = pl;
        kd.host = pl.host_x != nullptr;
        const bool resident = pl.x && pl.y && pl.offsets && !pl.host_x && !pl.host_y;
        const bool host = pl.host_x && pl.host_y && !pl.x && !pl.y && !pl.offsets;
        if (!pl.ctx || !pl.host_offsets || pl.n_events < 1 || pl.reserved != 0 || resident == host ||
            hough_get_params(pl.ctx, &kd.p) != HOUGH_OK) {
            delete srv;
            return HOUGH_EINVAL;
        }
        srv->any_host = srv->any_host || host;
        srv->any_resident = srv->any_resident || resident;
        kd.acc_bytes = (size_t)kd.p.n_theta * kd.p.n_rho * (kd.p.acc_type == HOUGH_ACC_U16 ? 2 : 4);
        if ((size_t)kd.p.max_peaks > srv->cap_max) srv->cap_max = (size_t)kd.p.max_peaks;
        if (kd.acc_bytes > srv->acc_max) srv->acc_max = kd.acc_bytes;
        srv->kinds.push_back(kd);
    }
    std::vector<uint32_t> hits(n_reqs ? n_reqs : 1);
    srv->keep_off.resize(n_reqs ? n_reqs : 1);
    uint64_t acc_hits = 0;
    for (uint32_t i = 0; i < n_reqs; ++i) {
        if (reqs[i].kind < 0 || reqs[i].kind >= n_kinds || reqs[i].event >= srv->kinds[(size_t)reqs[i].kind].pool.n_events) {
            delete srv;
            return HOUGH_EINVAL;
        }
        hits[i] = srv->hits_of(reqs[i].kind, reqs[i].event);
        srv->keep_off[i] = acc_hits;
        acc_hits += hits[i];
    }
    hough_serve::Trace tr{reqs, n_reqs, hits.data()};
    int rc = hough_serve::validate(*cfg, n_kinds, tr);
    if (rc == HOUGH_OK) rc = srv->setup();
    if (rc == HOUGH_OK) {
        srv->t0 = Clock::now();
        rc = hough_serve::run(*srv, *cfg, n_kinds, tr, res);
    }
    delete srv;   // waits for its streams, frees its buffers
    return rc;
}

extern "C" int hough_serve_simulate(int32_t n_kinds, const hough_serve_config *cfg, const hough_serve_request *reqs,
                                    const uint32_t *hits, uint32_t n_reqs, const hough_serve_model *models,
                                    hough_serve_result *res) {
    if (!cfg || !models || (n_reqs && (!reqs || !hits || !res))) return HOUGH_EINVAL;
    for (int k = 0; k < n_kinds; ++k) {
        const hough_serve_model &m = models[k];
        if (!(m.fixed_us >= 0.0) || !(m.per_event_us >= 0.0) || !(m.per_hit_us >= 0.0) ||
            m.fixed_us + m.per_event_us + m.per_hit_us <= 0.0)
            return HOUGH_EINVAL;
    }
    hough_serve::Trace tr{reqs, n_reqs, hits};
    int rc = hough_serve::validate(*cfg, n_kinds, tr);
    if (rc != HOUGH_OK) return rc;
    if (cfg->plain)
        for (uint32_t i = 0; i < n_reqs; ++i)
            if (hits[i] > (uint32_t)cfg->max_batch_hits) return HOUGH_EINVAL;
    ModelServer m;
    m.models = models;
    m.finish.assign((size_t)cfg->n_streams, std::numeric_limits<double>::infinity());
    return hough_serve::run(m, *cfg, n_kinds, tr, res);
}
