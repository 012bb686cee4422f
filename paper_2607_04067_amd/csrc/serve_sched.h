// Scheduling core of the serving loop (include/hough_serve.h), independent of how batches are
// executed: open-loop arrivals into per-kind FIFO queues, memory-based admission into stream
// slots, continuous batching, and the per-request bookkeeping.  hough_serve.cpp runs it over HIP
// streams (hough_serve_run) and over a cost model with a simulated clock (hough_serve_simulate),
// so the host tests exercise exactly the code that serves.
//
// A Backend provides
//   double now();                      microseconds since the run's start
//   void idle(double wake_us);         nothing to do before wake_us (+inf: before a completion)
//   int launch(int slot, const Batch&) enqueue the batch on the slot; HOUGH_OK or an error
//   int poll(int slot, bool *done)     whether the slot's batch has completed
//   void complete(int slot, const Batch&, hough_serve_result *res)
//                                      write the batch's per-request outputs (counts, keep bytes)
#pragma once

#include <algorithm>
#include <cstdint>
#include <limits>
#include <vector>

#include "../../include/hough_serve.h"

namespace hough_serve {

struct Batch {
    int kind = 0;
    std::vector<uint32_t> reqs;     // request indices, largest event first (ties: earlier request)
    uint32_t hits = 0;              // hits of the batch (<= max_batch_hits)
    double t_launch = 0.0;
};

struct Trace {
    const hough_serve_request *reqs = nullptr;
    uint32_t n = 0;
    const uint32_t *hits = nullptr;  // [n] hits of each request's event
};

// Checks shared by both entry points: config ranges, request kinds, ordered arrivals, and every
// request's event fitting one slot's arena.
inline int validate(const hough_serve_config &cfg, int n_kinds, const Trace &tr) {
    if (n_kinds < 1 || cfg.n_streams < 1 || cfg.n_streams > 32 || cfg.max_batch_events < 1 ||
        cfg.max_batch_hits < 1 || cfg.small_batch_events < 0 || cfg.split_batch_events < 0 ||
        cfg.reserved != 0 || !(cfg.max_wait_us >= 0.0))
        return HOUGH_EINVAL;
    for (uint32_t i = 0; i < tr.n; ++i) {
        const hough_serve_request &r = tr.reqs[i];
        if (r.kind < 0 || r.kind >= n_kinds || tr.hits[i] > (uint32_t)cfg.max_batch_hits ||
            !(r.arrival_us >= 0.0) || (i && r.arrival_us < tr.reqs[i - 1].arrival_us))
            return HOUGH_EINVAL;
    }
    return HOUGH_OK;
}

// Run the trace to completion.  res[i]: launch_us, done_us, batch_events and slot are written
// here; the backend's complete() writes the rest.
template <class Backend>
int run(Backend &be, const hough_serve_config &cfg, int n_kinds, const Trace &tr, hough_serve_result *res) {
    const double inf = std::numeric_limits<double>::infinity();
    const uint32_t cap_events = cfg.plain ? 1u : (uint32_t)cfg.max_batch_events;
    // per-kind FIFO of arrived requests not yet admitted (arrivals are ordered, so each queue is)
    std::vector<std::vector<uint32_t>> pend((size_t)n_kinds);
    std::vector<size_t> head((size_t)n_kinds, 0);
    for (auto &q : pend) q.reserve(tr.n);
    std::vector<Batch> slot((size_t)cfg.n_streams);
    std::vector<char> busy((size_t)cfg.n_streams, 0);
    for (Batch &b : slot) b.reqs.reserve(cap_events);

    uint32_t next = 0, completed = 0;
    while (completed < tr.n) {
        double t = be.now();
        while (next < tr.n && tr.reqs[next].arrival_us <= t) {
            pend[(size_t)tr.reqs[next].kind].push_back(next);
            ++next;
        }
        bool progressed = false;
        for (size_t s = 0; s < slot.size(); ++s) {
            if (!busy[s]) continue;
            bool done = false;
            const int rc = be.poll((int)s, &done);
            if (rc != HOUGH_OK) return rc;
            if (!done) continue;
            const double t_done = be.now();
            Batch &b = slot[s];
            for (uint32_t r : b.reqs) {
                res[r].launch_us = b.t_launch;
                res[r].done_us = t_done;
                res[r].batch_events = (uint32_t)b.reqs.size();
                res[r].slot = (uint32_t)s;
            }
            be.complete((int)s, b, res);
            completed += (uint32_t)b.reqs.size();
            busy[s] = 0;
            progressed = true;
        }
        t = be.now();
        double wake = next < tr.n ? tr.reqs[next].arrival_us : inf;
        for (size_t s = 0; s < slot.size(); ++s) {
            if (busy[s]) continue;
            // the kind whose oldest waiting request arrived first
            int k = -1;
            double oldest = 0.0;
            for (int kk = 0; kk < n_kinds; ++kk) {
                if (head[(size_t)kk] >= pend[(size_t)kk].size()) continue;
                const double a = tr.reqs[pend[(size_t)kk][head[(size_t)kk]]].arrival_us;
                if (k < 0 || a < oldest) { k = kk; oldest = a; }
            }
            if (k < 0) break;
            std::vector<uint32_t> &q = pend[(size_t)k];
            size_t &h = head[(size_t)k];
            if (!cfg.plain && cfg.max_wait_us > 0.0 && q.size() - h < (size_t)cfg.max_batch_events &&
                t - oldest < cfg.max_wait_us) {
                wake = std::min(wake, oldest + cfg.max_wait_us);   // hold the partial batch a little
                break;
            }
            Batch &b = slot[s];
            b.kind = k;
            b.reqs.clear();
            b.hits = 0;
            while (h < q.size() && b.reqs.size() < cap_events) {      // memory-based admission
                const uint32_t H = tr.hits[q[h]];
                if ((uint64_t)b.hits + H > (uint64_t)cfg.max_batch_hits) break;
                b.reqs.push_back(q[h]);
                b.hits += H;
                ++h;
            }
            // largest first: the smallest events fill the kernel's tail
            std::sort(b.reqs.begin(), b.reqs.end(), [&](uint32_t a, uint32_t c) {
                return tr.hits[a] != tr.hits[c] ? tr.hits[a] > tr.hits[c] : a < c;
            });
            b.t_launch = t;
            const int rc = be.launch((int)s, b);
            if (rc != HOUGH_OK) return rc;
            busy[s] = 1;
            progressed = true;
        }
        if (!progressed) be.idle(wake);
    }
    return HOUGH_OK;
}

}  // namespace hough_serve
