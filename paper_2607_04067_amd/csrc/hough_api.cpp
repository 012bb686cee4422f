// Host side of libhough.so: parameter validation, the per-column constants, workspace
// ownership and kernel dispatch behind the C ABI declared in include/hough.h.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "hough_internal.h"

struct hough_ctx {
    hough_params p;
    int device;
    float *d_tables;        // C[n_theta] then S[n_theta]
    uint32_t *d_work;       // [0], [1]: work and exit counters of the fused kernels; from [64]:
                            // hough_peaks' per-block peak counts
    uint32_t *d_order;      // [kOrderMaxEvents] the fused kernel's largest-first schedule
    uint32_t *d_iter_bm;    // the iterative finder's suppression bitmap when it does not fit LDS
    hough::IterPlan iter1;  // the iterative finder on one event (hough_peaks_iterative)
    hough::IterPlan iterb;  // ... over a batch (hough_run_batch_iterative), two workgroups per CU
    hough::GridArgs g;
    hough::BatchPlan plan;  // the fused kernel's launch shape (fused != 0)
    int fused;              // 1: the fused kernel holds the grid's whole column (and windows of it);
                            // 2: only windows of it (taller grids, theta not periodic; the split
                            // form spills every event); 0: every batch event spills
    uint32_t *d_spill;      // spill_wgs slices of spill_stride words (the spill path's accumulators)
    size_t spill_stride;
    int spill_wgs;
    size_t lds_limit;
    int n_cu;
};

namespace {

constexpr double kPi = 3.14159265358979323846;

int lds_limit_bytes(int device, size_t *out) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
        return HOUGH_EDEVICE;
    *out = (size_t)v;
    return HOUGH_OK;
}

// Tallest rho axis the library takes: the per-event path's kernels need an LDS slab of at least
// one row (hough_vote), three theta rows of the grid (hough_peaks) and one 64-row group of
// dilated words (hough_retain); batches of grids whose column does not fit the fused kernel's
// tile run through the spill path.
constexpr int kMaxNRho = 8192;

bool grid_fits(int n_rho, size_t limit) {
    if (n_rho > kMaxNRho) return false;
    if (hough::vote_slab_rows(n_rho, limit) < 1) return false;
    if (hough::peak_block_waves(n_rho, limit) < 2) return false;
    const size_t words = (size_t)(n_rho + 31) / 32;
    return 8 * 64 * 8 + words * 64 * 4 + 512 <= limit;     // hough_retain's stages and one row group
}

bool fused_fits(int n_rho, size_t limit) {
    hough::BatchPlan p;
    return hough::plan_batch(1, n_rho, 4, 1, limit, &p) == 0;
}

// Spill-path workgroups: one per CU within a 2 GiB budget where every event may spill (each
// takes its own event, so the workgroup count is the path's parallelism: 1000 x 2000 bins with
// 4.8 MB per slice get one per CU), else a few for the rare events above the fused kernel's hit
// limit.
constexpr size_t kSpillBudgetBytes = (size_t)2048 << 20;
int spill_workgroups(size_t stride_words, int n_cu, bool all) {
    const size_t per = stride_words * 4;
    size_t n = per ? kSpillBudgetBytes / per : 1;
    if (!all && n > 4) n = 4;
    if (n > (size_t)n_cu) n = (size_t)n_cu;
    return n < 1 ? 1 : (int)n;
}

// Bound on u^2 + v^2 under which a hit's bin t = fma(u, C_j, fma(v, S_j, B)) lies strictly
// inside (0, n_rho) for every column: |t - B| is at most A * sqrt(u^2 + v^2) plus the rounding
// of C_j, S_j and the two fmas (a few 2^-24 of n_rho), well inside the margin kept here; the
// float sum u^2 + v^2 itself is within 2^-22 of the exact one, inside the 1e-6 shrink.
float safe_radius2(double A, double B, int n_rho) {
    const double margin = 1e-5 * n_rho + 0.01;
    const double room = (B < n_rho - B ? B : n_rho - B) - margin;
    if (!(room > 0.0)) return 0.0f;
    const double r = room / (fabs(A) * 1.0002);
    float f = (float)(r * r * (1.0 - 1e-6));
    if ((double)f > r * r * (1.0 - 1e-6)) f = nextafterf(f, 0.0f);
    return f;
}

// Default launch shape of the fused kernel: the candidate with the most resident waves per CU
// (from the occupancy API, which accounts for LDS, VGPRs and SGPRs); ties go to the earlier
// candidate.  8 waves split the 16-row peak units and the 32-row words of a 256-row tile evenly
// and measured fastest wherever they tie with 6, 12 or 16; 12 waves win where the tile leaves
// room for two workgroups per CU only (720 x 512: 24 resident waves instead of 16, 8% faster).
int default_plan(hough_ctx *c) {
    int best = -1;
    hough::BatchPlan pick{};
    const int waves_opts[5] = {8, 16, 12, 6, 4};
    for (int wi = 0; wi < 5; ++wi) {
        hough::BatchPlan p;
        if (hough::plan_batch(c->p.n_theta, c->p.n_rho, waves_opts[wi], 1, c->lds_limit, &p) != 0) continue;
        p.per_cu = hough::prepare_batch(&p);
        if (p.per_cu < 1 || p.split_per_cu < 1) continue;
        const int score = p.per_cu * p.waves;
        if (score > best) { best = score; pick = p; }
    }
    if (best < 0) return HOUGH_EINVAL;
    if (hough::prepare_batch(&pick) < 1) return HOUGH_EDEVICE;
    c->plan = pick;
    return HOUGH_OK;
}

// The tallest windowed tile (a multiple of 32 rows) that lets groups_per_cu workgroups share a
// CU, if any (one column group, theta not periodic): for more workgroups per CU than a
// whole-column tile allows, and for grids taller than that tile.  Events whose hits reach
// beyond the window go to the spill kernel.
int windowed_plan(const hough_ctx *c, int waves, int groups, int groups_per_cu, hough::BatchPlan *out) {
    if (groups != 1 || c->g.periodic) return -1;
    const bool need_split = c->fused == 1;
    for (int win = ((c->p.n_rho - 1) / 32) * 32; win >= 32; win -= 32) {
        hough::BatchPlan p;
        if (hough::plan_batch(c->p.n_theta, c->p.n_rho, waves, groups, c->lds_limit, &p, win, need_split) != 0)
            continue;
        p.per_cu = hough::prepare_batch(&p);
        if (p.per_cu >= groups_per_cu && (!need_split || p.split_per_cu >= 1)) {
            *out = p;
            return 0;
        }
    }
    return -1;
}

// Default launch shape where only windows of the column fit (fused == 2): the tallest window
// with the most resident waves per CU (the most events fit, the rest spill); ties go to the
// earlier candidate.
int default_windowed_plan(hough_ctx *c) {
    const int waves_opts[5] = {16, 8, 12, 6, 4};
    hough::BatchPlan cand[5];
    bool ok[5];
    int tallest = 0;
    for (int wi = 0; wi < 5; ++wi) {
        ok[wi] = windowed_plan(c, waves_opts[wi], 1, 1, &cand[wi]) == 0;
        if (ok[wi] && cand[wi].win > tallest) tallest = cand[wi].win;
    }
    // the most resident waves among the windows within one 32-row step of the tallest (a
    // window only has to hold the rows an event's hits reach; on 1000 x 2000 bins 16 waves
    // with 1,056 rows ran 0.72 ms per 1,000 events against 0.86 for 8 waves with 1,088),
    // then the taller window
    int best = -1;
    hough::BatchPlan pick{};
    for (int wi = 0; wi < 5; ++wi) {
        if (!ok[wi] || cand[wi].win < tallest - 32) continue;
        const int score = cand[wi].per_cu * cand[wi].waves * 65536 + cand[wi].win;
        if (score > best) { best = score; pick = cand[wi]; }
    }
    if (best < 0) return HOUGH_EINVAL;
    if (hough::prepare_batch(&pick) < 1) return HOUGH_EDEVICE;
    c->plan = pick;
    return HOUGH_OK;
}

// A context's tables and workspace live on the device it was configured on.
bool on_device(const hough_ctx *c) {
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess && dev == c->device;
}

}  // namespace

extern "C" {

const char *hough_status_string(int status) {
    switch (status) {
        case HOUGH_OK: return "ok";
        case HOUGH_EINVAL: return "invalid argument";
        case HOUGH_ENOMEM: return "out of memory";
        case HOUGH_EOVERFLOW: return "count may overflow the accumulator type";
        case HOUGH_EDEVICE: return "HIP runtime or launch failure";
        case HOUGH_ETOOLARGE: return "batch needs more than the library's static scratch";
        default: return "unknown status";
    }
}

int32_t hough_max_n_rho(void) {
    int dev = 0;
    size_t limit = 0;
    if (hipGetDevice(&dev) != hipSuccess || lds_limit_bytes(dev, &limit) != HOUGH_OK) return 0;
    int lo = 0, hi = 65535;
    while (lo < hi) {                      // largest n_rho whose kernels fit the LDS
        const int mid = (lo + hi + 1) / 2;
        if (grid_fits(mid, limit)) lo = mid; else hi = mid - 1;
    }
    return lo;
}

int hough_config(const hough_params *p, hough_ctx **out) {
    if (!p || !out) return HOUGH_EINVAL;
    *out = nullptr;
    if (p->n_theta < 1 || p->n_theta > 65535 || p->n_rho < 1 || p->n_rho > 65535) return HOUGH_EINVAL;
    if (!isfinite(p->rho_min) || !isfinite(p->rho_max) || !(p->rho_max > p->rho_min)) return HOUGH_EINVAL;
    if (p->acc_type != HOUGH_ACC_U16 && p->acc_type != HOUGH_ACC_I32) return HOUGH_EINVAL;
    if (p->threshold < 1 || p->rho_window < 0 || p->max_peaks < 0) return HOUGH_EINVAL;
    if ((p->flags & ~(HOUGH_FLAG_THETA_PERIODIC | HOUGH_FLAG_DEDUP)) != 0 || p->reserved != 0)
        return HOUGH_EINVAL;
    if ((p->flags & HOUGH_FLAG_THETA_PERIODIC) && (p->n_theta < 2 || p->rho_min != -p->rho_max))
        return HOUGH_EINVAL;
    if ((int64_t)p->n_theta * (int64_t)p->n_rho > (int64_t)INT32_MAX) return HOUGH_EINVAL;   // 32-bit cell indices
    const double A = (double)p->n_rho / (p->rho_max - p->rho_min);
    const double B = -p->rho_min * A;
    if (!isfinite(A) || !isfinite(B) || !(fabs(A) < 1e30) || !(fabs(B) < 1e30)) return HOUGH_EINVAL;

    const char *fail = getenv("HOUGH_TEST_FAIL_ALLOC");   // test hook for the ENOMEM path
    if (fail && fail[0] == '1') return HOUGH_ENOMEM;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HOUGH_EDEVICE;
    size_t limit = 0;
    int rc = lds_limit_bytes(dev, &limit);
    if (rc == HOUGH_OK) rc = hough::scratch_init(dev);   // once per device
    if (rc != HOUGH_OK) return rc;
    if (!grid_fits(p->n_rho, limit)) return HOUGH_EINVAL;

    hough_ctx *c = new (std::nothrow) hough_ctx();
    if (!c) return HOUGH_ENOMEM;
    c->p = *p;
    c->device = dev;
    c->lds_limit = limit;
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete c;
        return HOUGH_EDEVICE;
    }

    // Per-column constants: theta_j = (j*pi)/n_theta in double, times A, rounded once to float.
    std::vector<float> tab(2 * (size_t)p->n_theta);
    for (int j = 0; j < p->n_theta; ++j) {
        const double theta = ((double)j * kPi) / (double)p->n_theta;
        tab[j] = (float)(A * cos(theta));
        tab[p->n_theta + j] = (float)(A * sin(theta));
    }
    if (hipMalloc(&c->d_tables, tab.size() * sizeof(float)) != hipSuccess) {
        delete c;
        return HOUGH_ENOMEM;
    }
    const int peak_waves = hough::peak_block_waves(p->n_rho, limit);
    const size_t work_bytes = 256 + 4 * (size_t)((p->n_theta + peak_waves - 1) / peak_waves);
    if (hipMalloc(&c->d_work, work_bytes) != hipSuccess) {
        (void)hipFree(c->d_tables);
        delete c;
        return HOUGH_ENOMEM;
    }
    if (hipMalloc(&c->d_order, sizeof(uint32_t) * hough::kOrderMaxEvents) != hipSuccess) {
        (void)hipFree(c->d_work);
        (void)hipFree(c->d_tables);
        delete c;
        return HOUGH_ENOMEM;
    }
    c->iter1 = hough::plan_iterative(p->n_theta, p->n_rho, limit, 1);
    c->iterb = hough::plan_iterative(p->n_theta, p->n_rho, limit, 2);
    if (c->iter1.gbm && hipMalloc(&c->d_iter_bm, c->iter1.bm_bytes) != hipSuccess) {
        hough_destroy(c);
        return HOUGH_ENOMEM;
    }
    c->fused = fused_fits(p->n_rho, limit) ? 1 : ((p->flags & HOUGH_FLAG_THETA_PERIODIC) ? 0 : 2);
    c->spill_stride = hough::spill_stride(p->n_theta, p->n_rho);
    c->spill_wgs = spill_workgroups(c->spill_stride, c->n_cu, c->fused != 1);
    // fewer slices where the device cannot spare the budget
    while (hipMalloc(&c->d_spill, c->spill_stride * 4 * (size_t)c->spill_wgs) != hipSuccess) {
        (void)hipGetLastError();             // clear the failed allocation's error
        c->d_spill = nullptr;
        if (c->spill_wgs == 1) {
            hough_destroy(c);
            return HOUGH_ENOMEM;
        }
        c->spill_wgs = (c->spill_wgs + 1) / 2;
    }
    if (hipMemcpy(c->d_tables, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->d_work, 0, work_bytes) != hipSuccess) {
        hough_destroy(c);
        return HOUGH_EDEVICE;
    }

    hough::GridArgs &g = c->g;
    g.C = c->d_tables;
    g.S = c->d_tables + p->n_theta;
    g.n_theta = p->n_theta;
    g.n_rho = p->n_rho;
    g.Bf = (float)B;
    g.nrho_f = (float)p->n_rho;
    g.safe_r2 = safe_radius2(A, B, p->n_rho);
    g.threshold = (uint32_t)p->threshold;
    g.rho_window = p->rho_window < p->n_rho ? p->rho_window : p->n_rho;
    g.periodic = (p->flags & HOUGH_FLAG_THETA_PERIODIC) ? 1 : 0;
    g.dedup = (p->flags & HOUGH_FLAG_DEDUP) ? 1 : 0;
    g.vote_rows = hough::vote_slab_rows(p->n_rho, limit);
    g.peak_waves = peak_waves;
    // bounds for a windowed tile's rows: the largest |(C_j, S_j)| of the float tables and B
    g.wA = 0.0;
    for (int j = 0; j < p->n_theta; ++j) {
        const double cj = tab[j], sj = tab[p->n_theta + j];
        g.wA = std::max(g.wA, sqrt(cj * cj + sj * sj));
    }
    g.wB = (double)g.Bf;

    rc = c->fused == 1 ? default_plan(c) : (c->fused == 2 ? default_windowed_plan(c) : HOUGH_OK);
    if (rc != HOUGH_OK) {
        hough_destroy(c);
        return rc;
    }
    *out = c;
    return HOUGH_OK;
}

void hough_destroy(hough_ctx *c) {
    if (!c) return;
    if (c->d_tables) (void)hipFree(c->d_tables);
    if (c->d_work) (void)hipFree(c->d_work);
    if (c->d_order) (void)hipFree(c->d_order);
    if (c->d_iter_bm) (void)hipFree(c->d_iter_bm);
    if (c->d_spill) (void)hipFree(c->d_spill);
    delete c;
}

int hough_get_params(const hough_ctx *c, hough_params *out) {
    if (!c || !out) return HOUGH_EINVAL;
    *out = c->p;
    return HOUGH_OK;
}

uint32_t hough_max_batch_hits(const hough_ctx *c) { return c ? UINT32_MAX : 0u; }

int hough_get_batch_plan(const hough_ctx *c, hough_batch_plan *out) {
    if (!c || !out) return HOUGH_EINVAL;
    if (!c->fused) {                      // no fused kernel for this grid: all zero
        *out = hough_batch_plan{0, 0, 0, 0, 0};
        return HOUGH_OK;
    }
    out->waves_per_group = c->plan.waves;
    out->column_groups = c->plan.groups;
    out->groups_per_cu = c->plan.per_cu;
    out->lds_bytes = (int32_t)c->plan.lds_bytes;
    out->window_rows = c->plan.win;
    return HOUGH_OK;
}

int hough_set_batch_plan(hough_ctx *c, int32_t waves_per_group, int32_t column_groups,
                         int32_t groups_per_cu) {
    if (!c || groups_per_cu < 0 || !c->fused) return HOUGH_EINVAL;
    hough::BatchPlan p{};
    if (c->fused == 1) {
        if (hough::plan_batch(c->p.n_theta, c->p.n_rho, waves_per_group, column_groups, c->lds_limit, &p) != 0)
            return HOUGH_EINVAL;
        p.per_cu = hough::prepare_batch(&p);
        if (p.per_cu >= 1 && p.split_per_cu >= 1 && groups_per_cu > p.per_cu &&
            windowed_plan(c, waves_per_group, column_groups, groups_per_cu, &p) != 0)
            p.per_cu = 0;
        if (p.split_per_cu < 1) p.per_cu = 0;
    } else if (windowed_plan(c, waves_per_group, column_groups, groups_per_cu > 0 ? groups_per_cu : 1, &p) != 0) {
        p.per_cu = 0;                         // only windows of the column fit
    }
    if (p.per_cu < 1 || groups_per_cu > p.per_cu) {
        hough::BatchPlan keep = c->plan;
        (void)hough::prepare_batch(&keep);
        return HOUGH_EINVAL;
    }
    if (groups_per_cu > 0) p.per_cu = groups_per_cu;
    c->plan = p;
    return HOUGH_OK;
}

int hough_vote(hough_ctx *c, const float *x, const float *y, uint32_t n_hits, void *acc, void *stream) {
    if (!c || !acc) return HOUGH_EINVAL;
    if (c->p.flags & HOUGH_FLAG_DEDUP) return HOUGH_EINVAL;      // no duplicate pass on this path
    if (!on_device(c)) return HOUGH_EINVAL;
    if (n_hits && (!x || !y)) return HOUGH_EINVAL;
    if (c->p.acc_type == HOUGH_ACC_U16 && n_hits > 65535u) return HOUGH_EOVERFLOW;
    const hipError_t e = hough::launch_vote(c->g, x, y, n_hits, acc, c->p.acc_type, (hipStream_t)stream);
    return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
}

int hough_peaks(hough_ctx *c, const void *acc, hough_peak *peaks, uint32_t cap, uint32_t *n_peaks,
                void *stream) {
    if (!c || !acc || !n_peaks || (cap && !peaks)) return HOUGH_EINVAL;
    if (!on_device(c)) return HOUGH_EINVAL;
    if (((uintptr_t)peaks & 7u) != 0) return HOUGH_EINVAL;
    const hipError_t e = hough::launch_peaks(c->g, acc, c->p.acc_type, peaks, cap, n_peaks, c->d_work + 64,
                                             (hipStream_t)stream);
    return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
}

int hough_peaks_iterative(hough_ctx *c, const void *acc, uint32_t frac_num, uint32_t frac_den,
                          int32_t r_theta, int32_t r_rho, hough_peak *peaks, uint32_t cap,
                          uint32_t *n_peaks, uint32_t *status, void *stream) {
    if (!c || !acc || !n_peaks || !status || (cap && !peaks)) return HOUGH_EINVAL;
    if (!on_device(c)) return HOUGH_EINVAL;
    if (frac_den == 0 || r_theta < 0 || r_rho < 0) return HOUGH_EINVAL;
    if (((uintptr_t)peaks & 7u) != 0) return HOUGH_EINVAL;
    // a window wider than the grid suppresses what the grid's width does
    r_theta = r_theta < c->p.n_theta ? r_theta : c->p.n_theta;
    r_rho = r_rho < c->p.n_rho ? r_rho : c->p.n_rho;
    const hipError_t e = hough::launch_peaks_iterative(c->g, acc, c->p.acc_type, frac_num, frac_den,
                                                       r_theta, r_rho, peaks, cap, n_peaks, status, c->iter1,
                                                       c->d_iter_bm, (hipStream_t)stream);
    return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace of hough_run_batch_iterative: the events' 16-bit accumulators, then (when the
// finder's bitmap does not fit LDS) one suppression bitmap per event.
size_t hough_iterative_workspace_bytes(const hough_ctx *c, uint32_t n_events) {
    if (!c) return 0;
    const size_t acc = align256((size_t)n_events * (size_t)c->p.n_theta * (size_t)c->p.n_rho * sizeof(uint16_t));
    return acc + (c->iterb.gbm ? (size_t)n_events * c->iterb.bm_bytes : 0);
}

int hough_run_batch_iterative(hough_ctx *c, const float *x, const float *y, const uint32_t *offsets,
                              uint32_t n_events, uint32_t frac_num, uint32_t frac_den, int32_t r_theta,
                              int32_t r_rho, hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep,
                              uint32_t *status, void *workspace, size_t workspace_bytes, void *stream) {
    if (!c) return HOUGH_EINVAL;
    if (!on_device(c)) return HOUGH_EINVAL;
    if (frac_den == 0 || r_theta < 0 || r_rho < 0) return HOUGH_EINVAL;
    if (n_events == 0) return HOUGH_OK;
    if (!x || !y || !offsets || !n_peaks || !keep || !status || !workspace) return HOUGH_EINVAL;
    if (c->p.max_peaks > 0 && !peaks) return HOUGH_EINVAL;
    if (((uintptr_t)peaks & 7u) != 0 || ((uintptr_t)workspace & 255u) != 0) return HOUGH_EINVAL;
    if (workspace_bytes < hough_iterative_workspace_bytes(c, n_events)) return HOUGH_EINVAL;
    r_theta = r_theta < c->p.n_theta ? r_theta : c->p.n_theta;
    r_rho = r_rho < c->p.n_rho ? r_rho : c->p.n_rho;
    const size_t acc_bytes = align256((size_t)n_events * (size_t)c->p.n_theta * (size_t)c->p.n_rho * sizeof(uint16_t));
    uint32_t *gbm = c->iterb.gbm ? reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + acc_bytes) : nullptr;
    hough::BatchArgs a{};
    a.x = x;
    a.y = y;
    a.offsets = offsets;
    a.ids = nullptr;
    a.keep_offsets = nullptr;
    a.n_events = n_events;
    a.peaks = c->p.max_peaks > 0 ? peaks : nullptr;
    a.n_peaks = n_peaks;
    a.keep = keep;
    a.status = status;
    a.max_peaks = (uint32_t)c->p.max_peaks;
    a.order = nullptr;
    a.queue = nullptr;
    a.frac_num = 0;
    a.frac_den = 0;
    const hipError_t e = hough::launch_batch_iterative(c->g, a, static_cast<uint16_t *>(workspace), frac_num,
                                                       frac_den, r_theta, r_rho, c->iterb, gbm, (hipStream_t)stream);
    return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
}

int hough_track_params(hough_ctx *c, const float *x, const float *y, uint32_t n_hits,
                       const hough_peak *peaks, const uint32_t *n_peaks, uint32_t cap,
                       double b_tesla, hough_track *tracks, void *stream) {
    if (!c || !n_peaks || (cap && (!peaks || !tracks))) return HOUGH_EINVAL;
    if (!on_device(c)) return HOUGH_EINVAL;
    if (n_hits && (!x || !y)) return HOUGH_EINVAL;
    if (((uintptr_t)peaks & 7u) != 0 || ((uintptr_t)tracks & 7u) != 0) return HOUGH_EINVAL;
    if (!isfinite(b_tesla)) return HOUGH_EINVAL;
    const hipError_t e = hough::launch_track_params(c->g, x, y, n_hits, peaks, n_peaks, cap, c->p.rho_min,
                                                    c->p.rho_max, b_tesla, tracks, (hipStream_t)stream);
    return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
}

int hough_retain(hough_ctx *c, const float *x, const float *y, uint32_t n_hits,
                 const hough_peak *peaks, const uint32_t *n_peaks, uint32_t cap, uint8_t *keep,
                 void *stream) {
    if (!c || !n_peaks || (cap && !peaks)) return HOUGH_EINVAL;
    if (!on_device(c)) return HOUGH_EINVAL;
    if (n_hits && (!x || !y || !keep)) return HOUGH_EINVAL;
    if (((uintptr_t)peaks & 7u) != 0) return HOUGH_EINVAL;
    const hipError_t e = hough::launch_retain(c->g, x, y, n_hits, peaks, n_peaks, cap, keep,
                                              (hipStream_t)stream);
    return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
}

static int run_batch_common(hough_ctx *c, const float *x, const float *y, const uint32_t *offsets,
                            const uint32_t *ids, const uint32_t *keep_offsets, uint32_t n_events,
                            hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep, uint32_t *status,
                            void *stream, bool split = false, void *workspace = nullptr,
                            size_t workspace_bytes = 0, uint32_t frac_num = 0, uint32_t frac_den = 0) {
    if (!c) return HOUGH_EINVAL;
    if (!on_device(c)) return HOUGH_EINVAL;
    if (n_events == 0) return HOUGH_OK;
    if (!x || !y || !offsets || !n_peaks || !keep || !status) return HOUGH_EINVAL;
    if (c->p.max_peaks > 0 && !peaks) return HOUGH_EINVAL;
    if (((uintptr_t)peaks & 7u) != 0) return HOUGH_EINVAL;
    hough::BatchArgs a{};
    a.x = x;
    a.y = y;
    a.offsets = offsets;
    a.ids = ids;
    a.keep_offsets = keep_offsets;
    a.n_events = n_events;
    a.peaks = c->p.max_peaks > 0 ? peaks : nullptr;
    a.n_peaks = n_peaks;
    a.keep = keep;
    a.status = status;
    a.max_peaks = (uint32_t)c->p.max_peaks;
    a.order = nullptr;
    a.queue = c->d_work;
    a.frac_num = frac_num;
    a.frac_den = frac_den;
    // every event through the spill path: no fused kernel for this grid, or the split form on a
    // grid whose whole column does not fit it (the split form gives the same results)
    const bool spill_all = !c->fused || (split && c->fused == 2);
    hough::SpillArgs spill{c->d_spill, c->spill_stride, c->d_work + 2, spill_all ? 1u : 0u};
    // otherwise the fused (or split) kernel counts the events it leaves to the spill kernel in
    // the spill kernel's first counter, so that the spill kernel skips its scan when none
    a.spill_count = spill_all ? nullptr : c->d_work + 2;
    hipError_t e = hipSuccess;
    if (spill_all) {
        if (c->g.dedup) e = hough::launch_dedup(a, (hipStream_t)stream);
        if (e == hipSuccess) e = hough::launch_spill(c->g, a, spill, c->spill_wgs, (hipStream_t)stream);
        return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
    }
    hough::BatchPlan plan = c->plan;
    long grid = (long)plan.per_cu * c->n_cu;
    if (grid > (long)n_events) grid = n_events;
    plan.grid = (int)grid;
    hough::SplitArgs sp;
    if (split) {
        if (!hough::split_layout(c->p.n_theta, c->p.n_rho, c->plan.groups, n_events, workspace, workspace_bytes,
                                 &sp))
            return HOUGH_EINVAL;
        const long items = (long)n_events * sp.n_tiles;
        if (items >= (1L << 31)) return HOUGH_EINVAL;      // the work queue counts in 32 bits
        // the split form holds the whole column, whatever window the fused kernel's plan has
        const int per = c->plan.per_cu < c->plan.split_per_cu ? c->plan.per_cu : c->plan.split_per_cu;
        long g2 = (long)per * c->n_cu;
        plan.grid = (int)(g2 < items ? g2 : items);
    }
    if (c->g.dedup) e = hough::launch_dedup(a, (hipStream_t)stream);   // marks later copies in keep
    // more events than resident workgroups: take them largest first, so that the batch does not
    // end waiting for a large event begun last (a gathered batch keeps the caller's order)
    if (e == hipSuccess && !split && !ids && n_events > (uint32_t)plan.grid && n_events <= hough::kOrderMaxEvents) {
        e = hough::launch_order(offsets, n_events, c->d_order, (hipStream_t)stream);
        a.order = c->d_order;
    }
    if (e == hipSuccess)
        e = split ? hough::launch_batch_split(c->g, plan, a, sp, (hipStream_t)stream)
                  : hough::launch_batch(c->g, plan, a, (hipStream_t)stream);
    // events above the fused kernel's hit limit or beyond its window (flagged and skipped there),
    // through the spill path
    if (e == hipSuccess) e = hough::launch_spill(c->g, a, spill, c->spill_wgs, (hipStream_t)stream);
    return e == hipSuccess ? HOUGH_OK : HOUGH_EDEVICE;
}

int hough_run_batch(hough_ctx *c, const float *x, const float *y, const uint32_t *offsets,
                    uint32_t n_events, hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep,
                    uint32_t *status, void *stream) {
    return run_batch_common(c, x, y, offsets, nullptr, nullptr, n_events, peaks, n_peaks, keep,
                            status, stream);
}

int hough_run_batch_relative(hough_ctx *c, const float *x, const float *y, const uint32_t *offsets,
                             uint32_t n_events, uint32_t frac_num, uint32_t frac_den, hough_peak *peaks,
                             uint32_t *n_peaks, uint8_t *keep, uint32_t *status, void *stream) {
    if (frac_den == 0) return HOUGH_EINVAL;
    return run_batch_common(c, x, y, offsets, nullptr, nullptr, n_events, peaks, n_peaks, keep, status, stream,
                            false, nullptr, 0, frac_num, frac_den);
}

int hough_run_batch_gather(hough_ctx *c, const float *x, const float *y, const uint32_t *offsets,
                           const uint32_t *event_ids, const uint32_t *keep_offsets, uint32_t n_events,
                           hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep, uint32_t *status,
                           void *stream) {
    if (n_events && (!event_ids || !keep_offsets)) return HOUGH_EINVAL;
    return run_batch_common(c, x, y, offsets, event_ids, keep_offsets, n_events, peaks, n_peaks,
                            keep, status, stream);
}

uint32_t hough_max_dedup_hits(void) { return hough::kDedupMaxHits; }

size_t hough_split_workspace_bytes(const hough_ctx *c, uint32_t n_events) {
    if (!c || c->fused != 1) return 0;    // the split form spills every event: no workspace
    return hough::split_workspace_bytes(c->p.n_theta, c->p.n_rho, c->plan.groups, n_events);
}

int hough_run_batch_split(hough_ctx *c, const float *x, const float *y, const uint32_t *offsets,
                          const uint32_t *event_ids, const uint32_t *keep_offsets, uint32_t n_events,
                          hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep, uint32_t *status,
                          void *workspace, size_t workspace_bytes, void *stream) {
    if (n_events && ((event_ids == nullptr) != (keep_offsets == nullptr))) return HOUGH_EINVAL;
    if (n_events && !workspace && hough_split_workspace_bytes(c, n_events) > 0) return HOUGH_EINVAL;
    return run_batch_common(c, x, y, offsets, event_ids, keep_offsets, n_events, peaks, n_peaks, keep,
                            status, stream, true, workspace, workspace_bytes);
}

int hough_run_batch_split_static(hough_ctx *c, const float *x, const float *y, const uint32_t *offsets,
                                 const uint32_t *event_ids, const uint32_t *keep_offsets, uint32_t n_events,
                                 hough_peak *peaks, uint32_t *n_peaks, uint8_t *keep, uint32_t *status,
                                 void *stream) {
    if (!c) return HOUGH_EINVAL;
    if (!on_device(c)) return HOUGH_EINVAL;
    if (n_events && ((event_ids == nullptr) != (keep_offsets == nullptr))) return HOUGH_EINVAL;
    const size_t need = hough_split_workspace_bytes(c, n_events);
    if (need > hough::kStaticScratchBytes) return HOUGH_ETOOLARGE;
    void *ws = hough::scratch_ptr(c->device);
    if (!ws) return HOUGH_EDEVICE;
    return run_batch_common(c, x, y, offsets, event_ids, keep_offsets, n_events, peaks, n_peaks, keep,
                            status, stream, true, ws, hough::kStaticScratchBytes);
}

}  // extern "C"
