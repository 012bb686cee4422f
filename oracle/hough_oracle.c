/*
 * CPU oracle for the conformal Hough transform hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into a separate shared library that only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark load.  The product
 * path (the HIP library) never links, loads or calls it, and the two share no code: each
 * builds its own binning tables from the rule stated below.
 *
 * It is deliberately plain: one event at a time, scalar loops in the order the definitions
 * are written, no blocking or reordering.  Floating point follows the stated FP32 rule with
 * explicit fmaf() and is compiled with -ffp-contract=off and without fast-math, so every bin
 * index is the one the rule defines.
 *
 * What is computed, and where it comes from in the paper:
 *   conformal map (Eq. 1):            u = x/(x^2+y^2), v = y/(x^2+y^2)
 *   Hough line map (Sec. II):         rho_ij = u_i cos(theta_j) + v_i sin(theta_j)
 *   uniform discretisation (Sec. II): theta on [0, pi) in n_theta bins, rho on
 *                                     [rho_min, rho_max) in n_rho bins
 *   voting (Sec. II, Sec. III):       acc[j][k] += 1 for every hit i whose rho_ij falls in bin k
 *   peak finding (Sec. II):           threshold plus local-maximum test in the 3x3 neighbourhood
 *   retention (Sec. I, Sec. II):      a hit is kept when it lies within rho_window rho bins of a
 *                                     peak at the peak's own theta
 *
 * Readings of points the paper leaves open (all fixed here and in the HIP library alike):
 *   - theta_j is the lower bin edge, theta_j = (j * pi) / n_theta, evaluated in double.
 *   - A = n_rho / (rho_max - rho_min), B = -rho_min * A (double).  The per-column constants
 *     are C_j = (float)(A cos theta_j), S_j = (float)(A sin theta_j), Bf = (float)B, each
 *     rounded once from double (libm cos/sin).
 *   - a hit is valid iff r2 = fmaf(x, x, y*y) satisfies 0 < r2 <= FLT_MAX; then u = x/r2,
 *     v = y/r2 (IEEE single division, round to nearest).  Invalid hits cast no votes and are
 *     never kept.
 *   - bin rule: w = fmaf(v, S_j, Bf); t = fmaf(u, C_j, w); the vote is in range iff
 *     t >= 0 and t < n_rho (as float), and then k = (int)t.  Out-of-range votes are dropped.
 *   - peak (j,k): acc[j][k] >= threshold, and for every 8-neighbour inside the grid,
 *     acc[j][k] > neighbour if the neighbour precedes (j,k) in raster order (smaller j, or same
 *     j and smaller k), otherwise acc[j][k] >= neighbour.  No wrap of theta (unless the
 *     theta-periodic topology is asked for: oracle_is_peak_periodic).  Peaks are listed
 *     in raster order.
 *   - keep_i iff hit i is valid and some peak (jp,kp) has k_i(jp) in range with
 *     |k_i(jp) - kp| <= rho_window, k_i(jp) computed with the bin rule above.
 *   - the paper's own peak finder (relative threshold, then iterative extraction with
 *     neighbourhood suppression) is oracle_peaks_iterative; its readings are stated there.
 *   - optional duplicate suppression (curlers fire the same wires on every turn): a hit whose
 *     coordinates are bit-identical to an earlier hit of its event casts no votes; retention
 *     still judges every copy by its coordinates (oracle_vote_dedup).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846

/* Binning constants for the uniform (theta, rho) grid of Sec. II. */
int oracle_tables(int n_theta, int n_rho, double rho_min, double rho_max,
                  float *C, float *S, float *Bf)
{
    if (n_theta <= 0 || n_rho <= 0 || !(rho_max > rho_min)) return -1;
    double A = (double)n_rho / (rho_max - rho_min);
    double B = -rho_min * A;
    for (int j = 0; j < n_theta; ++j) {
        double theta = ((double)j * ORACLE_PI) / (double)n_theta;
        C[j] = (float)(A * cos(theta));
        S[j] = (float)(A * sin(theta));
    }
    *Bf = (float)B;
    return 0;
}

/* Eq. (1): conformal map.  Returns 1 for a valid hit, 0 otherwise. */
int oracle_conformal(float x, float y, float *u, float *v)
{
    float y2 = y * y;
    float r2 = fmaf(x, x, y2);
    if (!(r2 > 0.0f && r2 <= FLT_MAX)) { *u = 0.0f; *v = 0.0f; return 0; }
    *u = x / r2;
    *v = y / r2;
    return 1;
}

/* rho = u cos(theta_j) + v sin(theta_j), scaled to bin units and floored.  -1 if out of range. */
int oracle_rho_bin(float u, float v, float Cj, float Sj, float Bf, int n_rho)
{
    float w = fmaf(v, Sj, Bf);
    float t = fmaf(u, Cj, w);
    if (t >= 0.0f && t < (float)n_rho) return (int)t;
    return -1;
}

/* The binned parameter matrix of Sec. III: bins[i*n_theta + j] = bin of rho_ij, or -1 when the
 * hit is invalid or rho_ij falls outside [rho_min, rho_max).  Used by the tests. */
void oracle_bins(int n_theta, int n_rho, const float *C, const float *S, float Bf,
                 const float *x, const float *y, long n_hits, int32_t *bins)
{
    for (long i = 0; i < n_hits; ++i) {
        float u, v;
        int ok = oracle_conformal(x[i], y[i], &u, &v);
        for (int j = 0; j < n_theta; ++j)
            bins[(size_t)i * n_theta + j] = ok ? oracle_rho_bin(u, v, C[j], S[j], Bf, n_rho) : -1;
    }
}

/* Voting: acc[j*n_rho + k] counts the hits whose rho at theta_j falls in bin k. */
void oracle_vote(int n_theta, int n_rho, const float *C, const float *S, float Bf,
                 const float *x, const float *y, long n_hits, int32_t *acc)
{
    memset(acc, 0, sizeof(int32_t) * (size_t)n_theta * (size_t)n_rho);
    for (long i = 0; i < n_hits; ++i) {
        float u, v;
        if (!oracle_conformal(x[i], y[i], &u, &v)) continue;
        for (int j = 0; j < n_theta; ++j) {
            int k = oracle_rho_bin(u, v, C[j], S[j], Bf, n_rho);
            if (k >= 0) acc[(size_t)j * n_rho + k] += 1;
        }
    }
}

/* Duplicate hits (a multi-turn track fires the same wire again): first[i] = 1 iff no earlier
 * hit of the list has bit-identical coordinates, by direct comparison with every earlier hit. */
void oracle_first_copies(const float *x, const float *y, long n_hits, uint8_t *first)
{
    for (long i = 0; i < n_hits; ++i) {
        uint32_t xi, yi;
        memcpy(&xi, &x[i], 4);
        memcpy(&yi, &y[i], 4);
        first[i] = 1;
        for (long j = 0; j < i; ++j) {
            uint32_t xj, yj;
            memcpy(&xj, &x[j], 4);
            memcpy(&yj, &y[j], 4);
            if (xi == xj && yi == yj) { first[i] = 0; break; }
        }
    }
}

/* Voting with each distinct hit counted once: only the first copy of a hit votes. */
void oracle_vote_dedup(int n_theta, int n_rho, const float *C, const float *S, float Bf,
                       const float *x, const float *y, long n_hits, int32_t *acc)
{
    uint8_t *first = (uint8_t *)malloc(n_hits > 0 ? (size_t)n_hits : 1);
    memset(acc, 0, sizeof(int32_t) * (size_t)n_theta * (size_t)n_rho);
    if (!first) return;
    oracle_first_copies(x, y, n_hits, first);
    for (long i = 0; i < n_hits; ++i) {
        float u, v;
        if (!first[i] || !oracle_conformal(x[i], y[i], &u, &v)) continue;
        for (int j = 0; j < n_theta; ++j) {
            int k = oracle_rho_bin(u, v, C[j], S[j], Bf, n_rho);
            if (k >= 0) acc[(size_t)j * n_rho + k] += 1;
        }
    }
    free(first);
}

/* Is cell (j,k) a peak?  Threshold plus the 3x3 local-maximum test with the raster tie rule. */
int oracle_is_peak(const int32_t *acc, int n_theta, int n_rho, int threshold, int j, int k)
{
    int32_t c = acc[(size_t)j * n_rho + k];
    if (c < threshold) return 0;
    for (int dj = -1; dj <= 1; ++dj) {
        for (int dk = -1; dk <= 1; ++dk) {
            if (dj == 0 && dk == 0) continue;
            int jn = j + dj, kn = k + dk;
            if (jn < 0 || jn >= n_theta || kn < 0 || kn >= n_rho) continue;
            int32_t n = acc[(size_t)jn * n_rho + kn];
            int precedes = (dj < 0) || (dj == 0 && dk < 0);
            if (precedes) { if (!(c > n)) return 0; }
            else          { if (!(c >= n)) return 0; }
        }
    }
    return 1;
}

/* The 3x3 test on a theta-periodic grid.  With a symmetric rho range the line (theta + pi, rho)
 * is the line (theta, -rho), so column n_theta - 1 borders column 0 with rho reversed: a
 * neighbour step across that border from (j, k) to row k + dk lands on row n_rho - 1 - (k + dk)
 * of the other edge column.  "Earlier in raster order" compares the neighbour's own (j, k);
 * a cell that reaches itself across the border (n_theta == 1) is skipped. */
int oracle_is_peak_periodic(const int32_t *acc, int n_theta, int n_rho, int threshold, int j, int k)
{
    int32_t c = acc[(size_t)j * n_rho + k];
    if (c < threshold) return 0;
    for (int dj = -1; dj <= 1; ++dj) {
        for (int dk = -1; dk <= 1; ++dk) {
            if (dj == 0 && dk == 0) continue;
            int jn = j + dj, kn = k + dk;
            if (jn < 0) { jn = n_theta - 1; kn = n_rho - 1 - kn; }
            else if (jn >= n_theta) { jn = 0; kn = n_rho - 1 - kn; }
            if (kn < 0 || kn >= n_rho) continue;
            if (jn == j && kn == k) continue;
            int32_t n = acc[(size_t)jn * n_rho + kn];
            int precedes = (jn < j) || (jn == j && kn < k);
            if (precedes) { if (!(c > n)) return 0; }
            else          { if (!(c >= n)) return 0; }
        }
    }
    return 1;
}

long oracle_peaks_mode(const int32_t *acc, int n_theta, int n_rho, int threshold, int periodic,
                       int32_t *pj, int32_t *pk, int32_t *pc, long cap);

/* Peak list in raster order.  Writes at most cap entries, returns the true number of peaks. */
long oracle_peaks(const int32_t *acc, int n_theta, int n_rho, int threshold,
                  int32_t *pj, int32_t *pk, int32_t *pc, long cap)
{
    return oracle_peaks_mode(acc, n_theta, n_rho, threshold, 0, pj, pk, pc, cap);
}

/* The same list with the 3x3 test of either grid topology (periodic != 0: theta-periodic). */
long oracle_peaks_mode(const int32_t *acc, int n_theta, int n_rho, int threshold, int periodic,
                       int32_t *pj, int32_t *pk, int32_t *pc, long cap)
{
    long n = 0;
    for (int j = 0; j < n_theta; ++j)
        for (int k = 0; k < n_rho; ++k)
            if (periodic ? oracle_is_peak_periodic(acc, n_theta, n_rho, threshold, j, k)
                         : oracle_is_peak(acc, n_theta, n_rho, threshold, j, k)) {
                if (n < cap) { pj[n] = j; pk[n] = k; pc[n] = acc[(size_t)j * n_rho + k]; }
                ++n;
            }
    return n;
}

/*
 * Peak finding as Sec. II describes it for multi-track events: a threshold relative to the
 * accumulator's global maximum, then iterative extraction.  The threshold is
 *     thr = max(t_abs, ceil(max_count * frac_num / frac_den))
 * (t_abs >= 1 keeps an empty accumulator from yielding peaks).  Each step takes the largest
 * count among the cells still available and at or above thr, the first in raster order among
 * equal counts; it becomes a peak, and every cell within r_theta columns and r_rho rows of it
 * (inside the grid, no wrap of theta) stops being available.  The steps repeat until no
 * available cell reaches thr.  Peaks are listed in the order they were taken; at most cap are
 * written and the true number is returned (-1 on allocation failure).
 */
long oracle_peaks_iterative(const int32_t *acc, int n_theta, int n_rho, int t_abs,
                            int frac_num, int frac_den, int r_theta, int r_rho,
                            int32_t *pj, int32_t *pk, int32_t *pc, long cap)
{
    const size_t cells = (size_t)n_theta * (size_t)n_rho;
    int32_t max_count = 0;
    for (size_t c = 0; c < cells; ++c)
        if (acc[c] > max_count) max_count = acc[c];
    const int64_t rel = ((int64_t)max_count * frac_num + frac_den - 1) / frac_den;
    const int64_t thr = rel > t_abs ? rel : t_abs;
    uint8_t *gone = (uint8_t *)calloc(cells ? cells : 1, 1);
    if (!gone) return -1;
    long n = 0;
    for (;;) {
        long best = -1;
        int32_t best_count = 0;
        for (size_t c = 0; c < cells; ++c)
            if (!gone[c] && acc[c] >= thr && (best < 0 || acc[c] > best_count)) {
                best = (long)c;
                best_count = acc[c];
            }
        if (best < 0) break;
        const int j = (int)(best / n_rho), k = (int)(best % n_rho);
        if (n < cap) { pj[n] = j; pk[n] = k; pc[n] = best_count; }
        ++n;
        for (int jj = j - r_theta; jj <= j + r_theta; ++jj) {
            if (jj < 0 || jj >= n_theta) continue;
            for (int kk = k - r_rho; kk <= k + r_rho; ++kk)
                if (kk >= 0 && kk < n_rho) gone[(size_t)jj * n_rho + kk] = 1;
        }
    }
    free(gone);
    return n;
}

/*
 * The same extraction as oracle_peaks_iterative in its order form, for accumulators where the
 * step-by-step rescan would take too long (many cells at or above the threshold and many
 * peaks).  The cells at or above the threshold are sorted by count descending, then raster
 * index ascending, and visited in that order: a cell that no earlier peak's window covers
 * becomes a peak and covers its own window.  Step by step, the extraction takes among the cells
 * still available the first one in this order; a cell visited here while covered was covered
 * by a peak taken before it, and a cell never becomes available again, so the two forms take
 * the same cells in the same order.  Arguments and result as for oracle_peaks_iterative.
 */
static int oracle_key_desc(const void *a, const void *b)
{
    const uint64_t ka = *(const uint64_t *)a, kb = *(const uint64_t *)b;
    return ka < kb ? 1 : (ka > kb ? -1 : 0);
}

long oracle_peaks_iterative_sorted(const int32_t *acc, int n_theta, int n_rho, int t_abs,
                                   int frac_num, int frac_den, int r_theta, int r_rho,
                                   int32_t *pj, int32_t *pk, int32_t *pc, long cap)
{
    const size_t cells = (size_t)n_theta * (size_t)n_rho;
    int32_t max_count = 0;
    for (size_t c = 0; c < cells; ++c)
        if (acc[c] > max_count) max_count = acc[c];
    const int64_t rel = ((int64_t)max_count * frac_num + frac_den - 1) / frac_den;
    const int64_t thr = rel > t_abs ? rel : t_abs;
    size_t n_cand = 0;
    for (size_t c = 0; c < cells; ++c)
        if (acc[c] >= thr) ++n_cand;
    /* key: count in the high half, the raster index counted down in the low half */
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (n_cand ? n_cand : 1));
    uint8_t *gone = (uint8_t *)calloc(cells ? cells : 1, 1);
    if (!keys || !gone) { free(keys); free(gone); return -1; }
    size_t m = 0;
    for (size_t c = 0; c < cells; ++c)
        if (acc[c] >= thr) keys[m++] = ((uint64_t)(uint32_t)acc[c] << 32) | (uint64_t)(0xffffffffu - (uint32_t)c);
    qsort(keys, n_cand, sizeof(uint64_t), oracle_key_desc);
    long n = 0;
    for (size_t i = 0; i < n_cand; ++i) {
        const size_t c = 0xffffffffu - (uint32_t)keys[i];
        if (gone[c]) continue;
        const int j = (int)(c / n_rho), k = (int)(c % n_rho);
        if (n < cap) { pj[n] = j; pk[n] = k; pc[n] = acc[c]; }
        ++n;
        for (int jj = j - r_theta; jj <= j + r_theta; ++jj) {
            if (jj < 0 || jj >= n_theta) continue;
            for (int kk = k - r_rho; kk <= k + r_rho; ++kk)
                if (kk >= 0 && kk < n_rho) gone[(size_t)jj * n_rho + kk] = 1;
        }
    }
    free(keys);
    free(gone);
    return n;
}

/* Retention mask: keep_i = 1 iff hit i is within rho_window bins of a peak at the peak's theta. */
void oracle_retain(int n_rho, const float *C, const float *S, float Bf, int rho_window,
                   const float *x, const float *y, long n_hits,
                   const int32_t *pj, const int32_t *pk, long n_peaks, uint8_t *keep)
{
    for (long i = 0; i < n_hits; ++i) {
        float u, v;
        keep[i] = 0;
        if (!oracle_conformal(x[i], y[i], &u, &v)) continue;
        for (long p = 0; p < n_peaks; ++p) {
            int k = oracle_rho_bin(u, v, C[pj[p]], S[pj[p]], Bf, n_rho);
            if (k < 0) continue;
            int d = k - pk[p];
            if (d < 0) d = -d;
            if (d <= rho_window) { keep[i] = 1; break; }
        }
    }
}

/*
 * Candidate circles and track parameters of peaks (Sec. II, Eq. (2) read with the factor two
 * that Eq. (1) implies).  The line u cos(theta) + v sin(theta) = rho of the conformal plane is
 * the circle through the origin with centre (cos theta, sin theta) / (2 rho) and radius
 * 1 / (2 |rho|).  A peak (j, k) stands for theta_j = j pi / n_theta (the column's own angle)
 * and the centre of rho bin k, rho = rho_min + (k + 1/2) (rho_max - rho_min) / n_rho.
 * Transverse momentum: p_T [GeV/c] = 0.299792458 * B [T] * R [m].
 * The peak's hits are those the retention rule associates with it alone (|k_i(j) - k| <=
 * rho_window at the peak's column).  A track starting at the origin runs along the half of the
 * circle on one side of the line from the origin through the centre; its charge is +1 when
 * more of those hits lie counter-clockwise of that line than clockwise (side test
 * C_j y - S_j x, times the sign of rho, in float with one fma), -1 in the opposite case and 0 on
 * a tie.  The direction at the origin is phi0 = phi_c + q pi / 2, phi_c = atan2(b, a).
 * out[7 * p + ...] = {a, b, R, pT, phi_c, q, n_hits} as doubles.
 */
void oracle_track_params(int n_theta, int n_rho, double rho_min, double rho_max, const float *C,
                         const float *S, float Bf, int rho_window, double b_tesla,
                         const float *x, const float *y, long n_hits,
                         const int32_t *pj, const int32_t *pk, long n_peaks, double *out)
{
    const double pi = 3.14159265358979323846;
    const double drho = (rho_max - rho_min) / (double)n_rho;
    for (long p = 0; p < n_peaks; ++p) {
        const int j = pj[p], k = pk[p];
        const double theta = ((double)j * pi) / (double)n_theta;
        const double rho = rho_min + ((double)k + 0.5) * drho;
        const double a = cos(theta) / (2.0 * rho), b = sin(theta) / (2.0 * rho);
        const double R = 1.0 / (2.0 * fabs(rho));
        long ccw = 0, cw = 0, n = 0;
        for (long i = 0; i < n_hits; ++i) {
            float u, v;
            if (!oracle_conformal(x[i], y[i], &u, &v)) continue;
            const int ki = oracle_rho_bin(u, v, C[j], S[j], Bf, n_rho);
            if (ki < 0) continue;
            const int d = ki > k ? ki - k : k - ki;
            if (d > rho_window) continue;
            ++n;
            float side = fmaf(C[j], y[i], -(S[j] * x[i]));
            if (rho < 0.0) side = -side;
            if (side > 0.0f) ++ccw;
            else if (side < 0.0f) ++cw;
        }
        double *o = out + 7 * p;
        o[0] = a;
        o[1] = b;
        o[2] = R;
        o[3] = 0.299792458 * b_tesla * R * 1e-3;
        o[4] = atan2(b, a);
        o[5] = (double)(ccw > cw ? 1 : (ccw < cw ? -1 : 0));
        o[6] = (double)n;
    }
}

/*
 * Whole hot path over CSR-packed events: per event vote, find all peaks, keep hits near any
 * of them, and return the first `cap` peaks of each event (raster order) with the true count.
 * dedup != 0: only the first copy of bit-identical hits votes (every copy is still retained or
 * not by its coordinates).  frac_den > 0: each event's threshold is
 * max(threshold, ceil(its largest count * frac_num / frac_den)), the relative form of Sec. II.
 * Events are independent (Sec. III), so they are spread over n_threads OpenMP threads; each
 * event is still computed by the plain single-event routines above.
 * peaks_out holds cap triples (j, k, count) per event.  Returns 0, or -1 on allocation failure.
 */
int oracle_run_batch(int n_theta, int n_rho, double rho_min, double rho_max, int threshold,
                     int rho_window, const float *x, const float *y, const uint32_t *offsets,
                     long n_events, long cap, int32_t *peaks_out, int64_t *n_peaks_out,
                     uint8_t *keep, int n_threads, int periodic, int dedup, int frac_num, int frac_den)
{
    float *C = (float *)malloc(sizeof(float) * (size_t)n_theta);
    float *S = (float *)malloc(sizeof(float) * (size_t)n_theta);
    float Bf;
    int failed = 0;
    if (!C || !S || oracle_tables(n_theta, n_rho, rho_min, rho_max, C, S, &Bf) != 0) {
        free(C); free(S); return -1;
    }
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
    for (long e = 0; e < n_events; ++e) {
        long a = offsets[e], h = (long)offsets[e + 1] - (long)offsets[e];
        long max_p = (long)n_theta * n_rho;
        int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * (size_t)max_p);
        int32_t *pj = (int32_t *)malloc(sizeof(int32_t) * (size_t)max_p);
        int32_t *pk = (int32_t *)malloc(sizeof(int32_t) * (size_t)max_p);
        int32_t *pc = (int32_t *)malloc(sizeof(int32_t) * (size_t)max_p);
        if (!acc || !pj || !pk || !pc) {
#pragma omp atomic write
            failed = 1;
        } else {
            if (dedup)
                oracle_vote_dedup(n_theta, n_rho, C, S, Bf, x + a, y + a, h, acc);
            else
                oracle_vote(n_theta, n_rho, C, S, Bf, x + a, y + a, h, acc);
            int thr = threshold;
            if (frac_den > 0) {            /* relative threshold: max(T, ceil(max * num / den)) */
                int32_t mx = 0;
                for (long c = 0; c < max_p; ++c)
                    if (acc[c] > mx) mx = acc[c];
                const int64_t rel = ((int64_t)mx * frac_num + frac_den - 1) / frac_den;
                thr = rel > thr ? (int)(rel > 0x7fffffff ? 0x7fffffff : rel) : thr;
            }
            long np = oracle_peaks_mode(acc, n_theta, n_rho, thr, periodic, pj, pk, pc, max_p);
            oracle_retain(n_rho, C, S, Bf, rho_window, x + a, y + a, h, pj, pk, np, keep + a);
            n_peaks_out[e] = np;
            for (long p = 0; p < np && p < cap; ++p) {
                peaks_out[(e * cap + p) * 3 + 0] = pj[p];
                peaks_out[(e * cap + p) * 3 + 1] = pk[p];
                peaks_out[(e * cap + p) * 3 + 2] = pc[p];
            }
        }
        free(acc); free(pj); free(pk); free(pc);
    }
    free(C); free(S);
    return failed ? -1 : 0;
}

/*
 * The paper's finder over CSR-packed events, one event at a time: vote (only first copies of
 * duplicate hits with dedup != 0), the iterative extraction in its order form
 * (oracle_peaks_iterative_sorted), then retention against the event's first min(n, cap) peaks
 * (the peaks a caller receives).  Events are independent, so they are spread over n_threads
 * OpenMP threads.  peaks_out holds cap triples (j, k, count) per event in extraction order;
 * n_peaks_out the true counts.  Returns 0, or -1 on allocation failure.
 */
int oracle_run_batch_iterative(int n_theta, int n_rho, double rho_min, double rho_max, int t_abs,
                               int frac_num, int frac_den, int r_theta, int r_rho, int rho_window,
                               const float *x, const float *y, const uint32_t *offsets, long n_events,
                               long cap, int32_t *peaks_out, int64_t *n_peaks_out, uint8_t *keep,
                               int n_threads, int dedup)
{
    float *C = (float *)malloc(sizeof(float) * (size_t)n_theta);
    float *S = (float *)malloc(sizeof(float) * (size_t)n_theta);
    float Bf;
    int failed = 0;
    if (!C || !S || oracle_tables(n_theta, n_rho, rho_min, rho_max, C, S, &Bf) != 0) {
        free(C); free(S); return -1;
    }
    if (n_threads < 1) n_threads = 1;
    const long room = cap > 0 ? cap : 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
    for (long e = 0; e < n_events; ++e) {
        long a = offsets[e], h = (long)offsets[e + 1] - (long)offsets[e];
        int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_theta * (size_t)n_rho);
        int32_t *pj = (int32_t *)malloc(sizeof(int32_t) * (size_t)room);
        int32_t *pk = (int32_t *)malloc(sizeof(int32_t) * (size_t)room);
        int32_t *pc = (int32_t *)malloc(sizeof(int32_t) * (size_t)room);
        if (!acc || !pj || !pk || !pc) {
#pragma omp atomic write
            failed = 1;
        } else {
            if (dedup)
                oracle_vote_dedup(n_theta, n_rho, C, S, Bf, x + a, y + a, h, acc);
            else
                oracle_vote(n_theta, n_rho, C, S, Bf, x + a, y + a, h, acc);
            long np = oracle_peaks_iterative_sorted(acc, n_theta, n_rho, t_abs, frac_num, frac_den, r_theta,
                                                    r_rho, pj, pk, pc, cap);
            if (np < 0) {
#pragma omp atomic write
                failed = 1;
                np = 0;
            }
            const long listed = np < cap ? np : cap;
            oracle_retain(n_rho, C, S, Bf, rho_window, x + a, y + a, h, pj, pk, listed, keep + a);
            n_peaks_out[e] = np;
            for (long p = 0; p < listed; ++p) {
                peaks_out[(e * cap + p) * 3 + 0] = pj[p];
                peaks_out[(e * cap + p) * 3 + 1] = pk[p];
                peaks_out[(e * cap + p) * 3 + 2] = pc[p];
            }
        }
        free(acc); free(pj); free(pk); free(pc);
    }
    free(C); free(S);
    return failed ? -1 : 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
