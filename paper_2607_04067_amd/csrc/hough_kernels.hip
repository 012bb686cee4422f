// HIP kernels of libhough.so (gfx950 / CDNA4, wave64).
//
// Layout shared by every kernel that votes: a theta tile of TW = 64*G columns lives in LDS
// rho-major, one row of the tile per rho bin, two 16-bit counters per dword (see Lane below).
// Lane l of a wave owns column c = 64*q + l of group q, so the 64 atomics one ds_add_u32
// issues for one hit land in 32 consecutive dwords of one row, the two lanes of a dword in
// different halves of the wave: no bank conflict, never the same address.  Hits are
// wave-uniform: a wave maps 64 hits at a time (one per lane), compacts the valid ones into a
// per-wave LDS stage with ballot/mbcnt, then every lane sweeps its own column over the staged
// hits (the theta sweep of Sec. III: one column = one parallel task, hits streamed through it).
//
// Row n_rho of the tile is a dummy row: lanes whose column lies outside [0, n_theta) carry
// C = S = 0 and B = n_rho, so they "vote" there instead of taking a branch per vote.
//
// Floating point: the bin of a hit in a column is t = fma(u, C_j, fma(v, S_j, B)) with
// k = (int)t, exactly as the C-ABI header states.  Hits whose votes are provably all in range
// (|rho| bounded by sqrt(u^2+v^2) with slack for rounding) skip the range test; the others take
// the literal test 0 <= t < n_rho.
#include <float.h>

#include <algorithm>
#include <type_traits>

#include "hough_internal.h"

namespace hough {
namespace {

constexpr int kStageBytes = kWave * (int)sizeof(float2);

// ------------------------------------------------------------------ per-hit arithmetic
// Eq. (1).  Returns false for a hit whose r2 is zero, non-finite or overflowed.
__device__ __forceinline__ bool conformal(float x, float y, float &u, float &v) {
    const float y2 = y * y;
    const float r2 = __builtin_fmaf(x, x, y2);
    const bool ok = (r2 > 0.0f) && (r2 <= FLT_MAX);
    const float d = ok ? r2 : 1.0f;
    u = x / d;
    v = y / d;
    return ok;
}

// The validity part of the map alone (no division).
__device__ __forceinline__ bool valid_hit(float x, float y) {
    const float r2 = __builtin_fmaf(x, x, y * y);
    return (r2 > 0.0f) && (r2 <= FLT_MAX);
}

// True when every column's t lies strictly inside (0, n_rho).  |rho| <= sqrt(u^2 + v^2) for
// every theta, so u^2 + v^2 below safe_r2 (set on the host with slack for the rounding of this
// sum and of t) keeps every vote of the hit in range.
__device__ __forceinline__ bool all_in_range(float u, float v, const GridArgs &g) {
    return __builtin_fmaf(u, u, v * v) < g.safe_r2;
}

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void lds_add(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-lane constants of the columns a lane owns in the current tile.  On a theta-periodic grid
// the halo column left of column 0 is column n_theta - 1 and the one right of column
// n_theta - 1 is column 0, both with rho reversed: such a lane votes with that column's own
// constants into row n_rho - 1 - k, i.e. with a negative row stride from the top row (rs, rb:
// row stride and base in bytes, used only by the periodic kernels).
template <int G>
struct Cols {
    float C[G], S[G], B[G];
    int rs[G], rb[G];
};

template <int G, bool PER = false>
__device__ __forceinline__ Cols<G> load_cols(const GridArgs &g, int first_col, int lane, int stride,
                                             const uint32_t *col, float dummy_row = -1.0f) {
    Cols<G> cl;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const int j = first_col + 64 * q + lane;
        const bool in = (j >= 0) && (j < g.n_theta);
        const bool wrap = PER && (j == -1 || j == g.n_theta);
        const int jw = j < 0 ? g.n_theta - 1 : 0;
        cl.C[q] = in ? g.C[j] : (wrap ? g.C[jw] : 0.0f);
        cl.S[q] = in ? g.S[j] : (wrap ? g.S[jw] : 0.0f);
        // out-of-grid lanes land in the dummy row (row n_rho, or the row a windowed tile gives it)
        cl.B[q] = (in || wrap) ? g.Bf : (dummy_row >= 0.0f ? dummy_row : g.nrho_f);
        cl.rs[q] = 4 * (wrap ? -stride : stride);                                    // bytes
        cl.rb[q] = 4 * (wrap ? (g.n_rho - 1) * stride + (int)col[q] : (int)col[q]);
    }
    return cl;
}

// Where a lane's cells live in a tile row.  Unpacked: one 32-bit counter per cell, column
// 64q + l at dword 64q + l.  Packed: two 16-bit counters per dword, columns 64q + l and
// 64q + l + 32 (l < 32) share dword 32q + l; the two lanes sharing a dword sit in different
// halves of the wave, which the LDS serves in separate passes, so they never conflict.
template <int G, bool PACKED>
struct Lane {
    static constexpr int TW = 64 * G;
    static constexpr int STRIDE = PACKED ? TW / 2 : TW;    // dwords per tile row
    uint32_t col[G];
    uint32_t shift, inc, cmask;
    __device__ __forceinline__ explicit Lane(int lane) {
#pragma unroll
        for (int q = 0; q < G; ++q) col[q] = PACKED ? 32 * q + (lane & 31) : 64 * q + lane;
        shift = PACKED ? 16u * (uint32_t)(lane >> 5) : 0u;
        inc = 1u << shift;
        cmask = PACKED ? 0xffffu : ~0u;
    }
    __device__ __forceinline__ uint32_t count(uint32_t dword) const { return (dword >> shift) & cmask; }
};

// Map up to 64 hits [base, end) (one per lane) and compact the valid ones into the wave's
// stage: all-in-range hits first, then the others.  Returns (n_safe, n_total) and, through
// `bad`, whether this lane met an invalid hit, through `slot` the stage slot of the lane's hit
// (-1 if none).  `skip` hides hits the caller is done with.
struct StageCount { uint32_t safe, total; };

// Stage the lane's hit (xi, yi) when `in`.
__device__ __forceinline__ StageCount stage_values(float2 *st, float xi, float yi,
                                                   bool in, const GridArgs &g,
                                                   uint32_t &bad, int &slot) {
    float u, v;
    const bool ok = conformal(in ? xi : 0.0f, in ? yi : 0.0f, u, v);
    const bool valid = in && ok;
    if (in && !ok) bad = 1u;
    const bool safe = valid && all_in_range(u, v, g);
    const uint64_t bs = __ballot(safe);
    const uint64_t bu = __ballot(valid && !safe);
    const uint32_t ns = (uint32_t)__popcll(bs);
    const uint32_t pos = safe ? mbcnt(bs) : ns + mbcnt(bu);
    if (valid) st[pos] = make_float2(u, v);
    slot = valid ? (int)pos : -1;
    wave_sync();
    return StageCount{ns, ns + (uint32_t)__popcll(bu)};
}

__device__ __forceinline__ StageCount stage_hits(float2 *st, const float *x,
                                                 const float *y, uint32_t base, uint32_t end,
                                                 bool skip, const GridArgs &g, int lane,
                                                 uint32_t &bad, int &slot) {
    const uint32_t i = base + lane;
    const bool in = (i < end) && !skip;
    float xi = 0.0f, yi = 0.0f;
    if (in) { xi = x[i]; yi = y[i]; }
    return stage_values(st, xi, yi, in, g, bad, slot);
}

// Steps 2-3: sweep one staged hit through the lane's columns and vote.
// The lane's cell of row k in group q.  Periodic kernels use the per-lane row stride (a 24-bit
// multiply-add, full rate) so that the reversed halo lanes need no other instruction.
template <int G, bool P, bool PER = false>
__device__ __forceinline__ uint32_t *cell_of(uint32_t *tile, int k, const Cols<G> &cl, const Lane<G, P> &ln,
                                             int q) {
    if (PER)
        return reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(tile) + (__mul24(k, cl.rs[q]) + cl.rb[q]));
    return &tile[k * Lane<G, P>::STRIDE + (int)ln.col[q]];
}

template <int G, bool P, bool PER = false>
__device__ __forceinline__ void vote1(uint32_t *tile, float u, float v, const Cols<G> &cl,
                                      const Lane<G, P> &ln) {
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const float w = __builtin_fmaf(v, cl.S[q], cl.B[q]);
        const float t = __builtin_fmaf(u, cl.C[q], w);
        lds_add(cell_of<G, P, PER>(tile, (int)t, cl, ln, q), ln.inc);
    }
}

// Four staged hits, one vote each per column.
template <int G, bool P, bool PER = false>
__device__ __forceinline__ void vote4(uint32_t *tile, const float4 &a, const float4 &b,
                                      const Cols<G> &cl, const Lane<G, P> &ln) {
    vote1<G, P, PER>(tile, a.x, a.y, cl, ln);
    vote1<G, P, PER>(tile, a.z, a.w, cl, ln);
    vote1<G, P, PER>(tile, b.x, b.y, cl, ln);
    vote1<G, P, PER>(tile, b.z, b.w, cl, ln);
}

// Wait for every outstanding LDS operation of the wave (lgkmcnt(0), other counters untouched).
__device__ __forceinline__ void lds_wait() { __builtin_amdgcn_s_waitcnt(0xc07f); }

// Keep the compiler's scheduler from moving instructions across this point.
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// The staged hits are read four at a time (two 16-byte broadcast reads), one group ahead of
// the votes that use them, alternating between two register sets.  The read of group c + 1 is
// issued before the atomics of group c, and LDS operations complete in order, so the votes of
// group c + 1 wait only for operations issued before the atomics of group c: a wave never
// waits for its latest atomics.  The fences keep the compiler from reordering the groups.
template <int G, bool P, bool PER = false>
__device__ __forceinline__ void vote_staged(uint32_t *tile, const float2 *st, StageCount n,
                                            const Cols<G> &cl, const Lane<G, P> &ln, float nrho_f) {
    const float4 *st4 = reinterpret_cast<const float4 *>(st);
    const uint32_t n4 = n.safe >> 2;
    if (n4) {
        float4 a0 = st4[0], b0 = st4[1];
        lds_wait();
        uint32_t c = 0;
        for (; c + 2 < n4; c += 2) {
            const float4 a1 = st4[2 * c + 2], b1 = st4[2 * c + 3];
            sched_fence();
            vote4<G, P, PER>(tile, a0, b0, cl, ln);
            sched_fence();
            a0 = st4[2 * c + 4];
            b0 = st4[2 * c + 5];
            sched_fence();
            vote4<G, P, PER>(tile, a1, b1, cl, ln);
            sched_fence();
        }
        vote4<G, P, PER>(tile, a0, b0, cl, ln);
        if (c + 1 < n4) {
            const float4 a1 = st4[2 * c + 2], b1 = st4[2 * c + 3];
            vote4<G, P, PER>(tile, a1, b1, cl, ln);
        }
    }
    for (uint32_t h = n4 * 4; h < n.safe; ++h) vote1<G, P, PER>(tile, st[h].x, st[h].y, cl, ln);
    for (uint32_t h = n.safe; h < n.total; ++h) {
        const float2 p = st[h];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const float w = __builtin_fmaf(p.y, cl.S[q], cl.B[q]);
            const float t = __builtin_fmaf(p.x, cl.C[q], w);
            if (t >= 0.0f && t < nrho_f) lds_add(cell_of<G, P, PER>(tile, (int)t, cl, ln, q), ln.inc);
        }
    }
}

// Votes of hits [hb, he); returns the number of valid hits seen.  The next 64 hits are loaded
// while the current ones vote.  dup (duplicate suppression, else null): the event's keep bytes
// as the duplicate pass left them; a later copy of a hit is counted as valid but not staged.
template <int G, bool P, bool PER = false>
__device__ uint32_t vote_range(uint32_t *tile, float2 *st, const float *x, const float *y,
                               uint32_t hb, uint32_t he, const Cols<G> &cl, const Lane<G, P> &ln,
                               const GridArgs &g, int lane, uint32_t &bad, const uint8_t *dup = nullptr) {
    uint32_t n_valid = 0;
    float xn = 0.0f, yn = 0.0f;
    if (hb + lane < he) { xn = x[hb + lane]; yn = y[hb + lane]; }
    for (uint32_t base = hb; base < he; base += 64) {
        const uint32_t i = base + lane;
        const float xi = xn, yi = yn;
        if (i + 64 < he) { xn = x[i + 64]; yn = y[i + 64]; }
        bool live = i < he;
        if (dup) {
            const bool copy = live && (dup[i] & kKeepDuplicate) != 0;
            n_valid += (uint32_t)__popcll(__ballot(copy && valid_hit(xi, yi)));
            live = live && !copy;
        }
        int slot;
        const StageCount n = stage_values(st, xi, yi, live, g, bad, slot);
        n_valid += n.total;
        vote_staged<G, P, PER>(tile, st, n, cl, ln, g.nrho_f);
        wave_sync();
    }
    return n_valid;
}

// Step 4 on rows [16*u, 16*u + 16) of the lane's columns: bit b of mask[q] is set iff cell
// (column 64q + lane, row 16*u + b) is a peak.  Raster order is (theta, rho), so the column to
// the left and the row above come first:
//   peak <=> count >= threshold, count > every earlier neighbour, count >= every later one
//        <=> count >= max(threshold, max(earlier) + 1, max(later)).
// The lane slides a three-row window down its own column, reading four rows at a time; the
// vertical maxima of the neighbouring columns come from the neighbouring lanes through DPP wave
// shifts (and across a 64-column group boundary through readlane).  Rows outside the grid count
// as 0.  The two edge columns of the tile are halo columns; the caller drops their bits.
constexpr int kPeakRows = 16;

// Count of cell (row k, column of group q) or 0 outside the grid's rows.  Row k is the same for
// every lane.  Interior units (CHECK false) never leave the grid; at the edges the address is
// clamped into the tile so that the read is unconditional and only its value is dropped.
template <bool CHECK, int G, bool P>
__device__ __forceinline__ uint32_t cell_or_zero(const uint32_t *tile, int k, int n_rho,
                                                 const Lane<G, P> &ln, int q) {
    if (!CHECK) return ln.count(tile[k * Lane<G, P>::STRIDE + ln.col[q]]);
    const int kk = min(max(k, 0), n_rho);
    const uint32_t d = tile[kk * Lane<G, P>::STRIDE + ln.col[q]];
    return (k >= 0 && k < n_rho) ? ln.count(d) : 0u;
}

// WRAP (theta-periodic grid, first and last tile): the halo column beside column 0 is column
// n_theta - 1 and follows it in raster order, the one beside column n_theta - 1 is column 0 and
// precedes it, so for those two lanes the strict and the non-strict side trade places.
// UNROLL: issue the reads of all four 4-row blocks together (for kernels with the registers).
template <bool CHECK, int G, bool P, bool WRAP = false, bool UNROLL = false>
__device__ __forceinline__ void peak_rows(const uint32_t *tile, int unit, int n_rho, uint32_t T,
                                          const Lane<G, P> &ln, int lane, uint32_t *mask,
                                          int first_col = 0, int n_theta = 0) {
    const int k0 = unit * kPeakRows;
    uint32_t Mp[G], Mc[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        Mp[q] = cell_or_zero<CHECK, G, P>(tile, k0 - 1, n_rho, ln, q);
        Mc[q] = cell_or_zero<CHECK, G, P>(tile, k0, n_rho, ln, q);
        mask[q] = 0u;
    }
    auto block = [&](int r0) {
        uint32_t N[G][4];
#pragma unroll
        for (int d = 0; d < 4; ++d)
#pragma unroll
            for (int q = 0; q < G; ++q) N[q][d] = cell_or_zero<CHECK, G, P>(tile, k0 + r0 + d + 1, n_rho, ln, q);
        // rows r0 .. r0+3 are tested; when no lane's count there reaches the threshold none of
        // them can be a peak and only the window moves on
        uint32_t bm = 0;
#pragma unroll
        for (int q = 0; q < G; ++q) bm = max(bm, max(max(Mc[q], N[q][0]), max(N[q][1], N[q][2])));
        if (__ballot(bm >= T) == 0ull) {
#pragma unroll
            for (int q = 0; q < G; ++q) { Mp[q] = N[q][2]; Mc[q] = N[q][3]; }
            return;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int k = k0 + r0 + d;
            uint32_t V[G];
#pragma unroll
            for (int q = 0; q < G; ++q) V[q] = max(max(Mp[q], Mc[q]), N[q][d]);
#pragma unroll
            for (int q = 0; q < G; ++q) {
                uint32_t VL = __builtin_amdgcn_update_dpp(0u, V[q], 0x138, 0xf, 0xf, true);   // lane - 1
                uint32_t VR = __builtin_amdgcn_update_dpp(0u, V[q], 0x130, 0xf, 0xf, true);   // lane + 1
                if (q > 0) {
                    const uint32_t x = __builtin_amdgcn_readlane(V[q > 0 ? q - 1 : 0], 63);
                    VL = lane == 0 ? x : VL;
                }
                if (q + 1 < G) {
                    const uint32_t x = __builtin_amdgcn_readlane(V[q + 1 < G ? q + 1 : 0], 0);
                    VR = lane == 63 ? x : VR;
                }
                uint32_t before, after;
                if (WRAP) {
                    const int j = first_col + 64 * q + lane;
                    const bool wl = j == 0, wr = j == n_theta - 1;
                    before = max(max(wl ? 0u : VL, wr ? VR : 0u), Mp[q]);
                    after = max(max(wl ? VL : 0u, wr ? 0u : VR), N[q][d]);
                } else {
                    before = max(VL, Mp[q]);
                    after = max(VR, N[q][d]);
                }
                const uint32_t need = max(max(T, before + 1u), after);
                mask[q] |= (uint32_t)((!CHECK || k < n_rho) && Mc[q] >= need) << (r0 + d);
            }
#pragma unroll
            for (int q = 0; q < G; ++q) { Mp[q] = Mc[q]; Mc[q] = N[q][d]; }
        }
    };
    if constexpr (UNROLL) {
#pragma unroll
        for (int r0 = 0; r0 < kPeakRows; r0 += 4) block(r0);
    } else {
#pragma unroll 1
        for (int r0 = 0; r0 < kPeakRows; r0 += 4) block(r0);
    }
}

// True when no count of the 16-row unit `unit` reaches T (then it holds no peak).  The unit's
// rows are contiguous in the packed tile, so the wave reads them whole, 16 bytes per lane per
// read, and takes the maximum of each lane's 16-bit counts: a few instructions where the 3x3
// test reads and compares every row.
template <int G>
__device__ __forceinline__ bool unit_below(const uint32_t *tile, int unit, uint32_t T, int lane) {
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    constexpr int ST = Lane<G, true>::STRIDE, READS = ST * kPeakRows / 4 / 64;
    const uint4 *p = reinterpret_cast<const uint4 *>(tile + unit * kPeakRows * ST) + lane;
    u16x2 m = {0, 0};
#pragma unroll
    for (int i = 0; i < READS; ++i) {
        const uint4 v = p[64 * i];
        const u16x2 a = __builtin_elementwise_max(__builtin_bit_cast(u16x2, v.x), __builtin_bit_cast(u16x2, v.y));
        const u16x2 b = __builtin_elementwise_max(__builtin_bit_cast(u16x2, v.z), __builtin_bit_cast(u16x2, v.w));
        m = __builtin_elementwise_max(m, __builtin_elementwise_max(a, b));
    }
    const uint32_t mx = max((uint32_t)m.x, (uint32_t)m.y);
    return __ballot(mx >= T) == 0ull;
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row broadcasts (no LDS).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int) {
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
    return v;
}

__device__ __forceinline__ void store_peak(hough_peak *out, uint32_t j, uint32_t k, uint32_t c) {
    uint2 *p = reinterpret_cast<uint2 *>(out);
    *p = make_uint2((j & 0xffffu) | (k << 16), c);
}

// Step 4 (listing) and the retention marks of step 5, shared by all waves.  pmask[wd * TW + c]
// holds the peak bits of column c, rows 32*wd ...  Every wave computes the per-column peak
// counts and their prefix over the tile's columns (raster order is column-major), then lists
// the peaks of its own words at base + (peaks in earlier columns) + (peaks above in the same
// column).  It also writes the dilated words dil[wd * TW + c]: bit b set iff a peak of column c
// lies within rho_window rows of row 32*wd + b.  For rho_window < 32 a word follows from the
// peak words above and below it; wider windows OR the row range of every peak into dil (which
// the peak phase cleared).  colcnt (optional): each column's peak count, summed by the peak
// phase (else counted here from pmask).  tpk (optional): when the tile has at most kTilePeaks peaks, all of
// them in raster order, each with its column's C and S (and its row as the bits of z), for the
// retention of tiles with few peaks.  Returns the tile's peak count.
constexpr uint32_t kTilePeaks = 64;
// Deferred retention (sparse-grid kernels): a tile with at most kDeferTilePeaks peaks, all of
// them in the caller's peak list, leaves its retention to a later pass over the event's hits
// against the peak list itself, which then covers up to kDeferPeaks peaks of several tiles.
constexpr uint32_t kDeferTilePeaks = 80;
constexpr uint32_t kDeferPeaks = 256;

template <int G, bool P>
__device__ uint32_t emit_and_dilate(const uint32_t *tile, const uint32_t *pmask, uint32_t *dil, int w0,
                                    int nwords, int first_col, const GridArgs &g, hough_peak *out,
                                    uint32_t cap, uint32_t base, const Lane<G, P> &ln, int lane,
                                    int wave, int n_waves, float4 *tpk = nullptr,
                                    const Cols<G> *cl = nullptr, const uint32_t *colcnt = nullptr,
                                    uint32_t *edge = nullptr) {
    constexpr int TW = 64 * G, ST = Lane<G, P>::STRIDE;
    const int W = g.rho_window;
    uint32_t colbase[G];
    uint32_t carry = 0;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        uint32_t tot = 0;
        if (colcnt)
            tot = colcnt[64 * q + lane];
        else
            for (int w = w0; w < w0 + nwords; ++w) tot += __popc(pmask[w * TW + 64 * q + lane]);
        const uint32_t incl = wave_inclusive_scan(tot, lane);
        colbase[q] = carry + incl - tot;
        carry += __shfl(incl, 63, 64);
    }
    if (carry == 0u) return 0u;
    const bool rec = tpk != nullptr && carry <= kTilePeaks;   // then every local index fits
    const int w1 = w0 + nwords;
    for (int wd = w0 + wave; wd < w1; wd += n_waves) {
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int c = 64 * q + lane;
            uint32_t m = pmask[wd * TW + c];
            if (W < 32) {
                const uint32_t up = wd > w0 ? pmask[(wd - 1) * TW + c] : 0u;
                const uint32_t dn = wd + 1 < w1 ? pmask[(wd + 1) * TW + c] : 0u;
                uint32_t d = m;
                for (int sft = 1; sft <= W; ++sft)
                    d |= (m << sft) | (m >> sft) | (up >> (32 - sft)) | (dn << (32 - sft));
                dil[wd * TW + c] = d;
            }
            if (!m) continue;
            uint32_t idx = base + colbase[q];
            for (int w = w0; w < wd; ++w) idx += __popc(pmask[w * TW + c]);
            const uint32_t j = (uint32_t)(first_col + c);
            while (m) {
                const int b = __builtin_ctz(m);
                m &= m - 1u;
                const int k = wd * 32 + b;
                const uint32_t cv = ln.count(tile[k * ST + ln.col[q]]);
                if (idx < cap) store_peak(out + idx, j, (uint32_t)k, cv);
                if (rec) {
                    tpk[idx - base] = make_float4(cl->C[q], cl->S[q], __int_as_float(k - W), 0.0f);
                    if (edge && (k <= W || k >= g.n_rho - W)) *edge = 1u;
                }
                ++idx;
                if (W >= 32) {
                    const int lo = k - W > 0 ? k - W : 0;
                    const int hi = k + W < g.n_rho - 1 ? k + W : g.n_rho - 1;
                    // words outside [w0, w1) hold rows no hit of the event reaches
                    for (int w = max(lo >> 5, w0); w <= min(hi >> 5, w1 - 1); ++w) {
                        const int a = max(lo, w * 32) - w * 32, e = min(hi, w * 32 + 31) - w * 32;
                        const uint32_t rm = (e == 31 ? ~0u : ((1u << (e + 1)) - 1u)) & ~((1u << a) - 1u);
                        __hip_atomic_fetch_or(&dil[w * TW + c], rm, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            }
        }
    }
    return carry;
}

// Step 5 on the current tile: a hit is kept when its own cell in some column of the tile has
// its dil bit set.  Returns bit 0 set iff kept.
template <int G>
__device__ __forceinline__ uint32_t lookup1(const uint32_t *dil, float u, float v, bool checked,
                                            const Cols<G> &cl, int lane, float nrho_f) {
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const float w = __builtin_fmaf(v, cl.S[q], cl.B[q]);
        const float t = __builtin_fmaf(u, cl.C[q], w);
        if (!checked || (t >= 0.0f && t < nrho_f)) {
            const uint32_t k = (uint32_t)(int)t;
            // word k / 32 of the column (a shift and one shift-add: the empty asm keeps the
            // compiler from turning the pair into shift, mask and add), then bit k mod 32 (the
            // bit-field extract takes its offset modulo 32)
            uint32_t kw = k >> 5;
            asm("" : "+v"(kw));
            m |= __builtin_amdgcn_ubfe(dil[kw * (64u * G) + 64u * q + (uint32_t)lane], k, 1u);
        }
    }
    return m;
}

// OR over the 64 lanes (DPP row shifts and row broadcasts, no LDS), returned wave-uniform.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Look up the staged hits st[0 .. n.total) (the first n.safe need no range test), four at a
// time so that their reads are in flight together.  Each lane gathers its own column's verdicts
// as bits (hit h at bit h mod 32 of one of two words) and one OR across the wave at the end
// turns them into the mask of kept stage slots.
template <int G>
__device__ __forceinline__ uint64_t lookup_staged(const uint32_t *dil, const float2 *st, StageCount n,
                                                  const Cols<G> &cl, int lane, float nrho_f) {
    const float4 *st4 = reinterpret_cast<const float4 *>(st);
    uint32_t w[2] = {0u, 0u};
    uint32_t h = 0;
    // hits h .. h+3 into bits h mod 32 .. of word `half` (h is a multiple of 4, so a group
    // never straddles the two words)
    auto four = [&](uint32_t &acc, uint32_t sh) {
        const float4 a = st4[h >> 1], b = st4[(h >> 1) + 1];
        const float uu[4] = {a.x, a.z, b.x, b.z}, vv[4] = {a.y, a.w, b.y, b.w};
        uint32_t kk[4][G], wd[4][G];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const float t = __builtin_fmaf(uu[i], cl.C[q], __builtin_fmaf(vv[i], cl.S[q], cl.B[q]));
                kk[i][q] = (uint32_t)(int)t;
                uint32_t kw = kk[i][q] >> 5;        // see lookup1
                asm("" : "+v"(kw));
                wd[i][q] = kw * (64u * G) + 64u * q + (uint32_t)lane;
            }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < G; ++q) wd[i][q] = dil[wd[i][q]];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < G; ++q) {
                // one shift-or per bit (the empty asm keeps the compiler from regrouping the ORs
                // into separate shifts and three-input ORs)
                acc |= __builtin_amdgcn_ubfe(wd[i][q], kk[i][q], 1u) << (sh + i);
                asm("" : "+v"(acc));
            }
    };
    for (; h + 4 <= n.safe && h < 32; h += 4) four(w[0], h);
    for (; h + 4 <= n.safe; h += 4) four(w[1], h - 32);
    for (; h < n.total; ++h) {
        const float2 p = st[h];
        const uint32_t m = lookup1<G>(dil, p.x, p.y, h >= n.safe, cl, lane, nrho_f);
        if (h < 32) w[0] |= m << h; else w[1] |= m << (h - 32);
    }
    if (n.total == 0) return 0ull;
    const uint32_t klo = wave_or(w[0]);
    const uint32_t khi = n.total > 32 ? wave_or(w[1]) : 0u;
    return ((uint64_t)khi << 32) | klo;
}

__device__ __forceinline__ uint64_t low_bits(uint32_t n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

// Hits of a wave's range that are valid and not yet kept, once there are at most 64 of them:
// lane l holds one entry (an event-local hit index, bit 31 set for a later copy of a hit under
// duplicate suppression) while bit l of `live` is set.  Later tiles look up only these instead
// of mapping the whole range again.
struct Pending {
    uint32_t idx;
    uint64_t live;   // wave-uniform
    bool on;         // wave-uniform
};

// Collect the valid unkept hits of [hb, he) into the pending list (caller: at most 64 of
// them): their indices are compacted through the wave's stage.
__device__ void build_pending(Pending &pd, float2 *st, const float *x, const float *y,
                             const uint8_t *ke, uint32_t hb, uint32_t he, int lane) {
    // runs once per wave and event: keep the compiler from holding its per-lane addresses in
    // registers across the whole event
    asm volatile("" : "+v"(lane));
    uint32_t *st32 = reinterpret_cast<uint32_t *>(st);
    uint32_t n = 0;
    for (uint32_t base = hb; base < he; base += 64) {
        const uint32_t i = base + lane;
        const uint32_t kv = (i < he) ? ke[i] : 1u;
        const bool cand = (i < he) && !(kv & 1u);
        float xi = 0.0f, yi = 0.0f;
        if (cand) { xi = x[i]; yi = y[i]; }
        float u, v;
        const bool ok = conformal(xi, yi, u, v) && cand;
        const uint64_t b = __ballot(ok);
        if (ok) st32[n + mbcnt(b)] = i | ((kv & (uint32_t)kKeepDuplicate) << 30);
        n += (uint32_t)__popcll(b);
    }
    wave_sync();
    pd.on = true;
    pd.live = low_bits(n);
    if ((uint32_t)lane < n) pd.idx = st32[lane];
    wave_sync();
}

// Step 5 for the pending list: map and stage the live entries, look them up (every lookup
// takes the literal range test), write the keep byte of each kept entry and drop it.
template <int G>
__device__ uint32_t retain_pending(Pending &pd, const uint32_t *dil, float2 *st, const float *x,
                                   const float *y, uint8_t *ke, const Cols<G> &cl,
                                   const GridArgs &g, int lane) {
    if (pd.live == 0ull) return 0u;
    const bool me = (pd.live >> lane) & 1ull;
    const uint32_t pos = mbcnt(pd.live);
    const uint32_t idx = pd.idx & 0x7fffffffu;
    if (me) {
        float u, v;
        (void)conformal(x[idx], y[idx], u, v);
        st[pos] = make_float2(u, v);
    }
    wave_sync();
    const uint64_t kept = lookup_staged<G>(dil, st, StageCount{0u, (uint32_t)__popcll(pd.live)}, cl,
                                           lane, g.nrho_f);
    const bool k_me = me && ((kept >> pos) & 1ull);
    if (k_me) ke[idx] = (uint8_t)(1u | ((pd.idx >> 30) & (uint32_t)kKeepDuplicate));
    const uint64_t kept_lanes = __ballot(k_me);
    pd.live &= ~kept_lanes;
    wave_sync();
    return (uint32_t)__popcll(kept_lanes);
}

// Step 5 over the whole range [hb, he): every unkept valid hit is mapped again, staged and
// looked up; each lane sets the kept bit of its own hit's keep byte when its stage slot was
// kept (the event's keep bytes were cleared, or written by the duplicate pass, when it
// started, and only this lane touches them).  Returns
// the number of hits newly kept; `left` receives how many valid hits remain unkept.
template <int G>
__device__ uint32_t retain_range(const uint32_t *dil, float2 *st, const float *x,
                                 const float *y, uint8_t *ke, uint32_t hb, uint32_t he,
                                 const Cols<G> &cl, const GridArgs &g, int lane, uint32_t &left) {
    uint32_t unused = 0, newly = 0;
    left = 0;
    for (uint32_t base = hb; base < he; base += 64) {
        const uint32_t i = base + lane;
        const uint32_t kv = (i < he) ? ke[i] : 1u;
        const bool done = (i < he) && (kv & 1u);
        if (__ballot((i < he) && !done) == 0ull) continue;      // whole chunk already kept
        int slot;
        const StageCount n = stage_hits(st, x, y, base, he, done, g, lane, unused, slot);
        const uint64_t kept = lookup_staged<G>(dil, st, n, cl, lane, g.nrho_f);
        if (slot >= 0 && ((kept >> slot) & 1ull)) ke[i] = (uint8_t)(kv | 1u);
        const uint32_t nk = (uint32_t)__popcll(kept);
        newly += nk;
        left += n.total - nk;
        wave_sync();
    }
    return newly;
}

// Step 5 on a tile with at most kTilePeaks peaks, one lane per hit: hit (u, v) is kept by
// peak (column j, row k) when its own bin in column j (the vote's arithmetic, in range) is
// within rho_window of k, which is what a lookup of the dilated words tests; here it costs
// one step per peak for 64 hits instead of one step per hit for the tile's columns.  The list
// holds k - W (as int bits in z).  For a peak with W < k < N_rho - W the range test is implied:
// a bin t outside [0, N_rho) truncates to an integer below 1 or at least N_rho, out of
// [k - W, k + W]; so unless the tile has a peak nearer an edge (`edge`) a peak costs two fmas,
// a conversion, a subtraction and one unsigned compare.  t is first clamped to [-2, N_rho + W + 2]
// (one v_med3), which keeps the conversion defined and changes no verdict: a clamped bin lies
// outside every peak's window either way.  Returns the mask of kept lanes among `valid`, and
// stops once every valid lane is kept.
__device__ __forceinline__ uint64_t kept_by_peaks(const float4 *tpk, uint32_t np, float u, float v, bool valid,
                                                  bool edge, const GridArgs &g) {
    const uint64_t want = __ballot(valid);
    const uint32_t w2 = 2u * (uint32_t)g.rho_window;
    const float hi = g.nrho_f + (float)g.rho_window + 2.0f;
    uint64_t km = 0;
    // one peak: its compares go straight into wave masks (scalar ORs and ANDs)
    auto test = [&](const float4 &P) {
        const float t = __builtin_fmaf(u, P.x, __builtin_fmaf(v, P.y, g.Bf));
        const uint32_t dd = (uint32_t)(int)__builtin_amdgcn_fmed3f(t, -2.0f, hi) - __float_as_uint(P.z);
        uint64_t m = __ballot(dd <= w2);
        if (edge) m &= __ballot(t >= 0.0f) & __ballot(t < g.nrho_f);
        km |= m;
    };
    uint32_t p = 0;
    // four peaks at a time, their list reads issued together; done once every valid lane is kept
    for (; p + 4 <= np; p += 4) {
        float4 P[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) P[q] = tpk[p + q];       // the same address in every lane
#pragma unroll
        for (int q = 0; q < 4; ++q) test(P[q]);
        if ((km & want) == want) return want;
    }
    for (; p < np; ++p) test(tpk[p]);
    return km & want;
}

// retain_pending with the tile's peak list.
__device__ uint32_t retain_pending_peaks(Pending &pd, const float4 *tpk, uint32_t np, bool edge, const float *x,
                                         const float *y, uint8_t *ke, const GridArgs &g, int lane) {
    if (pd.live == 0ull) return 0u;
    const bool me = (pd.live >> lane) & 1ull;
    const uint32_t idx = pd.idx & 0x7fffffffu;
    float u = 0.0f, v = 0.0f;
    if (me) (void)conformal(x[idx], y[idx], u, v);
    const uint64_t kept_lanes = kept_by_peaks(tpk, np, u, v, me, edge, g);
    if ((kept_lanes >> lane) & 1ull) ke[idx] = (uint8_t)(1u | ((pd.idx >> 30) & (uint32_t)kKeepDuplicate));
    pd.live &= ~kept_lanes;
    return (uint32_t)__popcll(kept_lanes);
}

// retain_range with the tile's peak list: each lane maps and tests its own unkept hit.
__device__ uint32_t retain_range_peaks(const float4 *tpk, uint32_t np, bool edge, const float *x, const float *y,
                                       uint8_t *ke, uint32_t hb, uint32_t he, const GridArgs &g, int lane,
                                       uint32_t &left) {
    uint32_t newly = 0;
    left = 0;
    // the keep bytes and hits of the next 64 are loaded while these are tested
    uint32_t kn = 1u;
    float xn = 0.0f, yn = 0.0f;
    if (hb + lane < he) { kn = ke[hb + lane]; xn = x[hb + lane]; yn = y[hb + lane]; }
    for (uint32_t base = hb; base < he; base += 64) {
        const uint32_t i = base + lane;
        const uint32_t kv = kn;
        const float xi = xn, yi = yn;
        if (i + 64 < he) { kn = ke[i + 64]; xn = x[i + 64]; yn = y[i + 64]; }
        const bool cand = (i < he) && !(kv & 1u);
        if (__ballot(cand) == 0ull) continue;            // whole chunk already kept
        float u = 0.0f, v = 0.0f;
        bool valid = false;
        if (cand) valid = conformal(xi, yi, u, v);
        const uint64_t km = kept_by_peaks(tpk, np, u, v, valid, edge, g);
        if ((km >> lane) & 1ull) ke[i] = (uint8_t)(kv | 1u);
        const uint32_t nk = (uint32_t)__popcll(km);
        newly += nk;
        left += (uint32_t)__popcll(__ballot(valid)) - nk;
    }
    return newly;
}

// ------------------------------------------------------------------------ plain path
// Internal accumulator form of the iterative finder's batch path: 16-bit cells stored rho-major
// (acc[k * n_theta + j]), so that the write-out of a tile row is one contiguous run per wave.
constexpr int kAccU16RhoMajor = 3;

// Votes of hits [hb, he) into rows [r0, r1) of the lane's column only (a rho slab of the tile:
// tile row k - r0 holds grid row k): every vote takes the range test r0 <= t < r1, which for an
// integer r0 >= 0 is the same as r0 <= (int)t, so a vote lands exactly where the whole-grid rule
// puts it, or is left to another slab.  Returns the number of valid hits seen.
template <int NW>
__device__ uint32_t vote_range_slab(uint32_t *tile, float2 *st, const float *x, const float *y, uint32_t hb,
                                    uint32_t he, const Cols<1> &cl, const Lane<1, true> &ln, const GridArgs &g,
                                    int lane, uint32_t &bad, const uint8_t *dup, int r0, int r1) {
    const float lo_f = (float)r0, hi_f = (float)r1;
    uint32_t n_valid = 0;
    for (uint32_t base = hb; base < he; base += 64) {
        const uint32_t i = base + lane;
        bool live = i < he;
        float xi = 0.0f, yi = 0.0f;
        if (live) { xi = x[i]; yi = y[i]; }
        if (dup) {
            const bool copy = live && (dup[i] & kKeepDuplicate) != 0;
            n_valid += (uint32_t)__popcll(__ballot(copy && valid_hit(xi, yi)));
            live = live && !copy;
        }
        int slot;
        const StageCount n = stage_values(st, xi, yi, live, g, bad, slot);
        n_valid += n.total;
        for (uint32_t h = 0; h < n.total; ++h) {
            const float2 p = st[h];
            const float t = __builtin_fmaf(p.x, cl.C[0], __builtin_fmaf(p.y, cl.S[0], cl.B[0]));
            if (t >= lo_f && t < hi_f) lds_add(&tile[((int)t - r0) * Lane<1, true>::STRIDE + (int)ln.col[0]], ln.inc);
        }
        wave_sync();
    }
    return n_valid;
}

// Steps 1-3 of one event into one 64-column group of acc, rows [r0, r1) (the whole column, or a
// rho slab of it when the column does not fit LDS), by one workgroup: all hits of the event are
// swept through the group's tile.  Counters are packed two per dword, so the hits go through in
// chunks of at most 65,535 (a count then fits 16 bits); each chunk's tile is written out (first
// chunk) or added (later chunks) to acc, each element by the one thread that owns it.  dup as
// for vote_range.  Returns this thread's invalid-hit flag.
template <int NW>
__device__ uint32_t vote_group_to_acc(const GridArgs &g, const float *__restrict__ x,
                                      const float *__restrict__ y, uint32_t n_hits, void *acc,
                                      int acc_type, int group, const uint8_t *dup, int r0, int r1) {
    using L = Lane<1, true>;
    constexpr uint32_t kChunk = 65535u;
    extern __shared__ __align__(16) uint32_t lds[];
    const bool whole = r0 == 0 && r1 == g.n_rho;
    const int rows = r1 - r0;
    uint32_t *tile = lds;                                                  // [(rows + 1) * 32]
    float2 *stage = reinterpret_cast<float2 *>(tile + (size_t)(rows + 1) * L::STRIDE);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int first = group * 64;
    const L ln(lane);
    const Cols<1> cl = load_cols<1>(g, first, lane, L::STRIDE, ln.col);
    const int j = first + lane;
    const int kb = r0 + (int)((int64_t)rows * wave / NW), ke = r0 + (int)((int64_t)rows * (wave + 1) / NW);
    uint32_t bad = 0;
    uint32_t c0 = 0;
    do {
        const uint32_t c1 = n_hits - c0 > kChunk ? c0 + kChunk : n_hits;
        for (int i = threadIdx.x; i < (rows + 1) * L::STRIDE / 4; i += NW * 64)
            reinterpret_cast<uint4 *>(tile)[i] = make_uint4(0u, 0u, 0u, 0u);
        __syncthreads();
        const uint32_t hb = c0 + (uint32_t)((uint64_t)(c1 - c0) * wave / NW);
        const uint32_t he = c0 + (uint32_t)((uint64_t)(c1 - c0) * (wave + 1) / NW);
        if (whole)
            vote_range<1, true>(tile, stage + wave * 64, x, y, hb, he, cl, ln, g, lane, bad, dup);
        else
            vote_range_slab<NW>(tile, stage + wave * 64, x, y, hb, he, cl, ln, g, lane, bad, dup, r0, r1);
        __syncthreads();
        // write-out: lane = column (theta row of acc), wave = a slice of the slab's rows
        if (j < g.n_theta) {
            if (acc_type == kAccU16RhoMajor) {         // acc[k][j]: a wave stores 64 adjacent cells
                uint16_t *col = static_cast<uint16_t *>(acc) + j;
                for (int k = kb; k < ke; ++k) {
                    const uint32_t v = ln.count(tile[(k - r0) * L::STRIDE + ln.col[0]]);
                    uint16_t *cell = col + (size_t)k * g.n_theta;
                    *cell = (uint16_t)(c0 ? *cell + v : v);
                }
            } else if (acc_type == HOUGH_ACC_U16) {
                uint16_t *row = static_cast<uint16_t *>(acc) + (size_t)j * g.n_rho;
                for (int k = kb; k < ke; ++k) {
                    const uint32_t v = ln.count(tile[(k - r0) * L::STRIDE + ln.col[0]]);
                    row[k] = (uint16_t)(c0 ? row[k] + v : v);
                }
            } else {
                uint32_t *row = static_cast<uint32_t *>(acc) + (size_t)j * g.n_rho;
                for (int k = kb; k < ke; ++k) {
                    const uint32_t v = ln.count(tile[(k - r0) * L::STRIDE + ln.col[0]]);
                    row[k] = c0 ? row[k] + v : v;
                }
            }
        }
        __syncthreads();
        c0 = c1;
    } while (c0 < n_hits);
    return bad;
}

// hough_vote: workgroup (64-column group, rho slab of slab_rows rows).
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_vote(GridArgs g, const float *__restrict__ x,
                                                  const float *__restrict__ y, uint32_t n_hits,
                                                  void *acc, int acc_type, int slab_rows) {
    const int r0 = (int)blockIdx.y * slab_rows, r1 = min(r0 + slab_rows, g.n_rho);
    (void)vote_group_to_acc<NW>(g, x, y, n_hits, acc, acc_type, (int)blockIdx.x, nullptr, r0, r1);
}

// Steps 1-3 for a batch of CSR events into per-event 16-bit accumulators (the iterative
// finder's batch form): workgroup (event, 64-column group, rho slab).  Workgroup (e, 0, 0) writes
// the event's status (invalid hits, too many hits, duplicate pass skipped); the later kernels OR
// into it.  An event above kMaxBatchHits hits, or with malformed offsets, gets no accumulator.
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_vote_batch(GridArgs g, const float *__restrict__ x,
                                                        const float *__restrict__ y,
                                                        const uint32_t *__restrict__ offsets,
                                                        uint16_t *acc, const uint8_t *keep,
                                                        uint32_t *status, int slab_rows) {
    const uint32_t e = blockIdx.x;
    const bool first_wg = blockIdx.y == 0 && blockIdx.z == 0;
    const uint32_t h0 = offsets[e], h1 = offsets[e + 1];
    const bool ok = h1 >= h0 && h1 - h0 <= kMaxBatchHits;
    if (!ok) {
        if (first_wg && threadIdx.x == 0) status[e] = HOUGH_EV_TOO_MANY_HITS;
        return;
    }
    const uint32_t H = h1 - h0;
    const size_t cells = (size_t)g.n_theta * (size_t)g.n_rho;
    const int r0 = (int)blockIdx.z * slab_rows, r1 = min(r0 + slab_rows, g.n_rho);
    const uint32_t bad = vote_group_to_acc<NW>(g, x + h0, y + h0, H, acc + (size_t)e * cells, kAccU16RhoMajor,
                                               (int)blockIdx.y, g.dedup ? keep + h0 : nullptr, r0, r1);
    __shared__ uint32_t s_bad;
    if (threadIdx.x == 0) s_bad = 0u;
    __syncthreads();
    if (bad) s_bad = 1u;
    __syncthreads();
    // every workgroup sees every hit of the event, so the first one's flags are the event's
    if (first_wg && threadIdx.x == 0)
        status[e] = (s_bad ? HOUGH_EV_INVALID_HITS : 0u) |
                    (g.dedup && H > kDedupMaxHits ? HOUGH_EV_DEDUP_SKIPPED : 0u);
}

// hough_peaks: workgroup b tests theta rows [NW*b, NW*b + NW), staged in LDS with one halo row
// on each side, one wave per row, lanes over rho.  Two launches: the first writes each block's
// peak count to counts[b]; the second lists each block's peaks at the sum of the earlier blocks'
// counts plus the earlier waves' (raster order), and block 0 writes the total.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    return v;
}

template <int NW, typename T, bool WRITE>
__global__ __launch_bounds__(NW * 64) void k_peaks(GridArgs g, const T *__restrict__ acc,
                                                   hough_peak *out, uint32_t cap,
                                                   uint32_t *n_peaks, uint32_t *counts) {
    extern __shared__ __align__(16) uint32_t lds[];
    uint32_t *rows = lds;   // [(NW + 2) * n_rho], buffer row r holds grid row jb - 1 + r
    __shared__ uint32_t s_cnt[NW];
    __shared__ uint32_t s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nr = g.n_rho;
    const int jb = (int)blockIdx.x * NW;
    for (int idx = threadIdx.x; idx < (NW + 2) * nr; idx += NW * 64) {
        const int r = idx / nr, k = idx - r * nr, jj = jb - 1 + r;
        uint32_t v = 0u;
        if (jj >= 0 && jj < g.n_theta) v = (uint32_t)acc[(size_t)jj * nr + k];
        else if (g.periodic && (jj == -1 || jj == g.n_theta))   // the other edge, rho reversed
            v = (uint32_t)acc[(size_t)(jj < 0 ? g.n_theta - 1 : 0) * nr + (nr - 1 - k)];
        rows[idx] = v;
    }
    if (WRITE && wave == 0) {                     // peaks of the earlier blocks, and of all
        uint32_t before = 0, all = 0;
        for (uint32_t q = (uint32_t)lane; q < gridDim.x; q += 64) {
            const uint32_t c = counts[q];
            all += c;
            if (q < blockIdx.x) before += c;
        }
        before = wave_sum(before);
        all = wave_sum(all);
        if (lane == 0) {
            s_base = before;
            if (blockIdx.x == 0) *n_peaks = all;
        }
    }
    __syncthreads();
    const int j = jb + wave;
    const uint32_t *up = rows + wave * nr, *mid = up + nr, *dn = mid + nr;
    // on a periodic grid the row above column 0 is column n_theta - 1 (later in raster order)
    // and the row below column n_theta - 1 is column 0 (earlier)
    const bool up_later = g.periodic && j == 0, dn_earlier = g.periodic && j == g.n_theta - 1;
    auto is_peak = [&](int k) -> bool {
        const uint32_t c = mid[k];
        const uint32_t l = k > 0 ? 1u : 0u, r = k + 1 < nr ? 1u : 0u;
        const uint32_t u3 = max(max(l ? up[k - 1] : 0u, up[k]), r ? up[k + 1] : 0u);
        const uint32_t d3 = max(max(l ? dn[k - 1] : 0u, dn[k]), r ? dn[k + 1] : 0u);
        const uint32_t before = max(max(up_later ? 0u : u3, dn_earlier ? d3 : 0u), l ? mid[k - 1] : 0u);
        const uint32_t after = max(max(up_later ? u3 : 0u, dn_earlier ? 0u : d3), r ? mid[k + 1] : 0u);
        return c >= max(max(g.threshold, before + 1u), after);
    };
    uint32_t cnt = 0;
    if (j < g.n_theta) {
        for (int kc = 0; kc < nr; kc += 64) {
            const int k = kc + lane;
            cnt += (uint32_t)__popcll(__ballot(k < nr && is_peak(k)));
        }
    }
    if (lane == 0) s_cnt[wave] = cnt;
    __syncthreads();
    if (!WRITE) {
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int w = 0; w < NW; ++w) t += s_cnt[w];
            counts[blockIdx.x] = t;
        }
        return;
    }
    uint32_t base = s_base;
    for (int w = 0; w < wave; ++w) base += s_cnt[w];
    if (j < g.n_theta) {
        for (int kc = 0; kc < nr; kc += 64) {
            const int k = kc + lane;
            const bool p = k < nr && is_peak(k);
            const uint64_t m = __ballot(p);
            if (p) {
                const uint32_t idx = base + mbcnt(m);
                if (idx < cap) store_peak(out + idx, (uint32_t)j, (uint32_t)k, mid[k]);
            }
            base += (uint32_t)__popcll(m);
        }
    }
}

// hough_peaks_iterative: the paper's peak finder (relative threshold, then iterative extraction
// with neighbourhood suppression) for one event, in one workgroup of kIterWaves waves.
//
// A cell at or above the threshold is a candidate, keyed count << 32 | ~(raster index).  The
// step-by-step extraction takes the candidates in descending key order (larger count first, then
// earlier in raster order) and passes over those an earlier taken cell suppresses: suppression
// depends only on the cells already taken.  The kernel does exactly that in chunks.  A chunk is
// the next run of the sorted candidates that fits the LDS key buffer (K keys): its key range
// comes from a histogram of the remaining candidates' counts (and, when one count alone has more
// than K candidates, of their raster indices); it is gathered, sorted (bitonic, descending) and
// walked in order by wave 0, 64 keys at a time, against a suppression bitmap of the whole grid
// (one bit per cell, raster-indexed, set for every cell within r_theta columns and r_rho rows of
// a taken cell).  Candidates the bitmap covers are left out of later chunks.  The bitmap lives in
// LDS after the keys when it fits (GBM false), else in device memory (GBM true).
constexpr int kIterWaves = 16;
constexpr uint32_t kIterThreads = kIterWaves * 64;
constexpr uint32_t kIterMaxKeys = 16384;     // 128 KB of LDS
constexpr uint32_t kIterMinKeys = 1024;

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

// The suppression bitmap: every access comes from the event's own workgroup, so workgroup-scope
// atomics order the marks of wave 0 against the later reads of every wave (LDS or device memory).
__device__ __forceinline__ bool bm_test(const uint32_t *bm, uint32_t r) {
    const uint32_t w = __hip_atomic_load(bm + (r >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return (w >> (r & 31)) & 1u;
}

// Set the bits of every cell within r_theta columns and r_rho rows of (jf, kf), clipped at the
// grid edges: per column one raster run jj * n_rho + [k0, k1], a few words each; the 64 lanes
// take the (column, word) pairs.
__device__ void mark_window(uint32_t *bm, int jf, int kf, int r_theta, int r_rho, int n_theta, int n_rho,
                            uint32_t lane) {
    const int j0 = max(jf - r_theta, 0), j1 = min(jf + r_theta, n_theta - 1);
    const int k0 = max(kf - r_rho, 0), k1 = min(kf + r_rho, n_rho - 1);
    const uint32_t per = (uint32_t)((k1 - k0) >> 5) + 2u;          // words one column can touch
    const uint32_t units = (uint32_t)(j1 - j0 + 1) * per;
    for (uint32_t u = lane; u < units; u += 64) {
        const uint32_t col = (uint32_t)j0 + u / per, slot = u % per;
        const uint32_t a = col * (uint32_t)n_rho + (uint32_t)k0, e = col * (uint32_t)n_rho + (uint32_t)k1;
        const uint32_t w = (a >> 5) + slot;
        if (w > (e >> 5)) continue;
        const uint32_t lo = w == (a >> 5) ? (a & 31u) : 0u, hi = w == (e >> 5) ? (e & 31u) : 31u;
        const uint32_t bits = (hi == 31u ? ~0u : ((1u << (hi + 1u)) - 1u)) & ~((1u << lo) - 1u);
        __hip_atomic_fetch_or(bm + w, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// Every cell of an accumulator of `cells` cells, eight loads in flight per lane: f(c, v, in) for
// storage index c, count v, and in = c < cells.  Every lane calls f the same number of times per
// wave, so f may use wave-wide operations.
template <typename T, typename F>
__device__ __forceinline__ void for_cells(const T *acc, uint32_t cells, F &&f) {
    constexpr int U = 8;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t base = wave * 64u; base < cells; base += U * kIterThreads) {
        uint32_t v[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint32_t c = base + (uint32_t)r * kIterThreads + lane;
            v[r] = c < cells ? (uint32_t)acc[c] : 0u;
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint32_t c = base + (uint32_t)r * kIterThreads + lane;
            f(c, v[r], c < cells);
        }
    }
}

// Append `key` for the lanes where p holds, at positions taken from the LDS counter *cnt (one
// atomic per wave); positions at or past `room` are counted but not stored.
__device__ __forceinline__ void append_key(uint64_t *keys, uint32_t *cnt, uint32_t room, bool p, uint64_t key,
                                           uint32_t lane) {
    const uint64_t b = __ballot(p);
    if (!b) return;
    uint32_t off = 0;
    if (lane == 0) off = atomicAdd(cnt, (uint32_t)__popcll(b));
    off = (uint32_t)__shfl((int)off, 0, 64);
    const uint32_t pos = off + mbcnt(b);
    if (p && pos < room) keys[pos] = key;
}

// Wave 0 reads hist[0 .. nb) in processing order (from bin nb - 1 down when `top`, else from bin
// 0 up) and returns, through *m, the number of leading bins whose counts sum to at most `room`
// and, through *first, the position of the first non-empty bin (nb when all are empty).  nb is a
// multiple of 64.
__device__ void hist_fit(const uint32_t *hist, uint32_t nb, bool top, uint32_t room, uint32_t lane, uint32_t *m,
                         uint32_t *first) {
    const uint32_t per = nb / 64u, q0 = lane * per;
    uint32_t s = 0, f = nb;
    for (uint32_t q = q0; q < q0 + per; ++q) {
        const uint32_t h = hist[top ? nb - 1u - q : q];
        if (h && f == nb) f = q;
        s += h;
    }
    const uint32_t incl = wave_inclusive_scan(s, (int)lane);
    const uint64_t over = __ballot(incl > room);
    uint32_t mm = nb;
    if (over) {
        const uint32_t cl = (uint32_t)__builtin_ctzll(over);
        if (lane == cl) {
            uint32_t run = incl - s;
            for (uint32_t q = q0; q < q0 + per; ++q) {
                run += hist[top ? nb - 1u - q : q];
                if (run > room) { mm = q; break; }
            }
        }
        mm = (uint32_t)__builtin_amdgcn_readlane((int)mm, (int)cl);
    }
    *m = mm;
    *first = wave_min(f);
}

// offsets (batch form, else null): workgroup e takes event e's accumulator (rho-major 16-bit
// cells) at acc + e * cells, writes its list at out + e * cap, n_peaks[e], and ORs
// HOUGH_EV_PEAKS_TRUNCATED into status[e] (which the batch vote wrote); events the vote skipped
// get no peaks.  K: keys in the LDS buffer (a power of two, kIterMinKeys .. kIterMaxKeys).
// gbm (GBM): device bitmaps of bm_words words, one per workgroup.
template <typename T, bool GBM>
__global__ __launch_bounds__(kIterThreads) void k_peaks_iter(GridArgs g, const T *__restrict__ acc,
                                                             uint32_t frac_num, uint32_t frac_den, int r_theta,
                                                             int r_rho, hough_peak *out, uint32_t cap,
                                                             uint32_t *n_peaks, uint32_t *status,
                                                             const uint32_t *offsets, uint32_t K, uint32_t *gbm) {
    extern __shared__ __align__(16) uint64_t keys[];       // [K]; the histograms reuse it as 2K words
    uint32_t *hist = reinterpret_cast<uint32_t *>(keys);
    __shared__ uint32_t s_red[kIterWaves];
    __shared__ uint32_t s_n, s_m, s_first, s_taken;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nr = (uint32_t)g.n_rho, nt = (uint32_t)g.n_theta;
    const uint32_t cells = nt * nr, bm_words = (cells + 31u) / 32u, NB = 2u * K;
    const bool batch = offsets != nullptr;
    // the batch form stores rho-major (see kAccU16RhoMajor); keys and the bitmap use raster order
    auto raster = [&](uint32_t c) -> uint32_t {
        if (!batch) return c;
        const uint32_t k = c / nt;
        return (c - k * nt) * nr + k;
    };
    if (batch) {
        const uint32_t e = blockIdx.x;
        acc += (size_t)e * cells;
        out = out ? out + (size_t)e * cap : nullptr;
        n_peaks += e;
        status += e;
        const uint32_t h0 = offsets[e], h1 = offsets[e + 1];
        if (h1 < h0 || h1 - h0 > kMaxBatchHits) {              // no accumulator was written
            if (tid == 0) *n_peaks = 0u;
            return;
        }
    }
    uint32_t *bm = GBM ? gbm + (batch ? (size_t)blockIdx.x * bm_words : (size_t)0)
                       : reinterpret_cast<uint32_t *>(keys + K);
    for (uint32_t w = tid; w < bm_words; w += kIterThreads) bm[w] = 0u;
    if (tid == 0) { s_n = 0u; s_taken = 0u; }
    __syncthreads();

    // pass 1: the maximum, and the candidates of the absolute floor while they fit
    const uint32_t floor_t = g.threshold;
    uint32_t m = 0;
    for_cells(acc, cells, [&](uint32_t c, uint32_t v, bool in) {
        m = max(m, v);
        const bool p = in && v >= floor_t;
        append_key(keys, &s_n, K, p, p ? ((uint64_t)v << 32) | (uint64_t)(~raster(c)) : 0ull, lane);
    });
    m = wave_max(m);
    if (lane == 0) s_red[wave] = m;
    __syncthreads();
    uint32_t mx = 0;
    for (int w = 0; w < kIterWaves; ++w) mx = max(mx, s_red[w]);
    const uint64_t rel = ((uint64_t)mx * frac_num + frac_den - 1u) / frac_den;
    const uint32_t thr = (uint32_t)min<uint64_t>(max<uint64_t>(rel, floor_t), 0xffffffffull);
    const uint32_t n1 = s_n;
    __syncthreads();

    bool bounded = false;      // keys below `hi` are what is left once a chunk has been walked
    uint64_t hi = 0;
    bool have_chunk = false;
    uint32_t n = 0;
    uint64_t lo = 0;           // the chunk's lowest key (0: the chunk holds every candidate left)
    if (n1 <= K) {
        // every floor candidate is in LDS: keep those that reach thr, in place
        if (thr > floor_t) {
            if (tid == 0) s_n = 0u;
            __syncthreads();
            for (uint32_t i0 = 0; i0 < n1; i0 += kIterThreads) {
                const uint32_t i = i0 + tid;
                const uint64_t key = i < n1 ? keys[i] : 0ull;
                __syncthreads();
                append_key(keys, &s_n, K, i < n1 && (uint32_t)(key >> 32) >= thr, key, lane);
                __syncthreads();
            }
        }
        n = s_n;
        have_chunk = true;
    }
    for (;;) {
        if (!have_chunk) {
            // the next chunk: the largest remaining keys whose number fits K
            uint32_t vlo = thr, vhi = bounded ? (uint32_t)(hi >> 32) : mx;
            bool none = vhi < vlo;
            while (!none) {
                const uint32_t w = (uint32_t)(((uint64_t)vhi - vlo + 1u + NB - 1u) / NB);
                for (uint32_t b = tid; b < NB; b += kIterThreads) hist[b] = 0u;
                __syncthreads();
                for_cells(acc, cells, [&](uint32_t c, uint32_t v, bool in) {
                    if (!in || v < vlo || v > vhi) return;
                    const uint32_t r = raster(c);
                    const uint64_t key = ((uint64_t)v << 32) | (uint64_t)(~r);
                    if ((bounded && key >= hi) || bm_test(bm, r)) return;
                    atomicAdd(&hist[(v - vlo) / w], 1u);
                });
                __syncthreads();
                if (wave == 0) hist_fit(hist, NB, true, K, lane, &s_m, &s_first);
                __syncthreads();
                const uint32_t mb = s_m, fb = s_first;
                __syncthreads();
                if (fb == NB) { none = true; break; }                   // nothing left
                if (mb > fb) {                                          // bins NB - mb .. NB - 1 fit
                    lo = (uint64_t)(vlo + (NB - mb) * w) << 32;
                    break;
                }
                const uint32_t bt = NB - 1u - fb;                       // the top non-empty bin, too full
                if (w > 1u) {
                    vhi = (uint32_t)min<uint64_t>((uint64_t)vhi, (uint64_t)vlo + (uint64_t)bt * w + w - 1u);
                    vlo = vlo + bt * w;
                    continue;
                }
                // one count vt has more than K candidates left: split them by raster index
                const uint32_t vt = vlo + bt;
                uint32_t rlo = (bounded && vt == (uint32_t)(hi >> 32)) ? ~(uint32_t)hi + 1u : 0u, rhi = cells - 1u;
                for (;;) {
                    const uint32_t wr = (uint32_t)(((uint64_t)rhi - rlo + 1u + NB - 1u) / NB);
                    for (uint32_t b = tid; b < NB; b += kIterThreads) hist[b] = 0u;
                    __syncthreads();
                    for_cells(acc, cells, [&](uint32_t c, uint32_t v, bool in) {
                        if (!in || v != vt) return;
                        const uint32_t r = raster(c);
                        if (r < rlo || r > rhi || bm_test(bm, r)) return;
                        atomicAdd(&hist[(r - rlo) / wr], 1u);
                    });
                    __syncthreads();
                    if (wave == 0) hist_fit(hist, NB, false, K, lane, &s_m, &s_first);
                    __syncthreads();
                    const uint32_t mr = s_m, fr = s_first;
                    __syncthreads();
                    if (mr > fr) {                                      // raster bins 0 .. mr - 1 fit
                        const uint32_t r_end = (uint32_t)min<uint64_t>((uint64_t)rhi, (uint64_t)rlo + (uint64_t)mr * wr - 1u);
                        lo = ((uint64_t)vt << 32) | (uint64_t)(~r_end);
                        break;
                    }
                    rhi = (uint32_t)min<uint64_t>((uint64_t)rhi, (uint64_t)rlo + (uint64_t)fr * wr + wr - 1u);
                    rlo = rlo + fr * wr;
                }
                break;
            }
            if (none) break;
            if (lo == ((uint64_t)thr << 32)) lo = 0;                    // every count down to thr
            // gather the chunk: the remaining keys in [lo, hi)
            if (tid == 0) s_n = 0u;
            __syncthreads();
            for_cells(acc, cells, [&](uint32_t c, uint32_t v, bool in) {
                bool p = in && v >= thr;
                uint64_t key = 0;
                if (p) {
                    const uint32_t r = raster(c);
                    key = ((uint64_t)v << 32) | (uint64_t)(~r);
                    p = key >= lo && (!bounded || key < hi) && !bm_test(bm, r);
                }
                append_key(keys, &s_n, K, p, key, lane);
            });
            __syncthreads();
            n = s_n;
        }
        have_chunk = false;
        // bitonic sort, descending, over the next power of two (n <= K)
        uint32_t P = 1;
        while (P < n) P <<= 1;
        for (uint32_t i = n + tid; i < P; i += kIterThreads) keys[i] = 0ull;
        __syncthreads();
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = tid; i < P; i += kIterThreads) {
                    const uint32_t ixj = i ^ j;
                    if (ixj > i) {
                        const uint64_t a = keys[i], b = keys[ixj];
                        const bool desc = (i & k) == 0u;
                        if (desc ? (a < b) : (a > b)) { keys[i] = b; keys[ixj] = a; }
                    }
                }
                __syncthreads();
            }
        }
        // the walk (wave 0): a key the bitmap covers is passed over; within a group of 64 the
        // first live key is taken and suppresses the later ones in its window; the group's taken
        // cells then mark their windows for the keys after them
        if (wave == 0) {
            uint32_t taken = s_taken;
            for (uint32_t base = 0; base < n; base += 64) {
                const uint32_t i = base + lane;
                bool live = i < n;
                const uint64_t key = live ? keys[i] : 0ull;
                const uint32_t r = ~(uint32_t)key, v = (uint32_t)(key >> 32);
                const int j = live ? (int)(r / nr) : 0, k = live ? (int)(r - (uint32_t)j * nr) : 0;
                live = live && !bm_test(bm, r);
                uint64_t b = __ballot(live), took = 0;
                while (b) {
                    const int f = __builtin_ctzll(b);
                    const int jf = __builtin_amdgcn_readlane(j, f), kf = __builtin_amdgcn_readlane(k, f);
                    const uint32_t vf = (uint32_t)__builtin_amdgcn_readlane((int)v, f);
                    if (lane == 0 && taken < cap) store_peak(out + taken, (uint32_t)jf, (uint32_t)kf, vf);
                    ++taken;
                    took |= 1ull << f;
                    live = live && (int)lane != f && !(abs(j - jf) <= r_theta && abs(k - kf) <= r_rho);
                    b = __ballot(live);
                }
                while (took) {
                    const int f = __builtin_ctzll(took);
                    took &= took - 1ull;
                    mark_window(bm, __builtin_amdgcn_readlane(j, f), __builtin_amdgcn_readlane(k, f), r_theta,
                                r_rho, (int)nt, (int)nr, lane);
                }
                wave_sync();
            }
            if (lane == 0) s_taken = taken;
        }
        __syncthreads();
        if (lo == 0) break;                       // the chunk reached the lowest candidate
        bounded = true;
        hi = lo;
    }
    if (tid == 0) {
        const uint32_t taken = s_taken;
        *n_peaks = taken;
        const uint32_t tr = taken > cap ? HOUGH_EV_PEAKS_TRUNCATED : 0u;
        *status = batch ? (*status | tr) : tr;
    }
}

// hough_track_params: one wave per peak.  The lanes sweep the event's hits 64 at a time and
// count, with ballots, the hits the retention rule associates with the peak and how many of
// them lie on either side of the line from the origin through the circle's centre; lane 0
// turns the peak into the circle (double precision) and writes the record.
constexpr int kTrackWaves = 4;

__global__ __launch_bounds__(kTrackWaves * 64) void k_track_params(GridArgs g, const float *__restrict__ x,
                                                                   const float *__restrict__ y,
                                                                   uint32_t n_hits, const hough_peak *peaks,
                                                                   const uint32_t *n_peaks, uint32_t cap,
                                                                   double rho_min, double rho_max,
                                                                   double b_tesla, hough_track *out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t p = blockIdx.x * kTrackWaves + (uint32_t)wave;
    const uint32_t np = min(*n_peaks, cap);
    if (p >= np) return;
    const uint2 rec = reinterpret_cast<const uint2 *>(peaks)[p];
    const int j = (int)(rec.x & 0xffffu), k = (int)(rec.x >> 16);
    const double pi = 3.14159265358979323846;
    const double drho = (rho_max - rho_min) / (double)g.n_rho;
    const double theta = ((double)j * pi) / (double)g.n_theta;
    const double rho = rho_min + ((double)k + 0.5) * drho;
    const bool in_grid = j < g.n_theta && k < g.n_rho;
    const float Cj = in_grid ? g.C[j] : 0.0f, Sj = in_grid ? g.S[j] : 0.0f;
    uint32_t n = 0, ccw = 0, cw = 0;
    for (uint32_t base = 0; in_grid && base < n_hits; base += 64) {
        const uint32_t i = base + lane;
        float xi = 0.0f, yi = 0.0f;
        if (i < n_hits) { xi = x[i]; yi = y[i]; }
        float u, v;
        const bool ok = conformal(xi, yi, u, v) && i < n_hits;
        const float w = __builtin_fmaf(v, Sj, g.Bf);
        const float t = __builtin_fmaf(u, Cj, w);
        const bool in = ok && t >= 0.0f && t < g.nrho_f;
        const int d = in ? abs((int)t - k) : 0;
        const bool mine = in && d <= g.rho_window;
        float side = __builtin_fmaf(Cj, yi, -(Sj * xi));
        if (rho < 0.0) side = -side;
        n += (uint32_t)__popcll(__ballot(mine));
        ccw += (uint32_t)__popcll(__ballot(mine && side > 0.0f));
        cw += (uint32_t)__popcll(__ballot(mine && side < 0.0f));
    }
    if (lane == 0) {
        hough_track tr;
        tr.a = cos(theta) / (2.0 * rho);
        tr.b = sin(theta) / (2.0 * rho);
        tr.radius = 1.0 / (2.0 * fabs(rho));
        tr.pt = 0.299792458 * b_tesla * tr.radius * 1e-3;
        tr.phi_c = atan2(tr.b, tr.a);
        tr.charge = ccw > cw ? 1 : (ccw < cw ? -1 : 0);
        tr.n_hits = n;
        out[p] = tr;
    }
}

// hough_retain: workgroup b takes hits b*NW*64 ..., 64 per wave, mapped and staged once.  The
// theta rows are processed in blocks that fit LDS: for each block the dilated peak bits (bit k
// of row j set iff a peak (j, k') has |k - k'| <= W) are built from the peak list, stored as
// [64-row group][word][row in group], and every wave looks its staged hits up 64 rows at a time
// with lane = row, exactly as the fused kernel looks them up in its tile's columns.
// offsets (batch form, else null): workgroup (e, b) covers hits b*NW*64 ... of event e, with
// event e's peak list at peaks + e * cap and n_peaks[e]; the keep bytes of an event the vote
// skipped for its size are zeroed (malformed offsets: nothing is touched).
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_retain(GridArgs g, const float *__restrict__ x,
                                                    const float *__restrict__ y, uint32_t n_hits,
                                                    const hough_peak *__restrict__ peaks,
                                                    const uint32_t *n_peaks, uint32_t cap,
                                                    uint8_t *keep, int rows_per_block,
                                                    const uint32_t *offsets = nullptr) {
    extern __shared__ __align__(16) uint32_t lds[];
    const int words = (g.n_rho + 31) / 32;
    float2 *stage = reinterpret_cast<float2 *>(lds);              // [NW * 64]
    uint32_t *dil = lds + 2 * NW * 64;                             // [rows_per_block / 64][words][64]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t blk = blockIdx.x;
    if (offsets) {
        const uint32_t e = blockIdx.x;
        blk = blockIdx.y;
        const uint32_t h0 = offsets[e], h1 = offsets[e + 1];
        if (h1 < h0) return;
        if (h1 - h0 > kMaxBatchHits) {
            for (uint32_t i = h0 + blk * (NW * 64) + threadIdx.x; i < h1; i += gridDim.y * (NW * 64)) keep[i] = 0u;
            return;
        }
        if (blk * (uint32_t)(NW * 64) >= h1 - h0) return;
        x += h0;
        y += h0;
        keep += h0;
        n_hits = h1 - h0;
        peaks += (size_t)e * cap;
        n_peaks += e;
    }
    const uint32_t np = min(*n_peaks, cap);
    const uint32_t base = blk * (NW * 64) + (uint32_t)wave * 64u;
    const uint32_t i = base + (uint32_t)lane;
    float2 *st = stage + wave * 64;
    uint32_t unused = 0;
    int slot;
    const StageCount n = stage_hits(st, x, y, base, n_hits, false, g, lane, unused, slot);
    uint64_t kept = 0;
    for (int ja = 0; ja < g.n_theta; ja += rows_per_block) {
        const int nrow = min(rows_per_block, g.n_theta - ja);
        const int ngroups = (nrow + 63) / 64;
        for (int t = threadIdx.x; t < ngroups * words * 64; t += NW * 64) dil[t] = 0u;
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < np; p += NW * 64) {
            const uint2 pk = reinterpret_cast<const uint2 *>(peaks)[p];
            const int j = (int)(pk.x & 0xffffu), k = (int)(pk.x >> 16);
            if (j < ja || j >= ja + nrow || k >= g.n_rho) continue;
            const int lo = k - g.rho_window > 0 ? k - g.rho_window : 0;
            const int hi = k + g.rho_window < g.n_rho - 1 ? k + g.rho_window : g.n_rho - 1;
            const int r = j - ja;
            uint32_t *col = dil + (size_t)(r >> 6) * words * 64 + (r & 63);
            for (int wd = lo >> 5; wd <= (hi >> 5); ++wd) {
                const int a = max(lo, wd * 32) - wd * 32, b = min(hi, wd * 32 + 31) - wd * 32;
                const uint32_t m = (b == 31 ? 0xffffffffu : ((1u << (b + 1)) - 1u)) & ~((1u << a) - 1u);
                __hip_atomic_fetch_or(&col[wd * 64], m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        __syncthreads();
        for (int q = 0; q < ngroups; ++q) {
            // lane = theta row ja + 64q + lane; rows past the grid look up a zero word of row 0
            const int j = ja + 64 * q + lane;
            Cols<1> cl;
            const bool row_in = j < g.n_theta;
            cl.C[0] = row_in ? g.C[j] : 0.0f;
            cl.S[0] = row_in ? g.S[j] : 0.0f;
            cl.B[0] = row_in ? g.Bf : 0.0f;
            kept |= lookup_staged<1>(dil + (size_t)q * words * 64, st, n, cl, lane, g.nrho_f);
        }
        __syncthreads();
    }
    if (i < n_hits) keep[i] = (slot >= 0 && ((kept >> slot) & 1ull)) ? 1u : 0u;
}

// Phase clock of the instrumented build (compiled with HOUGH_PHASE_TIMING; the product build
// compiles it away): thread 0 of a workgroup reads the constant-rate clock after each workgroup
// barrier and charges the interval to the phase that just ended; at exit it adds its totals to
// a device array that hough_debug_phase_ticks reads.
#ifdef HOUGH_PHASE_TIMING
}  // namespace
__device__ unsigned long long g_phase_ticks[kPhaseSlots];
namespace {
struct PhaseClock {
    uint64_t last = 0, t[kPhaseSlots] = {};
    __device__ __forceinline__ void start() {
        if (threadIdx.x == 0) last = (uint64_t)wall_clock64();
    }
    __device__ __forceinline__ void mark(int i) {
        if (threadIdx.x == 0) {
            const uint64_t n = (uint64_t)wall_clock64();
            t[i] += n - last;
            last = n;
        }
    }
    __device__ __forceinline__ void count(int i, uint64_t v) {
        if (threadIdx.x == 0) t[i] += v;
    }
    __device__ __forceinline__ void flush() {
        if (threadIdx.x == 0)
            for (int i = 0; i < kPhaseSlots; ++i) atomicAdd(&g_phase_ticks[i], (unsigned long long)t[i]);
    }
};
#else
struct PhaseClock {
    __device__ __forceinline__ void start() {}
    __device__ __forceinline__ void mark(int) {}
    __device__ __forceinline__ void count(int, uint64_t) {}
    __device__ __forceinline__ void flush() {}
};
#endif

// ------------------------------------------------------------------------ fused batch path
// One workgroup processes one event at a time, taken from a global work counter; the event's
// theta tiles are processed in order: vote, find peaks, list + dilate, then retain while the
// tile is cleared for the next one.  Counters are packed two per dword (an event has at most
// kMaxBatchHits hits, so a count fits 16 bits).  Wave w owns hits [hb, he) of the event for
// voting and retention and writes their keep bytes itself (each lane those of its own hits,
// the pending list aside).  Retention is skipped for the rest of the event once every valid
// hit is kept.
// queue[0] is the work counter and queue[1] counts workgroups that have left the loop; the
// last one to leave (every pop has then happened) puts both back to zero for the next launch,
// so a launch is a single kernel with no memset.
// SP: tiles with at most kTilePeaks peaks list them for the peak-list retention (the plan's
// choice for sparse grids and the relative threshold; compiled out otherwise, where it only
// costs).
// WIN: the tile holds a window of `win` rho rows (a multiple of 32) instead of the whole
// column.  The hits of an event vote only into the rows their radius lets them reach (|rho| is at
// most 1 / sqrt(x^2 + y^2) in every column), so each event is given the window [wb, wb + win)
// (wb a multiple of 16) that covers those rows; the rows outside are zero, cannot hold a peak
// and are never looked up.  Tile row r holds grid row wb - 1 + r: one zero halo row on each
// side, then the out-of-grid columns' dummy row.  The peak and dilated words stay aligned to
// the grid's 32-row words (those the window touches, plus one zero row), so retention looks
// up grid rows exactly as without a window.  An event whose hits reach beyond the window is
// left to the spill kernel (kStatusSpill).  A smaller tile lets more workgroups share a CU,
// which is what the window is for: on the paper's grid (rho range twice the reach of hits at
// 200 mm and beyond) half of the 1000 rows are enough.
// Launch bounds: a windowed tile exists to fit two or three workgroups of at most 8 waves on a
// CU, so 4 waves per SIMD are enough for it and leave it registers to spare.
template <int NW, int G, bool PER, bool SP, bool WIN>
__global__ __launch_bounds__(NW * 64, (NW == 16 || WIN) ? 4 : (G == 1 ? 6 : 4)) void k_batch(GridArgs g, BatchArgs a,
                                                                                            int n_tiles, int nwords,
                                                                                            int win) {
    using L = Lane<G, true>;
    constexpr int TW = L::TW, ST = L::STRIDE, OUT = TW - 2, NT = NW * 64;
    static_assert(!WIN || (G == 1 && !PER), "windowed tiles: one column group, theta not periodic");
    extern __shared__ __align__(16) uint32_t lds[];
    // tile rows (dummy row included) and peak-word rows of the LDS layout
    const int rows_t = WIN ? win + 3 : g.n_rho + 1;
    const int nwp = WIN ? win / 32 + 1 : nwords;
    uint32_t *tile = lds;                                                  // [rows_t * ST]
    float2 *stage = reinterpret_cast<float2 *>(tile + (size_t)rows_t * ST);   // [NW * 64]
    uint32_t *pmask = reinterpret_cast<uint32_t *>(stage + NW * 64);       // [nwp * TW]
    uint32_t *dil = pmask + (size_t)nwp * TW;                              // [(nwp + 1) * TW]
    float4 *tpk = reinterpret_cast<float4 *>(dil + (size_t)(nwp + 1) * TW);   // [kTilePeaks]
    uint32_t *colcnt = reinterpret_cast<uint32_t *>(tpk + kTilePeaks);            // [TW] peaks per column
    __shared__ uint32_t s_event, s_npeaks, s_flags, s_nvalid, s_nkept, s_max, s_minr2, s_wb, s_fit, s_edge;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const L ln(lane);
    const int tile_words4 = rows_t * ST / 4;

    // the tile is all zero at the start of every tile; the dil row past the last word is read
    // by the out-of-grid columns' dummy row and stays zero
    for (int i = threadIdx.x; i < tile_words4; i += NT)
        reinterpret_cast<uint4 *>(tile)[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int i = threadIdx.x; i < TW; i += NT) dil[nwp * TW + i] = 0u;
    for (int i = threadIdx.x; i < TW; i += NT) colcnt[i] = 0u;   // zero again after each listing
    PhaseClock pc;
    pc.start();

    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t q = atomicAdd(a.queue, 1u);
            s_event = (a.order && q < a.n_events) ? a.order[q] : q;
            s_npeaks = 0u;
            s_flags = 0u;
            s_nvalid = 0u;
            s_nkept = 0u;
            s_max = 0u;
            s_minr2 = __float_as_uint(FLT_MAX);
        }
        __syncthreads();
        pc.mark(kPhasePop);
        // wave-uniform values live in scalar registers
        const uint32_t e = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_event);
        if (e >= a.n_events) {
            pc.flush();
            if (threadIdx.x == 0 && atomicAdd(a.queue + 1, 1u) == gridDim.x - 1u) {
                __hip_atomic_store(a.queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(a.queue + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            break;
        }
        // event e of this launch is pool event ids[e] (or e itself); its keep bytes start at
        // keep_offsets[e] (or at its first hit)
        const uint32_t pe_id = (uint32_t)__builtin_amdgcn_readfirstlane((int)(a.ids ? a.ids[e] : e));
        const uint32_t h0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.offsets[pe_id]);
        const uint32_t h1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.offsets[pe_id + 1]);
        if (h1 < h0) {                       // malformed offsets: touch nothing but the counters
            if (threadIdx.x == 0) { a.n_peaks[e] = 0u; a.status[e] = HOUGH_EV_TOO_MANY_HITS; }
            __syncthreads();
            continue;
        }
        const uint32_t H = h1 - h0;
        if (H > kMaxBatchHits || H == 0u) {      // above the 16-bit counters: the spill kernel's
            uint8_t *ke = a.keep + (a.ids ? a.keep_offsets[e] : h0);
            for (uint32_t i = threadIdx.x; i < H; i += NT) ke[i] = 0u;
            if (threadIdx.x == 0) {
                a.n_peaks[e] = 0u;
                a.status[e] = H ? kStatusSpill : 0u;
                if (H && a.spill_count) atomicAdd(a.spill_count, 1u);
            }
            __syncthreads();
            continue;
        }
        const uint32_t hb = (uint32_t)((uint64_t)H * wave / NW);
        const uint32_t he = (uint32_t)((uint64_t)H * (wave + 1) / NW);
        const float *xe = a.x + h0, *ye = a.y + h0;
        hough_peak *pe = a.peaks ? a.peaks + (size_t)e * a.max_peaks : nullptr;
        const uint32_t cap = pe ? a.max_peaks : 0u;
        uint32_t bad = 0;
        uint8_t *ke = a.keep + (a.ids ? (uint32_t)__builtin_amdgcn_readfirstlane((int)a.keep_offsets[e]) : h0);
        // with duplicate suppression the duplicate pass has written every keep byte already
        if (!g.dedup) {
#pragma unroll 1
            for (uint32_t i = hb + lane; i < he; i += 64) ke[i] = 0u;
        } else if (H > kDedupMaxHits && threadIdx.x == 0) {
            atomicOr(&s_flags, HOUGH_EV_DEDUP_SKIPPED);
        }
        // the event's rho window: the smallest r2 = x^2 + y^2 among its valid hits (the same
        // float expression as the map's) bounds every bin they vote into, |t - B| <= wA / sqrt(r2)
        // with wA the largest |(C_j, S_j)|; the float map and the two fmas of t add a few 2^-24
        // relative, far inside the 1e-6 and 1e-5 margins kept here.  Rows are floor(t), so the
        // floors of the bounds are the first and last rows a vote can reach.
        int wb = 0;
        if constexpr (WIN) {
            uint32_t mn = __float_as_uint(FLT_MAX);
#pragma unroll 1
            for (uint32_t i = hb + lane; i < he; i += 64) {
                const float xi = xe[i], yi = ye[i];
                const float r2 = __builtin_fmaf(xi, xi, yi * yi);
                if (r2 > 0.0f && r2 <= FLT_MAX) mn = min(mn, __float_as_uint(r2));   // r2 > 0: bits order as values
            }
            mn = wave_min(mn);
            if (lane == 0) atomicMin(&s_minr2, mn);
            __syncthreads();
            if (threadIdx.x == 0) {
                const double rmax = (1.0 + 1e-6) / sqrt((double)__uint_as_float(s_minr2));
                const double span = g.wA * rmax, slack = 1e-5 * (fabs(g.wB) + span) + 1e-3;
                const double lo = g.wB - span - slack, hi = g.wB + span + slack;
                const double top = (double)(g.n_rho - 1);
                const int klo = lo <= 0.0 ? 0 : (lo >= top ? g.n_rho - 1 : (int)lo);
                const int khi = hi <= 0.0 ? 0 : (hi >= top ? g.n_rho - 1 : (int)hi);
                const int b0 = (klo / 16) * 16;
                s_wb = (uint32_t)b0;
                s_fit = khi < b0 + win ? 1u : 0u;
            }
            __syncthreads();
            wb = __builtin_amdgcn_readfirstlane((int)s_wb);
            if (__builtin_amdgcn_readfirstlane((int)s_fit) == 0) {
                // leave it to the spill kernel (its keep bytes are clear, or hold the duplicate
                // pass's marks, which the spill kernel reads)
                if (threadIdx.x == 0) {
                    a.n_peaks[e] = 0u;
                    a.status[e] = kStatusSpill;
                    if (a.spill_count) atomicAdd(a.spill_count, 1u);
                }
                __syncthreads();
                continue;
            }
        }
        // grid row k of the window lives in tile row k - wb + 1; grid word w of the peak and
        // dilated words in word row w - wb / 32
        uint32_t *tile_w = WIN ? tile + (ptrdiff_t)(1 - wb) * ST : tile;
        uint32_t *pmask_w = WIN ? pmask - (ptrdiff_t)(wb >> 5) * TW : pmask;
        uint32_t *dil_w = WIN ? dil - (ptrdiff_t)(wb >> 5) * TW : dil;
        const int w_lo = WIN ? (wb >> 5) : 0;
        const float dummy_row = WIN ? (float)(wb + win + 1) : -1.0f;
        uint32_t thr = g.threshold;
        if (a.frac_den) {
            // relative threshold: a first pass votes every tile only to find the event's
            // largest count (rows 0 .. n_rho-1: the dummy row is not part of the grid)
            uint32_t mloc = 0, bad0 = 0;
#pragma unroll 1
            for (int t = 0; t < n_tiles; ++t) {
                const Cols<G> cl = load_cols<G, PER>(g, t * OUT - 1, lane, ST, ln.col, dummy_row);
                (void)vote_range<G, true, PER>(tile_w, stage + wave * 64, xe, ye, hb, he, cl, ln, g, lane, bad0,
                                               g.dedup ? ke : nullptr);
                __syncthreads();
                // every tile row but the dummy one (a window's halo rows stay zero)
#pragma unroll 1
                for (int i = threadIdx.x; i < (rows_t - 1) * ST; i += NT) {
                    const uint32_t d = tile[i];
                    mloc = max(mloc, max(d & 0xffffu, d >> 16));
                    tile[i] = 0u;
                }
                for (int i = (rows_t - 1) * ST + threadIdx.x; i < rows_t * ST; i += NT) tile[i] = 0u;
                __syncthreads();
            }
            mloc = wave_max(mloc);
            if (lane == 0) atomicMax(&s_max, mloc);
            __syncthreads();
            const uint64_t rel = ((uint64_t)s_max * a.frac_num + a.frac_den - 1u) / a.frac_den;
            thr = (uint32_t)__builtin_amdgcn_readfirstlane(
                (int)min<uint64_t>(max<uint64_t>(rel, g.threshold), 0x7fffffffull));
        }
        pc.mark(kPhaseSetup);
        pc.count(kPhaseEvents, 1u);
        Pending pd;
        pd.idx = 0u;
        pd.live = 0ull;
        pd.on = false;
        uint32_t unkept = he - hb;           // this wave's unkept hits after its last full pass
        // Deferred retention: peaks [def0, def0 + defn) of the event's list still have to keep
        // their hits.  flush() tests every unkept hit against them, 64 peaks at a time staged in
        // the tile's peak list (wave 0 reads the records back, then every wave tests its own
        // hits), and drops the pending lists (their entries may have been kept meanwhile).
        // (only where the launch bound leaves registers for it: windowed and 16-wave kernels)
        constexpr bool DEF = SP && (WIN || NW == 16);
        uint32_t def0 = 0, defn = 0;
        auto flush = [&]() {
            for (uint32_t b = 0; b < defn; b += kTilePeaks) {
                const uint32_t nb = min(kTilePeaks, defn - b);
                if (wave == 0) {
                    bool near = false;
                    if ((uint32_t)lane < nb) {
                        const uint64_t rec = __hip_atomic_load(
                            reinterpret_cast<const uint64_t *>(pe + def0 + b + (uint32_t)lane), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
                        const int j = (int)(rec & 0xffffu), k = (int)((rec >> 16) & 0xffffu);
                        tpk[lane] = make_float4(g.C[j], g.S[j], __int_as_float(k - g.rho_window), 0.0f);
                        near = k <= g.rho_window || k >= g.n_rho - g.rho_window;
                    }
                    const uint64_t nm = __ballot(near);
                    if (lane == 0) s_edge = nm ? 1u : 0u;
                }
                __syncthreads();
                uint32_t left = 0;
                const uint32_t newly = retain_range_peaks(tpk, nb, s_edge != 0u, xe, ye, ke, hb, he, g, lane, left);
                if (lane == 0 && newly) atomicAdd(&s_nkept, newly);
                unkept = left;
                __syncthreads();
            }
            defn = 0;
            pd.on = false;
            pd.live = 0ull;
        };
        // sparse event (under a quarter of the threshold per cell on average): most peak units
        // hold no count that reaches it, so each unit is first tested whole (unit_below)
        const bool sparse_ev = SP && (uint64_t)H * 4u < (uint64_t)thr * (uint32_t)g.n_rho;
        for (int t = 0; t < n_tiles; ++t) {
            const int first = t * OUT - 1;      // grid column of lane 0 of group 0
            const Cols<G> cl = load_cols<G, PER>(g, first, lane, ST, ln.col, dummy_row);
            const uint32_t nv = vote_range<G, true, PER>(tile_w, stage + wave * 64, xe, ye, hb, he, cl, ln, g, lane,
                                                         bad, g.dedup ? ke : nullptr);
            if (t == 0 && lane == 0 && nv) atomicAdd(&s_nvalid, nv);
            __syncthreads();
            pc.mark(kPhaseVote);
            if (t == 0) pc.count(kPhaseStagedHits, (uint64_t)s_nvalid * (uint64_t)n_tiles);
            // 16-row units of grid rows; a windowed tile tests the units inside its window (the
            // halo rows above and below are in the tile, so no unit needs bounds tests) and
            // writes zero for the other halves of the words it touches
            for (int u = 2 * w_lo + wave; u < 2 * (w_lo + nwp); u += NW) {
                uint32_t m[G];
                const bool interior = WIN || (u >= 1 && (u + 1) * kPeakRows < g.n_rho);
                constexpr bool UR = NW == 16 || WIN;     // launch bound of 4 waves per SIMD: registers to spare
                if ((WIN && (u * kPeakRows < wb || (u + 1) * kPeakRows > wb + win)) ||
                    (sparse_ev && interior && !(PER && (t == 0 || t == n_tiles - 1)) && unit_below<G>(tile_w, u, thr, lane))) {
#pragma unroll
                    for (int q = 0; q < G; ++q) m[q] = 0u;
                } else if (PER && (t == 0 || t == n_tiles - 1)) {
                    if (interior)
                        peak_rows<false, G, true, true, UR>(tile, u, g.n_rho, thr, ln, lane, m, first, g.n_theta);
                    else
                        peak_rows<true, G, true, true, UR>(tile, u, g.n_rho, thr, ln, lane, m, first, g.n_theta);
                } else if (interior) {
                    peak_rows<false, G, true, false, UR>(tile_w, u, g.n_rho, thr, ln, lane, m);
                } else {
                    peak_rows<true, G, true, false, UR>(tile_w, u, g.n_rho, thr, ln, lane, m);
                }
                uint16_t *pm16 = reinterpret_cast<uint16_t *>(pmask_w);
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    const int c = 64 * q + lane;
                    const bool out_col = (c >= 1) && (c <= TW - 2) && (first + c < g.n_theta);
                    pm16[((u >> 1) * TW + c) * 2 + (u & 1)] = out_col ? (uint16_t)m[q] : (uint16_t)0;
                    if (out_col && m[q]) atomicAdd(&colcnt[c], (uint32_t)__popc(m[q]));
                }
            }
            if (g.rho_window >= 32) {
#pragma unroll 1
                for (int i = threadIdx.x; i < nwp * TW; i += NT) dil[i] = 0u;
            }
            if (SP && threadIdx.x == 0) s_edge = 0u;     // set by the listing for a peak near a rho edge
            __syncthreads();
            pc.mark(kPhasePeaks);
            const uint32_t base = s_npeaks;
            uint32_t np;
            if constexpr (SP)
                np = emit_and_dilate<G, true>(tile_w, pmask_w, dil_w, w_lo, nwp, first, g, pe, cap, base, ln, lane,
                                              wave, NW, tpk, &cl, colcnt, &s_edge);
            else
                np = emit_and_dilate<G, true>(tile_w, pmask_w, dil_w, w_lo, nwp, first, g, pe, cap, base, ln, lane,
                                              wave, NW, nullptr, nullptr, colcnt);
            __syncthreads();
            pc.mark(kPhaseList);
            if (threadIdx.x == 0) s_npeaks = base + np;
            for (int i = threadIdx.x; i < TW; i += NT) colcnt[i] = 0u;
            // the counts are dead: clear the tile for the next one while retention reads dil
#pragma unroll 1
            for (int i = threadIdx.x; i < tile_words4; i += NT)
                reinterpret_cast<uint4 *>(tile)[i] = make_uint4(0u, 0u, 0u, 0u);
            if (DEF && np && s_nkept < s_nvalid && pe && np <= kDeferTilePeaks && base + np <= cap &&
                defn + np <= kDeferPeaks) {
                if (defn == 0) def0 = base;          // the deferred peaks stay contiguous
                defn += np;
            } else if (np && s_nkept < s_nvalid) {
                // Few peaks: test each hit against the peak list (about 5 instructions per peak
                // for a chunk of 64 hits, kept or not; 9 when a peak lies near a rho edge) where
                // that beats looking the unkept hits up in every column's dilated words (about 7
                // per unkept hit, plus staging).  A flush of deferred peaks reuses the list's
                // storage, so after one this tile looks its hits up in the dilated words.
                bool few = SP && np <= kTilePeaks;
                const bool edge = SP && s_edge != 0u;
                if (DEF && defn) {
                    flush();
                    few = false;
                }
                const uint32_t cp = edge ? 9u : 5u;
                uint32_t newly;
                if (pd.on) {
                    const uint32_t n = (uint32_t)__popcll(pd.live);
                    newly = (few && np * cp < n * 7u + 10u)
                                ? retain_pending_peaks(pd, tpk, np, edge, xe, ye, ke, g, lane)
                                : retain_pending<G>(pd, dil_w, stage + wave * 64, xe, ye, ke, cl, g, lane);
                } else {
                    uint32_t left = 0;
                    const uint32_t chunks = (he - hb + 63u) >> 6;
                    newly = (few && np * cp * chunks < unkept * 7u + chunks * 10u)
                                ? retain_range_peaks(tpk, np, edge, xe, ye, ke, hb, he, g, lane, left)
                                : retain_range<G>(dil_w, stage + wave * 64, xe, ye, ke, hb, he, cl, g, lane, left);
                    if (SP) unkept = left;
                    if (left <= 64u) build_pending(pd, stage + wave * 64, xe, ye, ke, hb, he, lane);
                }
                if (lane == 0 && newly) atomicAdd(&s_nkept, newly);
            }
            __syncthreads();
            pc.mark(kPhaseRetain);
        }
        if (DEF && defn) {
            if (s_nkept < s_nvalid) flush();
            pc.mark(kPhaseRetain);
        }
        if (__ballot(bad != 0u) && lane == 0) atomicOr(&s_flags, HOUGH_EV_INVALID_HITS);
        if (g.dedup) {                       // drop the later-copy bit, leaving the kept bit
#pragma unroll 1
            for (uint32_t i = hb + lane; i < he; i += 64) {
                const uint32_t v = ke[i];
                if (v & kKeepDuplicate) ke[i] = (uint8_t)(v & 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t np = s_npeaks;
            a.n_peaks[e] = np;
            a.status[e] = s_flags | (np > a.max_peaks ? HOUGH_EV_PEAKS_TRUNCATED : 0u);
        }
        __syncthreads();
        pc.mark(kPhaseFinish);
    }
}

// ------------------------------------------------------------ split batch path (latency form)
// The same results as k_batch for batches small enough that latency matters more than
// throughput: the work items are the (event, theta tile) pairs, so the tiles of one event run
// on different workgroups at once.  A tile votes all of its event's hits, finds its peaks, lists
// them in raster order into its own slot of the workspace, dilates them, and sets the keep bits
// of the event's hits it keeps.  The workgroup that finishes an event's last tile merges: the
// tile lists in tile order (raster order) truncated at max_peaks, the true count, the status
// and the keep bytes, and it leaves the event's part of the workspace zero again.  Every tile
// examines all of the event's hits, so retention costs more in total than in k_batch, and
// each publish and merge is an agent-scope release or acquire: the price of the shorter
// latency.

// Step 5 of one tile in the split form: keep bits in global memory, shared by the tiles.  A
// wave tests 64 consecutive hits at a time and merges its kept bits into (at most three) words
// before it touches global memory, so that the tiles' atomics stay few.
template <int G>
__device__ void retain_split(const uint32_t *dil, float2 *st, const float *x, const float *y,
                             uint32_t *bits, uint32_t hb, uint32_t he, const Cols<G> &cl,
                             const GridArgs &g, int lane) {
    uint32_t unused = 0;
    float xn = 0.0f, yn = 0.0f;                       // the next 64 hits load while these are tested
    if (hb + lane < he) { xn = x[hb + lane]; yn = y[hb + lane]; }
    for (uint32_t base = hb; base < he; base += 64) {
        const float xi = xn, yi = yn;
        const uint32_t nb = base + 64u + (uint32_t)lane;
        if (nb < he) { xn = x[nb]; yn = y[nb]; }
        int slot;
        const StageCount n = stage_values(st, xi, yi, base + lane < he, g, unused, slot);
        const uint64_t kept = lookup_staged<G>(dil, st, n, cl, lane, g.nrho_f);
        const uint64_t m = __ballot(slot >= 0 && ((kept >> slot) & 1ull));   // bit l: hit base + l
        const uint32_t sh = base & 31u;
        if (m && lane < 3) {
            uint64_t part;                                                    // bits of word base/32 + lane
            if (lane == 0) part = m << sh;
            else if (lane == 1) part = m >> (32u - sh);
            else part = sh ? m >> (64u - sh) : 0ull;
            part &= 0xffffffffull;
            if (part) atomicOr(&bits[(base >> 5) + (uint32_t)lane], (uint32_t)part);
        }
        wave_sync();
    }
}

template <int NW, int G, bool PER>
__global__ __launch_bounds__(NW * 64, G == 1 ? 6 : 4) void k_batch_split(GridArgs g, BatchArgs a, SplitArgs sp,
                                                                         int nwords) {
    using L = Lane<G, true>;
    constexpr int TW = L::TW, ST = L::STRIDE, OUT = TW - 2, NT = NW * 64;
    extern __shared__ __align__(16) uint32_t lds[];
    uint32_t *tile = lds;                                                  // [(n_rho + 1) * ST]
    float2 *stage = reinterpret_cast<float2 *>(tile + (size_t)(g.n_rho + 1) * ST);   // [NW * 64]
    uint32_t *pmask = reinterpret_cast<uint32_t *>(stage + NW * 64);       // [nwords * TW]
    uint32_t *dil = pmask + (size_t)nwords * TW;                           // [(nwords + 1) * TW]
    __shared__ uint32_t s_item, s_flags, s_last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const L ln(lane);
    const int tile_words4 = (g.n_rho + 1) * ST / 4;
    const uint32_t T = sp.n_tiles;
    const uint32_t n_items = a.n_events * T;

    for (int i = threadIdx.x; i < tile_words4; i += NT)
        reinterpret_cast<uint4 *>(tile)[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int i = threadIdx.x; i < TW; i += NT) dil[nwords * TW + i] = 0u;

    for (;;) {
        if (threadIdx.x == 0) {
            s_item = atomicAdd(a.queue, 1u);
            s_flags = 0u;
            s_last = 0u;
        }
        __syncthreads();
        const uint32_t item = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_item);
        if (item >= n_items) {
            if (threadIdx.x == 0 && atomicAdd(a.queue + 1, 1u) == gridDim.x - 1u) {
                __hip_atomic_store(a.queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(a.queue + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            break;
        }
        const uint32_t e = item / T, t = item - e * T;
        const uint32_t pe_id = (uint32_t)__builtin_amdgcn_readfirstlane((int)(a.ids ? a.ids[e] : e));
        const uint32_t h0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.offsets[pe_id]);
        const uint32_t h1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.offsets[pe_id + 1]);
        const bool malformed = h1 < h0;
        const uint32_t H = malformed ? 0u : h1 - h0;
        uint32_t *bits = sp.kept + (size_t)e * kSplitKeepWords;
        uint8_t *ke = a.keep + (a.ids ? (uint32_t)__builtin_amdgcn_readfirstlane((int)a.keep_offsets[e]) : h0);
        if (malformed || H > kMaxBatchHits) {
            if (threadIdx.x == 0 && t == 0) {
                s_flags = HOUGH_EV_TOO_MANY_HITS;
                if (!malformed && a.spill_count) atomicAdd(a.spill_count, 1u);
            }
        } else if (H > 0) {
            if (g.dedup && H > kDedupMaxHits && threadIdx.x == 0 && t == 0) atomicOr(&s_flags, HOUGH_EV_DEDUP_SKIPPED);
            const uint32_t hb = (uint32_t)((uint64_t)H * wave / NW);
            const uint32_t he = (uint32_t)((uint64_t)H * (wave + 1) / NW);
            const float *xe = a.x + h0, *ye = a.y + h0;
            uint32_t bad = 0;
            const int first = (int)t * OUT - 1;
            const Cols<G> cl = load_cols<G, PER>(g, first, lane, ST, ln.col);
            vote_range<G, true, PER>(tile, stage + wave * 64, xe, ye, hb, he, cl, ln, g, lane, bad,
                                     g.dedup ? ke : nullptr);
            if (t == 0 && __ballot(bad != 0u) && lane == 0) atomicOr(&s_flags, HOUGH_EV_INVALID_HITS);
            __syncthreads();
            for (int u = wave; u < 2 * nwords; u += NW) {
                uint32_t m[G];
                const bool interior = u >= 1 && (u + 1) * kPeakRows < g.n_rho;
                if (PER && (t == 0 || t == T - 1)) {
                    if (interior)
                        peak_rows<false, G, true, true>(tile, u, g.n_rho, g.threshold, ln, lane, m, first, g.n_theta);
                    else
                        peak_rows<true, G, true, true>(tile, u, g.n_rho, g.threshold, ln, lane, m, first, g.n_theta);
                } else if (interior) {
                    peak_rows<false, G, true>(tile, u, g.n_rho, g.threshold, ln, lane, m);
                } else {
                    peak_rows<true, G, true>(tile, u, g.n_rho, g.threshold, ln, lane, m);
                }
                uint16_t *pm16 = reinterpret_cast<uint16_t *>(pmask);
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    const int c = 64 * q + lane;
                    const bool out_col = (c >= 1) && (c <= TW - 2) && (first + c < g.n_theta);
                    pm16[((u >> 1) * TW + c) * 2 + (u & 1)] = out_col ? (uint16_t)m[q] : (uint16_t)0;
                }
            }
            if (g.rho_window >= 32) {
#pragma unroll 1
                for (int i = threadIdx.x; i < nwords * TW; i += NT) dil[i] = 0u;
            }
            __syncthreads();
            hough_peak *slot = sp.staged + ((size_t)e * T + t) * sp.tile_cap;
            const uint32_t np = emit_and_dilate<G, true>(tile, pmask, dil, 0, nwords, first, g, slot, sp.tile_cap,
                                                         0u, ln, lane, wave, NW);
            __syncthreads();
            if (threadIdx.x == 0) sp.counts[(size_t)e * T + t] = np;
#pragma unroll 1
            for (int i = threadIdx.x; i < tile_words4; i += NT)
                reinterpret_cast<uint4 *>(tile)[i] = make_uint4(0u, 0u, 0u, 0u);
            if (np) retain_split<G>(dil, stage + wave * 64, xe, ye, bits, hb, he, cl, g, lane);
        }
        // publish this tile's results, then count it; the last tile of the event merges
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_flags) atomicOr(&sp.flags[e], s_flags);
            __threadfence();
            s_last = atomicAdd(&sp.done[e], 1u) == T - 1u ? 1u : 0u;
        }
        __syncthreads();
        if (s_last) {
            __threadfence();
            // the tile lists in tile order, 64 tiles at a time: wave 0 scans their counts into
            // pref (LDS, free now), then every thread copies peaks and clears the slots
            uint32_t *pref = pmask;
            hough_peak *pe = a.peaks ? a.peaks + (size_t)e * a.max_peaks : nullptr;
            const uint32_t cap = pe ? a.max_peaks : 0u;
            uint32_t run = 0;
            for (uint32_t t0 = 0; t0 < T; t0 += 64) {
                const uint32_t nt = T - t0 < 64u ? T - t0 : 64u;
                if (wave == 0) {
                    const uint32_t c = (uint32_t)lane < nt
                        ? __hip_atomic_load(&sp.counts[(size_t)e * T + t0 + lane], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : 0u;
                    const uint32_t incl = wave_inclusive_scan(c, lane);
                    pref[lane] = run + incl - c;
                    if (lane == 63) pref[64] = run + incl;
                }
                __syncthreads();
                const uint32_t lo_i = pref[0], hi_i = pref[64];
                for (uint32_t i = lo_i + threadIdx.x; i < hi_i; i += NT) {
                    uint32_t lo = 0, hi = nt - 1;             // the last tile whose list starts at or before i
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi + 1) >> 1;
                        if (pref[mid] <= i) lo = mid; else hi = mid - 1;
                    }
                    uint2 *src = reinterpret_cast<uint2 *>(sp.staged + ((size_t)e * T + t0 + lo) * sp.tile_cap) +
                                 (i - pref[lo]);
                    if (i < cap) reinterpret_cast<uint2 *>(pe)[i] = *src;
                    *src = make_uint2(0u, 0u);
                }
                run = hi_i;
                __syncthreads();                              // pref is rewritten by the next chunk
            }
            const uint32_t total = run;                       // the event's true peak count
            const uint32_t fl = __hip_atomic_load(&sp.flags[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!malformed) {                     // malformed offsets: touch nothing but the counters
                const bool skipped = H > kMaxBatchHits;
                for (uint32_t i = threadIdx.x; i < H; i += NT)
                    ke[i] = skipped ? (uint8_t)0 : (uint8_t)((bits[i >> 5] >> (i & 31)) & 1u);
            }
            __syncthreads();
            // leave the event's workspace zero for the next launch
            for (uint32_t i = threadIdx.x; i < (H + 31u) / 32u && i < kSplitKeepWords; i += NT) bits[i] = 0u;
            for (uint32_t tt = threadIdx.x; tt < T; tt += NT) sp.counts[(size_t)e * T + tt] = 0u;
            if (threadIdx.x == 0) {
                a.n_peaks[e] = total;
                a.status[e] = fl | (total > a.max_peaks ? HOUGH_EV_PEAKS_TRUNCATED : 0u);
                sp.flags[e] = 0u;
                sp.done[e] = 0u;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ spill path (rho slabs)
// Events whose accumulator the fused kernel cannot hold on chip: every event of a theta-periodic
// grid whose rho column is taller than the fused kernel's LDS tile, events whose hits reach
// beyond a windowed tile, every event of the split forms on such grids, and events above
// kMaxBatchHits hits on any grid (counts beyond 16 bits).  One workgroup processes one event at
// a time:
//   - steps 1-4 one slab at a time in LDS (62 owned columns with halo lanes by up to 1,120 owned
//     rows with halo rows; 32-bit counts and 544 rows for events above 65,535 hits): vote, then
//     the 3x3 test of every owned cell, which leaves each (column, 32-row block) its peak rows
//     as a bit mask and each peak's count in device memory; the accumulator stays on chip;
//   - a thread per column places each block's peaks within its column, a scan over the columns
//     gives raster order, and the listing pass writes the peaks and marks the dilated retention
//     bits D[w * n_theta + j] (bit b: a peak of column j within rho_window rows of row 32w + b);
//   - retention stages one 64-column group of D in LDS at a time and looks the event's hits up
//     in it, lane = column.
// Every (group, slab) maps all of the event's hits again, so this path is for what the fused
// kernel cannot take, not a fast path.
constexpr int kSpillWaves = 16;
constexpr int kSpillThreads = kSpillWaves * 64;
constexpr uint32_t kSpillBlock = 4;      // events per counter pop when only some events spill
// the slab: 143 KB of dynamic LDS, what the CU's 160 KB leave beside the kernel's static LDS
// (slabs of 1,024 rows split a 2,000-row column into three, 3.4 against 4.1 ms per 1,000
// events on 1000 x 2000 bins)
constexpr int kSpillSlabDwords = 36608;
constexpr int kSpillOwnedPacked = 1120;  // owned rows of a packed slab: 35 blocks + 2 halo rows <= 1,144
constexpr int kSpillOwnedWide = 544;     // owned rows of a 32-bit slab: 17 blocks + 2 halo rows <= 572

// A word of the dilated bits (ORed by atomics in L2) or a peak's count in the accumulator,
// read past the L1.
__device__ __forceinline__ uint32_t spill_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The spill kernel's device memory belongs to one workgroup, so workgroup scope orders it: the
// release waits for this wave's stores and atomics, the barrier lines the waves up.  The waves
// of a workgroup share one L1, which their plain stores go through; the dilation's atomic ORs
// are performed beyond it (in L2), so the dilated bits, and the peak counts with them, are read
// with loads that bypass the L1 (spill_load).  (Agent-scope fences here wrote back the whole
// L2 at every barrier: with many workgroups spilling at once that took most of the kernel's
// time.)
__device__ __forceinline__ void spill_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The spill kernel's LDS slab: one group of up to 62 owned columns with a halo lane on each
// side (lane l holds column first + l - 1; on a theta-periodic grid the halo beyond either edge
// holds the wrapped column with rho reversed, as in the fused kernel) and owned rows [ro, ro1)
// with one halo row on each side (slab row i holds grid row ro - 1 + i).  P: two 16-bit counts
// per dword (events of at most 65,535 hits), else one 32-bit count per cell.
template <bool P>
struct SpillSlab {
    const uint32_t *tile;
    static constexpr int STRIDE = Lane<1, P>::STRIDE;      // dwords per slab row
    __device__ __forceinline__ uint32_t count(int l, int i) const {
        if (P) return (tile[i * STRIDE + (l & 31)] >> (16 * (l >> 5))) & 0xffffu;
        return tile[i * STRIDE + l];
    }
};

// Steps 1-3 into the slab: votes of hits [hb, he) by the whole-grid rule (bin k of the lane's
// column, a wrapped halo lane taking row n_rho - 1 - k), kept when r0 <= k < r1, at slab row
// k - base.  dup as for vote_range.
template <bool P>
__device__ void spill_vote_slab(uint32_t *tile, float2 *st, const float *x, const float *y, uint32_t hb,
                                uint32_t he, const Cols<1> &cl, bool wrap, const GridArgs &g, int lane,
                                uint32_t &bad, const uint8_t *dup, int r0, int r1, int base) {
    const Lane<1, P> ln(lane);
    for (uint32_t b0 = hb; b0 < he; b0 += 64) {
        const uint32_t i = b0 + lane;
        bool live = i < he;
        float xi = 0.0f, yi = 0.0f;
        if (live) { xi = x[i]; yi = y[i]; }
        if (dup && live && (dup[i] & kKeepDuplicate)) live = false;
        int slot;
        const StageCount n = stage_values(st, xi, yi, live, g, bad, slot);
#pragma unroll 4
        for (uint32_t h = 0; h < n.total; ++h) {
            const float2 p = st[h];
            const float t = __builtin_fmaf(p.x, cl.C[0], __builtin_fmaf(p.y, cl.S[0], cl.B[0]));
            if (t >= 0.0f && t < g.nrho_f) {
                const int k = wrap ? g.n_rho - 1 - (int)t : (int)t;
                if (k >= r0 && k < r1) lds_add(&tile[(k - base) * Lane<1, P>::STRIDE + (int)ln.col[0]], ln.inc);
            }
        }
        wave_sync();
    }
}

// Step 4 on rows [k0, k1) of slab lane l (owned column j): bit k - k0 of the result is set iff
// cell (j, k) is a peak, and the i-th peak's count is stored to pc[i] for the listing pass (a
// block holds at most 16 peaks: of two vertically adjacent cells the later one must exceed the
// earlier, the earlier must not fall below the later, so not both are peaks).  Raster
// order: the column before (j - 1) and the row above come first, except that on a periodic
// grid the wrapped column left of column 0 comes later and the one right of the last column
// earlier; rows outside the grid are the slab's zero halo rows.
template <bool P>
__device__ uint32_t spill_slab_peaks(const SpillSlab<P> &s, int l, int j, int k0, int k1, int base,
                                     uint32_t thr, const GridArgs &g, uint32_t *pc) {
    const bool left_later = g.periodic && j == 0, right_earlier = g.periodic && j == g.n_theta - 1;
    int i = k0 - base;
    uint32_t l0 = s.count(l - 1, i - 1), c0 = s.count(l, i - 1), r0 = s.count(l + 1, i - 1);
    uint32_t l1 = s.count(l - 1, i), c1 = s.count(l, i), r1 = s.count(l + 1, i);
    uint32_t m = 0;
    for (int k = k0; k < k1; ++k, ++i) {
        const uint32_t l2 = s.count(l - 1, i + 1), c2 = s.count(l, i + 1), r2 = s.count(l + 1, i + 1);
        if (c1 >= thr) {
            const uint32_t lm = max(max(l0, l1), l2), rm = max(max(r0, r1), r2);
            const uint32_t before = max(max(left_later ? 0u : lm, right_earlier ? rm : 0u), c0);
            const uint32_t after = max(max(left_later ? lm : 0u, right_earlier ? 0u : rm), c2);
            if (c1 >= max(before + 1u, after)) {
                pc[__popc(m)] = c1;
                m |= 1u << (k - k0);
            }
        }
        l0 = l1; l1 = l2;
        c0 = c1; c1 = c2;
        r0 = r1; r1 = r2;
    }
    return m;
}

// Every (group, slab) of the grid in turn: clear the slab, vote the event's hits into it (wave
// w maps its slice of the hits), then f(slab, first owned column, ro, ro1, base) between
// barriers.
template <bool P, typename F>
__device__ void spill_for_slabs(uint32_t *tile, float2 *st, const float *x, const float *y, uint32_t H,
                                const GridArgs &g, int lane, int wave, uint32_t &bad, const uint8_t *dup, F &&f) {
    constexpr int owned = P ? kSpillOwnedPacked : kSpillOwnedWide;
    constexpr int stride = Lane<1, P>::STRIDE;
    const Lane<1, P> ln(lane);
    const uint32_t hb = (uint32_t)((uint64_t)H * wave / kSpillWaves);
    const uint32_t he = (uint32_t)((uint64_t)H * (wave + 1) / kSpillWaves);
    for (int jo = 0; jo < g.n_theta; jo += 62) {
        const int j = jo - 1 + lane;
        const bool wrap = g.periodic && (j == -1 || j == g.n_theta);
        const Cols<1> cl = g.periodic ? load_cols<1, true>(g, jo - 1, lane, stride, ln.col)
                                      : load_cols<1, false>(g, jo - 1, lane, stride, ln.col);
        for (int ro = 0; ro < g.n_rho; ro += owned) {
            const int ro1 = min(ro + owned, g.n_rho), base = ro - 1, rows = ro1 - ro + 2;
            for (int i = threadIdx.x; i < rows * stride / 4; i += kSpillThreads)
                reinterpret_cast<uint4 *>(tile)[i] = make_uint4(0u, 0u, 0u, 0u);
            __syncthreads();
            spill_vote_slab<P>(tile, st, x, y, hb, he, cl, wrap, g, lane, bad, dup, max(ro - 1, 0),
                               min(ro1 + 1, g.n_rho), base);
            __syncthreads();
            f(SpillSlab<P>{tile}, jo, ro, ro1, base);
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kSpillThreads) void k_spill(GridArgs g, BatchArgs a, SpillArgs sp) {
    extern __shared__ __align__(16) uint32_t spill_tile[];      // [kSpillSlabDwords]
    __shared__ float2 stage[kSpillWaves][64];
    __shared__ uint32_t s_event, s_flags, s_max, s_n, s_list[kSpillThreads], s_part[kSpillThreads];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int words = (g.n_rho + 31) / 32;
    uint32_t *dil = sp.work + (size_t)blockIdx.x * sp.stride;   // [words][n_theta]
    // Work items are (column, 32-row block) pairs, item it = block it / n_theta of column
    // it mod n_theta; the per-item arrays are stored in item order
    const int n_items = g.n_theta * words;
    uint32_t *pmask = dil + (size_t)words * g.n_theta;    // [n_items] each block's peak rows
    uint32_t *colpos = pmask + n_items;                   // [n_items] its first peak's place in its column
    uint32_t *colstart = colpos + n_items;                // [n_theta + 1] each column's first peak
    uint32_t *pcount = colstart + g.n_theta + 1;          // [n_items][16] its peaks' counts

    // Every value that steers control flow around a barrier is wave-uniform (scalar), and an
    // event that is skipped passes a barrier before it returns, as a processed one does at its
    // end.  Without that barrier the compiler sends the lanes other than thread 0 straight
    // from the return to the next event's first barrier (the counter read is thread 0's alone),
    // so a wave splits: thread 0's lane waits to take the counter while the rest of the wave,
    // and the other waves, go round the barriers again on the old event index.
    auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
    auto process = [&](uint32_t e) {
        const uint32_t pe_id = uni(a.ids ? a.ids[e] : e);
        const uint32_t h0 = uni(a.offsets[pe_id]), h1 = uni(a.offsets[pe_id + 1]);
        if (h1 <= h0) {                      // malformed offsets: touch nothing but the counters
            if (threadIdx.x == 0) { a.n_peaks[e] = 0u; a.status[e] = h1 < h0 ? HOUGH_EV_TOO_MANY_HITS : 0u; }
            __syncthreads();
            return;
        }
        const uint32_t H = h1 - h0;
        uint8_t *ke = a.keep + (a.ids ? uni(a.keep_offsets[e]) : h0);
        const float *xe = a.x + h0, *ye = a.y + h0;
        // the duplicate pass marked later copies in the keep bytes of events up to kDedupMaxHits
        const bool dup = g.dedup && H <= kDedupMaxHits;
        if (threadIdx.x == 0) {
            s_flags = (g.dedup && H > kDedupMaxHits) ? HOUGH_EV_DEDUP_SKIPPED : 0u;
            s_max = 0u;
        }
        if (!dup)
            for (uint32_t i = threadIdx.x; i < H; i += kSpillThreads) ke[i] = 0u;
        for (size_t i = threadIdx.x; i < (size_t)words * g.n_theta; i += kSpillThreads) dil[i] = 0u;
        spill_sync();

        // steps 1-4 on chip, one slab at a time: vote, then the 3x3 test of every owned cell,
        // giving each (column, 32-row block) item its peak rows as a bit mask (stored in item
        // order: neighbouring threads take neighbouring columns) and its peaks' counts.
        // Only peak cells reach device memory (writing the whole accumulator out and walking it
        // there was three quarters of the path's time).  The relative threshold needs the
        // event's largest count first: one more round of votes.
        uint32_t bad = 0;
        uint32_t thr = g.threshold;
        const uint8_t *dupk = dup ? ke : nullptr;
        auto slabs = [&](auto packed) {
            constexpr bool P = decltype(packed)::value;
            if (a.frac_den) {
                spill_for_slabs<P>(spill_tile, &stage[wave][0], xe, ye, H, g, lane, wave, bad, dupk,
                                   [&](const SpillSlab<P> &sl, int, int ro, int ro1, int) {
                    uint32_t m = 0;
                    for (int i = threadIdx.x; i < (ro1 - ro + 2) * SpillSlab<P>::STRIDE; i += kSpillThreads) {
                        const uint32_t v = sl.tile[i];
                        m = max(m, P ? max(v & 0xffffu, v >> 16) : v);
                    }
                    m = wave_max(m);
                    if (lane == 0) atomicMax(&s_max, m);
                });
                const uint64_t rel = ((uint64_t)uni(s_max) * a.frac_num + a.frac_den - 1u) / a.frac_den;
                thr = (uint32_t)min<uint64_t>(max<uint64_t>(rel, g.threshold), 0x7fffffffull);
            }
            spill_for_slabs<P>(spill_tile, &stage[wave][0], xe, ye, H, g, lane, wave, bad, dupk,
                               [&](const SpillSlab<P> &sl, int jo, int ro, int ro1, int base) {
                const int nl = min(62, g.n_theta - jo), nb = (ro1 - ro + 31) / 32;
                for (int t = threadIdx.x; t < nl * nb; t += kSpillThreads) {
                    const int bs = t / nl, l = 1 + (t - bs * nl), j = jo + l - 1;
                    const int k0 = ro + 32 * bs, k1 = min(k0 + 32, ro1);
                    const int it = (k0 >> 5) * g.n_theta + j;
                    pmask[it] = spill_slab_peaks<P>(sl, l, j, k0, k1, base, thr, g, pcount + (size_t)it * 16);
                }
            });
        };
        if (H <= 65535u) slabs(std::true_type{});
        else slabs(std::false_type{});
        if (__ballot(bad != 0u) && lane == 0) atomicOr(&s_flags, HOUGH_EV_INVALID_HITS);
        spill_sync();
        // raster order is column-major with rows in order within a column: a thread per column
        // places each block's peaks within the column (neighbouring threads, neighbouring
        // columns: coalesced), then an exclusive prefix over the columns' totals (each thread
        // sums a run of columns, the runs' totals are scanned, then each run is scanned again)
        for (int j = threadIdx.x; j < g.n_theta; j += kSpillThreads) {
            uint32_t in_col = 0;
            for (int b = 0; b < words; ++b) {
                colpos[b * g.n_theta + j] = in_col;
                in_col += (uint32_t)__popc(pmask[b * g.n_theta + j]);
            }
            colstart[j] = in_col;
        }
        spill_sync();
        const int per = (g.n_theta + kSpillThreads - 1) / kSpillThreads;
        const int c0 = min((int)threadIdx.x * per, g.n_theta), c1 = min(c0 + per, g.n_theta);
        uint32_t part = 0;
        for (int j = c0; j < c1; ++j) part += colstart[j];
        s_part[threadIdx.x] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (int t = 0; t < kSpillThreads; ++t) {
                const uint32_t v = s_part[t];
                s_part[t] = run;
                run += v;
            }
            s_n = run;
        }
        __syncthreads();
        uint32_t run = s_part[threadIdx.x];
        for (int j = c0; j < c1; ++j) {
            const uint32_t v = colstart[j];
            colstart[j] = run;
            run += v;
        }
        spill_sync();
        // second pass: list each block's peaks in row order at its position, and mark the rows
        // within rho_window of each peak in the column's dilated bits (words other blocks of the
        // column may mark too: atomic ORs, in L2)
        hough_peak *pe = a.peaks ? a.peaks + (size_t)e * a.max_peaks : nullptr;
        const uint32_t cap = pe ? a.max_peaks : 0u;
        for (int it = threadIdx.x; it < n_items; it += kSpillThreads) {
            const int b = it / g.n_theta, j = it - b * g.n_theta;
            uint32_t pos = colstart[j] + colpos[it];
            const uint32_t *pc = pcount + (size_t)it * 16;
            uint32_t r = 0;
            for (uint32_t m = pmask[it]; m; m &= m - 1u) {
                const int k = 32 * b + (__ffs(m) - 1);
                if (pos < cap) store_peak(pe + pos, (uint32_t)j, (uint32_t)k, spill_load(pc + r));
                ++pos;
                ++r;
                const int lo = max(k - g.rho_window, 0), hi = min(k + g.rho_window, g.n_rho - 1);
                for (int wd = lo >> 5; wd <= (hi >> 5); ++wd) {
                    const int b0 = max(lo, wd * 32) - wd * 32, b1 = min(hi, wd * 32 + 31) - wd * 32;
                    const uint32_t msk = (b1 == 31 ? 0xffffffffu : ((1u << (b1 + 1)) - 1u)) & ~((1u << b0) - 1u);
                    __hip_atomic_fetch_or(dil + (size_t)wd * g.n_theta + j, msk, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        spill_sync();

        // step 5, one 64-column group at a time: the group's dilated words are staged in LDS
        // (the vote's slab space), then each wave looks its hits, 64 at a time, up in every
        // column of the group (lane = column, the fused kernel's lookup); a hit kept by one
        // group is not looked up again.  Bit 0 of a keep byte is the verdict; a later copy's
        // bit 1 (duplicate pass) is dropped at the end.
        const uint32_t n_peaks = uni(s_n);
        if (n_peaks > 0) {
            const Lane<1, true> ln(lane);
            uint32_t unused = 0;
            for (int j0 = 0; j0 < g.n_theta; j0 += 64) {
                // [words + 1][64]: the extra zero row is where out-of-grid lanes look
                for (int q = threadIdx.x; q < (words + 1) * 64; q += kSpillThreads) {
                    const int w = q >> 6, c = j0 + (q & 63);
                    spill_tile[q] = (w < words && c < g.n_theta) ? spill_load(dil + (size_t)w * g.n_theta + c) : 0u;
                }
                __syncthreads();
                const Cols<1> cl = load_cols<1>(g, j0, lane, Lane<1, true>::STRIDE, ln.col);
                for (uint32_t base = (uint32_t)wave * 64; base < H; base += kSpillThreads) {
                    const uint32_t i = base + lane;
                    const uint32_t kv = i < H ? ke[i] : 1u;
                    const bool done = i < H && (kv & 1u);
                    if (__ballot(i < H && !done) == 0ull) continue;
                    int slot;
                    const StageCount n = stage_hits(&stage[wave][0], xe, ye, base, H, done, g, lane, unused, slot);
                    const uint64_t kept = lookup_staged<1>(spill_tile, &stage[wave][0], n, cl, lane, g.nrho_f);
                    if (slot >= 0 && ((kept >> slot) & 1ull)) ke[i] = (uint8_t)(kv | 1u);
                    wave_sync();
                }
                __syncthreads();
            }
            for (uint32_t i = threadIdx.x; i < H; i += kSpillThreads) ke[i] = (uint8_t)(ke[i] & 1u);
        } else if (dup) {
            for (uint32_t i = threadIdx.x; i < H; i += kSpillThreads) ke[i] = 0u;
        }
        spill_sync();
        if (threadIdx.x == 0) {
            a.n_peaks[e] = n_peaks;
            a.status[e] = s_flags | (n_peaks > a.max_peaks ? HOUGH_EV_PEAKS_TRUNCATED : 0u);
        }
        __syncthreads();
    };

    if (sp.all) {
        for (;;) {
            if (threadIdx.x == 0) s_event = atomicAdd(sp.queue, 1u);
            __syncthreads();
            const uint32_t e = uni(s_event);
            __syncthreads();
            if (e >= a.n_events) break;
            process(e);
        }
        if (threadIdx.x == 0 && atomicAdd(sp.queue + 1, 1u) == gridDim.x - 1u) {
            __hip_atomic_store(sp.queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(sp.queue + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    // only the events the fused or split kernel left (sp.queue[0] counts them; none: nothing to
    // scan): the workgroups take blocks of kSpillBlock events from a counter (sp.queue[2]) and
    // process the left ones of each block, so that a batch whose events mostly spill (a window
    // its events do not fit) keeps every workgroup busy.  The last workgroup to leave clears
    // the count and both counters.
    if (threadIdx.x == 0) s_n = __hip_atomic_load(sp.queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const bool any = uni(s_n) != 0u;
    __syncthreads();
    while (any) {
        if (threadIdx.x == 0) {
            s_event = atomicAdd(sp.queue + 2, 1u);
            s_n = 0u;
        }
        __syncthreads();
        const uint32_t b0 = uni(s_event) * kSpillBlock;
        if (b0 >= a.n_events) break;                   // every thread leaves together
        const uint32_t e = b0 + threadIdx.x;
        if (threadIdx.x < kSpillBlock && e < a.n_events) {
            const uint32_t pe_id = a.ids ? a.ids[e] : e;
            const uint32_t h0 = a.offsets[pe_id], h1 = a.offsets[pe_id + 1];
            // left here by the fused kernel (kStatusSpill), or by the split form (above its limit)
            if ((a.status[e] & kStatusSpill) || (h1 >= h0 && h1 - h0 > kMaxBatchHits)) s_list[atomicAdd(&s_n, 1u)] = e;
        }
        __syncthreads();
        const uint32_t n = uni(s_n);
        for (uint32_t p = 0; p < n; ++p) process(uni(s_list[p]));   // events are independent: any order
        __syncthreads();
    }
    if (threadIdx.x == 0 && atomicAdd(sp.queue + 1, 1u) == gridDim.x - 1u) {
        __hip_atomic_store(sp.queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(sp.queue + 2, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(sp.queue + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------ duplicate pass (HOUGH_FLAG_DEDUP)
// One workgroup per event.  Open addressing in LDS keyed by the bits of (x, y): every slot ends
// holding the smallest event-local index of its key (compare-and-swap into an empty slot, atomic
// min into a slot of the same key), so after the inserts a hit is a later copy iff the slot of
// its key holds another index.  The table has at least twice as many slots as hits, so every
// probe sequence meets its key or an empty slot; entries never empty again, so a lookup finds
// its key before any empty slot.  The probe loops are bounded by the table size all the same.
constexpr int kDedupThreads = 512;
constexpr uint32_t kEmptySlot = 0xffffffffu;

// ------------------------------------------------------------------ largest-first schedule
// Size class of an event of H hits, non-decreasing in H: H itself below 64, else the octave
// of H and its next six bits (classes of 1/64 of an octave), at most 1727.  Malformed events
// (offsets decreasing) count as empty.
__device__ __forceinline__ uint32_t size_class(const uint32_t *offsets, uint32_t e) {
    const uint32_t h0 = offsets[e], h1 = offsets[e + 1];
    const uint32_t H = h1 >= h0 ? h1 - h0 : 0u;
    if (H < 64u) return H;
    const uint32_t lg = 31u - (uint32_t)__builtin_clz(H);
    return ((lg - 5u) << 6) | ((H >> (lg - 6u)) & 63u);
}

constexpr int kOrderThreads = 1024;
constexpr int kOrderClasses = 2048;

// One workgroup: count the events of each size class, turn the counts into the first queue
// position of each class (largest class first) and scatter the event indices there.  Within a
// class the order is whatever the LDS atomics give.
__global__ __launch_bounds__(kOrderThreads) void k_order(const uint32_t *__restrict__ offsets, uint32_t n_events,
                                                          uint32_t *__restrict__ order) {
    __shared__ uint32_t cnt[kOrderClasses];
    for (int i = threadIdx.x; i < kOrderClasses; i += kOrderThreads) cnt[i] = 0u;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < n_events; e += kOrderThreads)
        atomicAdd(&cnt[kOrderClasses - 1 - size_class(offsets, e)], 1u);
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint32_t c[kOrderClasses / 64], sum = 0;
#pragma unroll
        for (int i = 0; i < kOrderClasses / 64; ++i) { c[i] = cnt[lane * (kOrderClasses / 64) + i]; sum += c[i]; }
        uint32_t start = wave_inclusive_scan(sum, lane) - sum;
#pragma unroll
        for (int i = 0; i < kOrderClasses / 64; ++i) {
            cnt[lane * (kOrderClasses / 64) + i] = start;
            start += c[i];
        }
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < n_events; e += kOrderThreads)
        order[atomicAdd(&cnt[kOrderClasses - 1 - size_class(offsets, e)], 1u)] = e;
}

__device__ __forceinline__ uint32_t dedup_hash(uint32_t kx, uint32_t ky) {
    uint32_t h = kx * 0x9e3779b1u;
    h ^= ky + 0x7f4a7c15u + (h << 6) + (h >> 2);
    h *= 0x85ebca6bu;
    return h ^ (h >> 16);
}

// Slot word: the index of the first copy seen so far (low kDedupIdxBits) under 18 bits of the
// key's hash, so that a probe that meets another key's slot is settled in LDS; only equal
// fingerprints read the two hits back to compare the keys.  Among entries of one key the high
// bits are equal, so an atomic minimum over the word is one over the index.
constexpr uint32_t kDedupIdxBits = 14;
constexpr uint32_t kDedupIdxMask = (1u << kDedupIdxBits) - 1u;
static_assert(kDedupMaxHits <= kDedupIdxMask, "hit indices must fit below the fingerprint");

__global__ __launch_bounds__(kDedupThreads) void k_dedup(BatchArgs a) {
    __shared__ uint32_t tab[kDedupSlots];
    const uint32_t e = blockIdx.x;
    const uint32_t pe_id = a.ids ? a.ids[e] : e;
    const uint32_t h0 = a.offsets[pe_id], h1 = a.offsets[pe_id + 1];
    if (h1 < h0) return;                                   // malformed: the batch kernel flags it
    const uint32_t H = h1 - h0;
    if (H == 0 || H > kMaxBatchHits) return;               // too many: the batch kernel zeroes keep
    uint8_t *ke = a.keep + (a.ids ? a.keep_offsets[e] : h0);
    const uint32_t *xb = reinterpret_cast<const uint32_t *>(a.x) + h0;
    const uint32_t *yb = reinterpret_cast<const uint32_t *>(a.y) + h0;
    if (H > kDedupMaxHits) {                               // every hit votes
        for (uint32_t i = threadIdx.x; i < H; i += kDedupThreads) ke[i] = 0u;
        return;
    }
    uint32_t slots = 64;
    while (slots < 2 * H) slots <<= 1;                     // <= kDedupSlots
    const uint32_t mask = slots - 1;
    for (uint32_t q = threadIdx.x; q < slots; q += kDedupThreads) tab[q] = kEmptySlot;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < H; i += kDedupThreads) {
        const uint32_t kx = xb[i], ky = yb[i];
        const uint32_t hsh = dedup_hash(kx, ky);
        const uint32_t fp = hsh >> kDedupIdxBits, word = (fp << kDedupIdxBits) | i;
        uint32_t q = hsh & mask;
        for (uint32_t probe = 0; probe < slots; ++probe, q = (q + 1) & mask) {
            const uint32_t cur = atomicCAS(&tab[q], kEmptySlot, word);
            if (cur == kEmptySlot) break;                  // first of its key so far
            if ((cur >> kDedupIdxBits) == fp) {
                const uint32_t j = cur & kDedupIdxMask;
                if (xb[j] == kx && yb[j] == ky) {
                    atomicMin(&tab[q], word);
                    break;
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < H; i += kDedupThreads) {
        const uint32_t kx = xb[i], ky = yb[i];
        const uint32_t hsh = dedup_hash(kx, ky);
        const uint32_t fp = hsh >> kDedupIdxBits;
        uint32_t q = hsh & mask, first = i;
        for (uint32_t probe = 0; probe < slots; ++probe, q = (q + 1) & mask) {
            const uint32_t cur = tab[q];
            if (cur == kEmptySlot) break;                  // cannot happen: every key was inserted
            if ((cur >> kDedupIdxBits) != fp) continue;
            const uint32_t j = cur & kDedupIdxMask;
            if (j == i) break;                             // its own slot: the first copy
            if (xb[j] == kx && yb[j] == ky) {
                first = j;
                break;
            }
        }
        ke[i] = first != i ? kKeepDuplicate : (uint8_t)0;
    }
}

// hough_retain's LDS: the wave stages, then the dilated bits of a block of theta rows (a whole
// number of 64-row groups, at most 60 KB of them).
constexpr int kRetainWaves = 8;
int retain_rows_per_block(const GridArgs &g) {
    const size_t words = (size_t)(g.n_rho + 31) / 32;
    const size_t budget = 60 * 1024;
    int groups = (int)(budget / (words * 64 * 4));
    const int need = (g.n_theta + 63) / 64;
    if (groups > need) groups = need;
    if (groups < 1) groups = 1;
    return groups * 64;
}
size_t retain_lds_bytes(const GridArgs &g, int rows) {
    const size_t words = (size_t)(g.n_rho + 31) / 32;
    return (size_t)kRetainWaves * 64 * sizeof(float2) + (size_t)(rows / 64) * words * 64 * 4;
}

constexpr int kVoteWaves = 16;
constexpr int kPeakWaves = kPeakRowsPerBlock;

// The dynamic-LDS limit is a per-kernel, process-wide attribute: every kernel is allowed the
// device maximum (less room for its static LDS) so that contexts with different grids, possibly
// on different host threads, never lower each other's limit.
template <typename K>
void allow_lds(K kernel) {
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim - 256);
}

}  // namespace

size_t vote_lds_bytes(int rows) {
    return (size_t)(rows + 1) * 32 * 4 + (size_t)kVoteWaves * kStageBytes + 256;
}

int vote_slab_rows(int n_rho, size_t lds_limit) {
    const size_t fixed = (size_t)kVoteWaves * kStageBytes + 256 + 256;    // stages, slack, static LDS
    if (lds_limit <= fixed + 2 * 128) return 0;
    const long rows = (long)((lds_limit - fixed) / 128) - 1;
    return (int)(rows < n_rho ? rows : n_rho);
}

size_t peaks_lds_bytes(int n_rho, int waves) { return (size_t)(waves + 2) * n_rho * 4 + 256; }

int peak_block_waves(int n_rho, size_t lds_limit) {
    for (int w = kPeakWaves; w >= 2; w >>= 1)
        if (peaks_lds_bytes(n_rho, w) + 256 <= lds_limit) return w;
    return 0;
}

// The fused kernel's dynamic LDS: the packed tile with its dummy row (a windowed tile: `win`
// rows, a zero halo row on each side and the dummy row), the wave stages, the peak and dilated
// words, the tile's peak list and the per-column peak counts.
size_t batch_lds_bytes(int n_rho, int waves, int groups, int win) {
    const size_t tw = 64u * groups;
    const size_t rows = win ? (size_t)win + 3 : (size_t)n_rho + 1;
    const size_t nwords = win ? (size_t)win / 32 + 1 : (size_t)(n_rho + 31) / 32;
    return rows * (tw / 2) * 4 + (size_t)waves * kStageBytes + nwords * tw * 4 + (nwords + 1) * tw * 4 +
           kTilePeaks * sizeof(float4) + tw * 4;
}

int plan_batch(int n_theta, int n_rho, int waves, int groups, size_t lds_limit, BatchPlan *out, int win,
               bool need_split) {
    if (!(waves == 4 || waves == 6 || waves == 8 || waves == 12 || waves == 16) || !(groups == 1 || groups == 2)) return -1;
    // a window is a whole number of 32-row words, one column group, shorter than the grid
    if (win != 0 && (groups != 1 || win < 32 || win % 32 != 0 || win >= n_rho)) return -1;
    BatchPlan p{};
    p.waves = waves;
    p.groups = groups;
    p.tile_cols = 64 * groups;
    p.out_cols = p.tile_cols - 2;
    p.n_tiles = (n_theta + p.out_cols - 1) / p.out_cols;
    p.win = win;
    p.lds_bytes = batch_lds_bytes(n_rho, waves, groups, win);
    p.split_lds_bytes = batch_lds_bytes(n_rho, waves, groups, 0);
    p.sparse = n_rho >= kSparseRhoRows ? 1 : 0;
    // room for the kernel's static LDS; the split form always holds the whole column (grids
    // taller than that run their split calls through the spill kernel: need_split false)
    if (p.lds_bytes + 256 > lds_limit || (need_split && p.split_lds_bytes + 256 > lds_limit)) return -1;
    p.grid = 0;
    *out = p;
    return 0;
}

hipError_t launch_order(const uint32_t *offsets, uint32_t n_events, uint32_t *order, hipStream_t s) {
    if (n_events == 0) return hipSuccess;
    hipLaunchKernelGGL(k_order, dim3(1), dim3(kOrderThreads), 0, s, offsets, n_events, order);
    return hipGetLastError();
}

size_t spill_stride(int n_theta, int n_rho) {
    const size_t words = (size_t)(n_rho + 31) / 32;
    // dilated words, per (column, 32-row block) a peak-row mask and the place of its first peak
    // within the column, per column the place of its first peak (and the end), per (column,
    // block) the counts of its at most 16 peaks
    const size_t n = 3 * words * n_theta + n_theta + 1 + 16 * words * n_theta;
    return (n + 63) & ~(size_t)63;                  // each workgroup's slice on a 256-byte boundary
}

hipError_t launch_spill(const GridArgs &g, const BatchArgs &a, const SpillArgs &sp, int n_wg, hipStream_t s) {
    if (a.n_events == 0 || n_wg < 1) return hipSuccess;
    // the slab's dynamic LDS beside the kernel's 16 KB of static LDS (allow_lds's limit would
    // not leave room for that); the slab doubles as the retention step's [words + 1][64]
    // dilated words (at most 257 * 64 dwords)
    constexpr int kBytes = kSpillSlabDwords * (int)sizeof(uint32_t);
    static const hipError_t lds_ok = hipFuncSetAttribute(reinterpret_cast<const void *>(k_spill),
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, kBytes);
    if (lds_ok != hipSuccess) return lds_ok;
    if (((size_t)(g.n_rho + 31) / 32 + 1) * 64u > (size_t)kSpillSlabDwords) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_spill, dim3(n_wg), dim3(kSpillThreads), (size_t)kBytes, s, g, a, sp);
    return hipGetLastError();
}

hipError_t launch_dedup(const BatchArgs &a, hipStream_t s) {
    if (a.n_events == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dedup, dim3(a.n_events), dim3(kDedupThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vote(const GridArgs &g, const float *x, const float *y, uint32_t n_hits,
                       void *acc, int acc_type, hipStream_t s) {
    if (g.vote_rows < 1) return hipErrorInvalidValue;
    const size_t lds = vote_lds_bytes(g.vote_rows);
    static const bool lds_ok = (allow_lds(k_vote<kVoteWaves>), true);
    (void)lds_ok;
    const int groups = (g.n_theta + 63) / 64, slabs = (g.n_rho + g.vote_rows - 1) / g.vote_rows;
    hipLaunchKernelGGL(k_vote<kVoteWaves>, dim3(groups, slabs), dim3(kVoteWaves * 64), lds, s, g, x, y,
                       n_hits, acc, acc_type, g.vote_rows);
    return hipGetLastError();
}

template <int NW, typename T>
static void launch_peaks_t(const GridArgs &g, const T *acc, hough_peak *peaks, uint32_t cap, uint32_t *n_peaks,
                           uint32_t *counts, hipStream_t s) {
    static const bool lds_ok = (allow_lds(k_peaks<NW, T, false>), allow_lds(k_peaks<NW, T, true>), true);
    (void)lds_ok;
    const size_t lds = peaks_lds_bytes(g.n_rho, NW);
    const int blocks = (g.n_theta + NW - 1) / NW;
    hipLaunchKernelGGL((k_peaks<NW, T, false>), dim3(blocks), dim3(NW * 64), lds, s, g, acc, peaks, cap, n_peaks,
                       counts);
    hipLaunchKernelGGL((k_peaks<NW, T, true>), dim3(blocks), dim3(NW * 64), lds, s, g, acc, peaks, cap, n_peaks,
                       counts);
}

template <typename T>
static hipError_t launch_peaks_w(const GridArgs &g, const T *acc, hough_peak *peaks, uint32_t cap,
                                 uint32_t *n_peaks, uint32_t *counts, hipStream_t s) {
    switch (g.peak_waves) {
        case 16: launch_peaks_t<16, T>(g, acc, peaks, cap, n_peaks, counts, s); break;
        case 8: launch_peaks_t<8, T>(g, acc, peaks, cap, n_peaks, counts, s); break;
        case 4: launch_peaks_t<4, T>(g, acc, peaks, cap, n_peaks, counts, s); break;
        case 2: launch_peaks_t<2, T>(g, acc, peaks, cap, n_peaks, counts, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// hough_peaks: workgroups of g.peak_waves theta rows (fewer for tall grids, whose rows take
// more LDS); counts holds one counter per workgroup.
hipError_t launch_peaks(const GridArgs &g, const void *acc, int acc_type, hough_peak *peaks,
                        uint32_t cap, uint32_t *n_peaks, uint32_t *counts, hipStream_t s) {
    if (acc_type == HOUGH_ACC_U16)
        return launch_peaks_w<uint16_t>(g, static_cast<const uint16_t *>(acc), peaks, cap, n_peaks, counts, s);
    return launch_peaks_w<uint32_t>(g, static_cast<const uint32_t *>(acc), peaks, cap, n_peaks, counts, s);
}

// Key buffer and bitmap placement of the iterative finder: the largest key buffer (a power of two
// of kIterMinKeys .. kIterMaxKeys keys) that fits beside an LDS bitmap of the grid, with room for
// `per_cu` workgroups per CU when that leaves at least 4096 keys, else one; a grid whose bitmap
// does not fit beside kIterMinKeys keys keeps it in device memory.
IterPlan plan_iterative(int n_theta, int n_rho, size_t lds_limit, int per_cu) {
    IterPlan p{};
    const size_t cells = (size_t)n_theta * (size_t)n_rho;
    p.bm_bytes = (cells + 31) / 32 * 4;
    const size_t room = lds_limit > 1024 ? lds_limit - 1024 : 0;      // static LDS and slack
    const size_t bm_lds = (p.bm_bytes + 15) & ~(size_t)15;
    for (int pc = per_cu; pc >= 1; --pc) {
        const uint32_t min_keys = pc > 1 ? 4096u : kIterMinKeys;
        for (uint32_t k = kIterMaxKeys; k >= min_keys; k >>= 1) {
            if ((size_t)pc * ((size_t)k * 8 + bm_lds) <= room) {
                p.keys = k;
                p.gbm = 0;
                p.lds_bytes = (size_t)k * 8 + bm_lds;
                return p;
            }
        }
    }
    for (uint32_t k = kIterMaxKeys; k >= kIterMinKeys; k >>= 1) {
        if ((size_t)per_cu * (size_t)k * 8 <= room || k == kIterMinKeys) {
            p.keys = k;
            break;
        }
    }
    p.gbm = 1;
    p.lds_bytes = (size_t)p.keys * 8;
    return p;
}

template <typename T>
static void launch_iter_t(const GridArgs &g, const T *acc, uint32_t frac_num, uint32_t frac_den, int r_theta,
                          int r_rho, hough_peak *peaks, uint32_t cap, uint32_t *n_peaks, uint32_t *status,
                          const uint32_t *offsets, uint32_t n_blocks, const IterPlan &ip, uint32_t *gbm,
                          hipStream_t s) {
    if (ip.gbm) {
        static const bool lds_ok = (allow_lds(k_peaks_iter<T, true>), true);
        (void)lds_ok;
        hipLaunchKernelGGL((k_peaks_iter<T, true>), dim3(n_blocks), dim3(kIterThreads), ip.lds_bytes, s, g, acc,
                           frac_num, frac_den, r_theta, r_rho, peaks, cap, n_peaks, status, offsets, ip.keys, gbm);
    } else {
        static const bool lds_ok = (allow_lds(k_peaks_iter<T, false>), true);
        (void)lds_ok;
        hipLaunchKernelGGL((k_peaks_iter<T, false>), dim3(n_blocks), dim3(kIterThreads), ip.lds_bytes, s, g, acc,
                           frac_num, frac_den, r_theta, r_rho, peaks, cap, n_peaks, status, offsets, ip.keys,
                           nullptr);
    }
}

hipError_t launch_peaks_iterative(const GridArgs &g, const void *acc, int acc_type, uint32_t frac_num,
                                  uint32_t frac_den, int r_theta, int r_rho, hough_peak *peaks,
                                  uint32_t cap, uint32_t *n_peaks, uint32_t *status, const IterPlan &ip,
                                  uint32_t *gbm, hipStream_t s) {
    if (acc_type == HOUGH_ACC_U16)
        launch_iter_t<uint16_t>(g, static_cast<const uint16_t *>(acc), frac_num, frac_den, r_theta, r_rho, peaks,
                                cap, n_peaks, status, nullptr, 1u, ip, gbm, s);
    else
        launch_iter_t<uint32_t>(g, static_cast<const uint32_t *>(acc), frac_num, frac_den, r_theta, r_rho, peaks,
                                cap, n_peaks, status, nullptr, 1u, ip, gbm, s);
    return hipGetLastError();
}

hipError_t launch_track_params(const GridArgs &g, const float *x, const float *y, uint32_t n_hits,
                               const hough_peak *peaks, const uint32_t *n_peaks, uint32_t cap,
                               double rho_min, double rho_max, double b_tesla, hough_track *out,
                               hipStream_t s) {
    if (cap == 0) return hipSuccess;
    const int blocks = (int)((cap + kTrackWaves - 1) / kTrackWaves);
    hipLaunchKernelGGL(k_track_params, dim3(blocks), dim3(kTrackWaves * 64), 0, s, g, x, y, n_hits, peaks,
                       n_peaks, cap, rho_min, rho_max, b_tesla, out);
    return hipGetLastError();
}

hipError_t launch_retain(const GridArgs &g, const float *x, const float *y, uint32_t n_hits,
                         const hough_peak *peaks, const uint32_t *n_peaks, uint32_t cap,
                         uint8_t *keep, hipStream_t s) {
    if (n_hits == 0) return hipSuccess;
    const int rows = retain_rows_per_block(g);
    const size_t lds = retain_lds_bytes(g, rows);
    static const bool lds_ok = (allow_lds(k_retain<kRetainWaves>), true);
    (void)lds_ok;
    const int blocks = (int)((n_hits + kRetainWaves * 64 - 1) / (kRetainWaves * 64));
    hipLaunchKernelGGL(k_retain<kRetainWaves>, dim3(blocks), dim3(kRetainWaves * 64), lds, s, g, x, y,
                       n_hits, peaks, n_peaks, cap, keep, rows);
    return hipGetLastError();
}

// The iterative finder's batch form: (duplicate pass), vote into per-event 16-bit accumulators,
// the finder, and retention with each event's first `cap` peaks, four launches for the batch.
hipError_t launch_batch_iterative(const GridArgs &g, const BatchArgs &a, uint16_t *acc, uint32_t frac_num,
                                  uint32_t frac_den, int r_theta, int r_rho, const IterPlan &ip, uint32_t *gbm,
                                  hipStream_t s) {
    if (a.n_events == 0) return hipSuccess;
    hipError_t e = hipSuccess;
    if (g.dedup) {
        e = launch_dedup(a, s);
        if (e != hipSuccess) return e;
    }
    {
        if (g.vote_rows < 1) return hipErrorInvalidValue;
        const size_t lds = vote_lds_bytes(g.vote_rows);
        static const bool lds_ok = (allow_lds(k_vote_batch<kVoteWaves>), true);
        (void)lds_ok;
        const int groups = (g.n_theta + 63) / 64, slabs = (g.n_rho + g.vote_rows - 1) / g.vote_rows;
        hipLaunchKernelGGL(k_vote_batch<kVoteWaves>, dim3(a.n_events, groups, slabs), dim3(kVoteWaves * 64), lds,
                           s, g, a.x, a.y, a.offsets, acc, a.keep, a.status, g.vote_rows);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    launch_iter_t<uint16_t>(g, acc, frac_num, frac_den, r_theta, r_rho, a.peaks, a.max_peaks, a.n_peaks, a.status,
                            a.offsets, a.n_events, ip, gbm, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        const int rows = retain_rows_per_block(g);
        const size_t lds = retain_lds_bytes(g, rows);
        static const bool lds_ok = (allow_lds(k_retain<kRetainWaves>), true);
        (void)lds_ok;
        const uint32_t blocks = (kMaxBatchHits + kRetainWaves * 64 - 1) / (kRetainWaves * 64);
        hipLaunchKernelGGL(k_retain<kRetainWaves>, dim3(a.n_events, blocks), dim3(kRetainWaves * 64), lds, s, g,
                           a.x, a.y, 0u, a.peaks, a.n_peaks, a.max_peaks, a.keep, rows, a.offsets);
        e = hipGetLastError();
    }
    return e;
}

template <int NW, int G, bool SP>
static void launch_batch_sp(const GridArgs &g, const BatchPlan &p, const BatchArgs &a, hipStream_t s) {
    const int nwords = (g.n_rho + 31) / 32;
    if constexpr (G == 1) {
        if (p.win) {
            hipLaunchKernelGGL((k_batch<NW, G, false, SP, true>), dim3(p.grid), dim3(NW * 64), p.lds_bytes, s, g, a,
                               p.n_tiles, nwords, p.win);
            return;
        }
    }
    if (g.periodic)
        hipLaunchKernelGGL((k_batch<NW, G, true, SP, false>), dim3(p.grid), dim3(NW * 64), p.lds_bytes, s, g, a,
                           p.n_tiles, nwords, 0);
    else
        hipLaunchKernelGGL((k_batch<NW, G, false, SP, false>), dim3(p.grid), dim3(NW * 64), p.lds_bytes, s, g, a,
                           p.n_tiles, nwords, 0);
}

template <int NW, int G>
static hipError_t launch_batch_t(const GridArgs &g, const BatchPlan &p, const BatchArgs &a,
                                 hipStream_t s) {
    if (p.win && (G != 1 || g.periodic)) return hipErrorInvalidValue;   // no such plan is made
    // a relative threshold leaves few peaks per tile whatever the grid
    if (p.sparse || a.frac_den != 0u)
        launch_batch_sp<NW, G, true>(g, p, a, s);
    else
        launch_batch_sp<NW, G, false>(g, p, a, s);
    return hipGetLastError();
}

hipError_t launch_batch(const GridArgs &g, const BatchPlan &p, const BatchArgs &a, hipStream_t s) {
    switch (p.waves * 10 + p.groups) {
        case 41: return launch_batch_t<4, 1>(g, p, a, s);
        case 42: return launch_batch_t<4, 2>(g, p, a, s);
        case 61: return launch_batch_t<6, 1>(g, p, a, s);
        case 62: return launch_batch_t<6, 2>(g, p, a, s);
        case 81: return launch_batch_t<8, 1>(g, p, a, s);
        case 82: return launch_batch_t<8, 2>(g, p, a, s);
        case 121: return launch_batch_t<12, 1>(g, p, a, s);
        case 122: return launch_batch_t<12, 2>(g, p, a, s);
        case 161: return launch_batch_t<16, 1>(g, p, a, s);
        case 162: return launch_batch_t<16, 2>(g, p, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int NW, int G>
static hipError_t launch_split_t(const GridArgs &g, const BatchPlan &p, const BatchArgs &a,
                                 const SplitArgs &sp, hipStream_t s) {
    const int nwords = (g.n_rho + 31) / 32;
    if (g.periodic)
        hipLaunchKernelGGL((k_batch_split<NW, G, true>), dim3(p.grid), dim3(NW * 64), p.split_lds_bytes, s, g, a,
                           sp, nwords);
    else
        hipLaunchKernelGGL((k_batch_split<NW, G, false>), dim3(p.grid), dim3(NW * 64), p.split_lds_bytes, s, g, a,
                           sp, nwords);
    return hipGetLastError();
}

hipError_t launch_batch_split(const GridArgs &g, const BatchPlan &p, const BatchArgs &a,
                              const SplitArgs &sp, hipStream_t s) {
    switch (p.waves * 10 + p.groups) {
        case 41: return launch_split_t<4, 1>(g, p, a, sp, s);
        case 42: return launch_split_t<4, 2>(g, p, a, sp, s);
        case 61: return launch_split_t<6, 1>(g, p, a, sp, s);
        case 62: return launch_split_t<6, 2>(g, p, a, sp, s);
        case 81: return launch_split_t<8, 1>(g, p, a, sp, s);
        case 82: return launch_split_t<8, 2>(g, p, a, sp, s);
        case 121: return launch_split_t<12, 1>(g, p, a, sp, s);
        case 122: return launch_split_t<12, 2>(g, p, a, sp, s);
        case 161: return launch_split_t<16, 1>(g, p, a, sp, s);
        case 162: return launch_split_t<16, 2>(g, p, a, sp, s);
        default: return hipErrorInvalidValue;
    }
}

// Workspace layout of the split form; every section starts on a 256-byte boundary.
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static void split_sizes(int n_theta, int n_rho, int groups, uint32_t n_events, uint32_t *n_tiles,
                        uint32_t *tile_cap, size_t off[6]) {
    const uint32_t out_cols = 64u * (uint32_t)groups - 2u;
    *n_tiles = ((uint32_t)n_theta + out_cols - 1u) / out_cols;
    *tile_cap = ((out_cols + 1u) / 2u) * (((uint32_t)n_rho + 1u) / 2u);
    const size_t E = n_events, T = *n_tiles;
    off[0] = 0;                                                          // counts
    off[1] = align256(off[0] + E * T * 4);                               // staged
    off[2] = align256(off[1] + E * T * (size_t)(*tile_cap) * sizeof(hough_peak));   // kept
    off[3] = align256(off[2] + E * kSplitKeepWords * 4);                 // done
    off[4] = align256(off[3] + E * 4);                                   // flags
    off[5] = align256(off[4] + E * 4);                                   // end
}

size_t split_workspace_bytes(int n_theta, int n_rho, int groups, uint32_t n_events) {
    uint32_t T, cap;
    size_t off[6];
    split_sizes(n_theta, n_rho, groups, n_events, &T, &cap, off);
    return off[5];
}

bool split_layout(int n_theta, int n_rho, int groups, uint32_t n_events, void *ws, size_t bytes,
                  SplitArgs *out) {
    uint32_t T, cap;
    size_t off[6];
    split_sizes(n_theta, n_rho, groups, n_events, &T, &cap, off);
    if (!ws || bytes < off[5] || ((uintptr_t)ws & 255u) != 0) return false;
    char *b = static_cast<char *>(ws);
    out->n_tiles = T;
    out->tile_cap = cap;
    out->counts = reinterpret_cast<uint32_t *>(b + off[0]);
    out->staged = reinterpret_cast<hough_peak *>(b + off[1]);
    out->kept = reinterpret_cast<uint32_t *>(b + off[2]);
    out->done = reinterpret_cast<uint32_t *>(b + off[3]);
    out->flags = reinterpret_cast<uint32_t *>(b + off[4]);
    return true;
}

template <typename K>
static int occupancy(K kernel, int threads, size_t lds) {
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, lds) == hipSuccess ? n : 0;
}

template <int NW, int G>
static int prepare_t(BatchPlan *p) {
    // both grid topologies and both forms: a context's plan serves whichever kernel it launches
    allow_lds(k_batch<NW, G, false, false, false>);
    allow_lds(k_batch<NW, G, true, false, false>);
    allow_lds(k_batch<NW, G, false, true, false>);
    allow_lds(k_batch<NW, G, true, true, false>);
    allow_lds(k_batch_split<NW, G, false>);
    allow_lds(k_batch_split<NW, G, true>);
    const int T = NW * 64;
    const size_t full = p->split_lds_bytes;
    int split = occupancy(k_batch_split<NW, G, false>, T, full);
    split = std::min(split, occupancy(k_batch_split<NW, G, true>, T, full));
    int fused = 0;
    if constexpr (G == 1) {
        if (p->win) {
            allow_lds(k_batch<NW, 1, false, false, true>);
            allow_lds(k_batch<NW, 1, false, true, true>);
            fused = std::min(occupancy(k_batch<NW, 1, false, false, true>, T, p->lds_bytes),
                             occupancy(k_batch<NW, 1, false, true, true>, T, p->lds_bytes));
        }
    }
    if (!p->win) {
        fused = std::min(occupancy(k_batch<NW, G, false, false, false>, T, full),
                         occupancy(k_batch<NW, G, true, false, false>, T, full));
        fused = std::min(fused, std::min(occupancy(k_batch<NW, G, false, true, false>, T, full),
                                         occupancy(k_batch<NW, G, true, true, false>, T, full)));
    }
    p->split_per_cu = split;
    return fused;
}

// Allow the plan's dynamic LDS for its kernels and return how many of the fused kernel's
// workgroups fit a CU (0 if none; split_per_cu gets the split form's).  Done once when a plan is
// chosen, so that launches make no other runtime calls.
int prepare_batch(BatchPlan *p) {
    switch (p->waves * 10 + p->groups) {
        case 41: return prepare_t<4, 1>(p);
        case 42: return prepare_t<4, 2>(p);
        case 61: return prepare_t<6, 1>(p);
        case 62: return prepare_t<6, 2>(p);
        case 81: return prepare_t<8, 1>(p);
        case 82: return prepare_t<8, 2>(p);
        case 121: return prepare_t<12, 1>(p);
        case 122: return prepare_t<12, 2>(p);
        case 161: return prepare_t<16, 1>(p);
        case 162: return prepare_t<16, 2>(p);
        default: return 0;
    }
}

}  // namespace hough

#ifdef HOUGH_PHASE_TIMING
// include/hough_debug.h: read (and optionally clear) the phase totals of the instrumented build.
extern "C" int hough_debug_phase_ticks(uint64_t *out, int32_t n, int32_t reset, uint32_t *clock_khz) {
    if (!out || n < 1 || n > hough::kPhaseSlots) return HOUGH_EINVAL;
    unsigned long long v[hough::kPhaseSlots] = {};
    int dev = 0, khz = 0;
    if (clock_khz && (hipGetDevice(&dev) != hipSuccess ||
                      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess))
        return HOUGH_EDEVICE;
    if (clock_khz) *clock_khz = (uint32_t)khz;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpyFromSymbol(v, HIP_SYMBOL(hough::g_phase_ticks), sizeof(v)) != hipSuccess)
        return HOUGH_EDEVICE;
    for (int i = 0; i < n; ++i) out[i] = (uint64_t)v[i];
    if (reset) {
        const unsigned long long z[hough::kPhaseSlots] = {};
        if (hipMemcpyToSymbol(HIP_SYMBOL(hough::g_phase_ticks), z, sizeof(z)) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)
            return HOUGH_EDEVICE;
    }
    return HOUGH_OK;
}
#endif
