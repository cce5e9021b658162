// hough.hip -- gfx950 kernels and C ABI of the Hough-transform track finder.
//
// The operations (prep, vote, peaks, assign) and their exact integer
// definitions are documented in include/hough.h.  This file is the MI355X
// implementation.  Every kernel handles a batch of events (blockIdx.y or a
// work queue selects the event); a single-event call is the batch of one.
//   prep    per-hit Q16.16 + integer CORDIC azimuth (one thread per hit), then
//           the valid hits are sorted by (layer, angle, hit) through cells
//           (layer, top azimuth bits): an event of one pass gets one workgroup
//           per layer (LDS histogram, scan, scatter, in-cell rank); a larger one
//           is bucketed by one workgroup and ranked by one thread per hit.  The
//           vote reads each layer's hits as one contiguous run, the assignment
//           finds a bin's hits as one run;
//   vote    one workgroup per (event, slab of 64 (l, k) columns) holds the
//           whole phi0 range of its columns in LDS as [bin][column] (16-bit
//           counters, columns c and c + 32 sharing a dword: one 128-byte row per
//           bin), loops over all hits of the event layer by layer and adds each
//           vote with a conflict-free ds_add_u32: one lane per column, one hit
//           per instruction (v_readlane broadcast, subtract, and-or, atomic);
//           the slab is then written once to HBM through a padded LDS tile (no
//           global atomics, slabs are disjoint, integer sums are order
//           independent).  Batches run it as a persistent kernel pulling
//           (event, slab) items from a device work queue, largest events first;
//   peaks   one thread per 8-bin strip of a column walks a range of d0 planes
//           keeping a 3-plane window in registers (separable 3-wide maxima,
//           edge bins from the neighbouring lanes), writes one flag byte per
//           strip and per-group candidate and vote counts; a scan of the group
//           counts and a write pass (one fused pass for single events and small
//           batches) compact the candidates in increasing linear index together
//           with their CSR offsets (the prefix sums of their vote counts);
//   assign  each candidate copies, layer by layer, the run of sorted hits
//           whose angle falls into its phi0 window, from hits staged in LDS
//           (one packed word per hit on grids of at most 16 angle bits); the
//           candidates of a wave assemble their stretch of the CSR list in LDS
//           and store it coalesced;
//   zvote   (second stage in r-z) a wave takes two candidates at a time: with
//           H <= 64 hits, min(8, 64 / H) rows of the cot(theta) x z0 grid are
//           voted at once, one lane per (row, hit), into per-row LDS histograms
//           whose words carry their own tie-break key, so the argmax is tracked
//           from the atomic's return value and each touched word is restored
//           right after the vote (no clearing pass, no scan of the grid);
//   fit     one lane per candidate sums the moments of the algebraic circle
//           fit over its list in list order (double), the wave's list stretch
//           staged in LDS (with the event's coordinates when they fit there),
//           and solves the 3x3 normal equations by Cramer's rule;
//   vertex  the second transform of the candidates: lane = radius row of an
//           LDS slab of the vertex space, one table-row load per run of
//           candidates sharing a column, candidate ranges counted apart and
//           added by a reduction kernel; its peaks reuse the peak finder;
//   cr      the vote with each hit's own radius: one thread per (hit, 16
//           columns), every sample computed (integer square root and integer
//           arcsine by CORDIC), global atomics.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "hough.h"

namespace {

constexpr int kMaxLayers = 32;
constexpr int kCordicSteps = 30;
constexpr int kVoteMaxThreads = 1024;
constexpr int kVoteCols = 64;       // columns per vote slab (one per lane)
constexpr int kStrip = 8;           // phi0 bins per peak-finder thread
constexpr int kScanThreads = 1024;
constexpr int kMaxCells = 32768;    // cells of a plan: the one-workgroup bucketing keeps all in LDS (128 KiB)
constexpr int kAssignThreads = 1024;
constexpr int kAssignBufMax = 2048;  // words of CSR list buffered per wave (less when the LDS is short)
constexpr int kAssignBufMin = 256;   // buffer below which an event's hits are not staged in LDS
constexpr int kLdsBytes = 160 * 1024;
constexpr int kZvoteThreads = 256;
constexpr int kZvoteSlots = 8;      // rows of the r-z grid one wave votes at once
constexpr int kZvoteMaxZ0 = 512;    // z0 bins (LDS: 4 waves x 8 rows x 4 bytes per bin + staging)

struct CordicTable {
    int32_t t[kCordicSteps];
};

struct LayerTable {
    int32_t valid_cols[kMaxLayers];  // number of (l, k) columns whose sample is valid, per layer
};

// Where the events of a call live.  One event: hit_off == nullptr and n_single hits.
struct Events {
    const int32_t* hit_off;  // (dev) [n_events + 1] start of each event in the packed hit arrays
    int32_t n_single;
    int32_t max_hits;        // events with more hits are not processed (flagged)
    size_t ws_stride;        // bytes between the workspaces of consecutive events
};

// Second-stage r-z grid in the kernels' integer units.  Row m has the Q16.16 cot(theta) centre
// c0 + m * dc (the plan checks that the centres form this exact progression); z0 bins have the
// width 2^shift in Q32.32 cm starting at z0min, so a z0 value v (Q32.32) falls into bin
// (v - z0min) >> shift when 0 <= v - z0min < lim = n_z0 << shift.
struct ZGrid {
    int32_t n_cot, n_z0, shift;
    int64_t z0min, c0, dc;
    uint64_t lim;
};

}  // namespace

struct hough_plan {
    int device;
    int n_layers;
    double r[kMaxLayers];
    double halflen[kMaxLayers];
    double B;
    hough_grid_t g;
    int log2_phi;
    int M;           // angle bits used by the vote
    int F;           // bits below one phi0 bin
    int cell_bits;   // m: azimuth cells per layer = 2^m
    int n_cols;      // n_d0 * n_qpt
    int n_cells;     // n_layers << m
    int64_t n_bins;
    CordicTable cordic;
    LayerTable layers;
    hough_tuning_t tuning;
    int32_t* d_E;    // [n_layers][n_d0][n_qpt], INT32_MIN = invalid
    const int32_t* d_Et;  // the same samples column by column, [n_d0 * n_qpt][et_stride] (inside d_E's block)
    int et_stride;        // layers per column of d_Et: n_layers, then INT32_MIN up to a multiple of 16
    bool zvote;      // second-stage grid present
    ZGrid zg;
    int32_t* d_S;    // [n_layers][n_d0][n_qpt] Q16.16 arc length to the layer, -1 = invalid (zvote only)
    hipEvent_t vote_start, vote_stop;  // recorded by every vote launch when set (kernel timing)
    hipEvent_t assign_start, assign_stop;  // the same for the window-table assignment
    int n_cu;        // compute units of the plan's device
    void* d_zero;    // one accumulator row of zeros (n_phi x 4 bytes): out-of-grid neighbours
    bool pt;         // window-table path: prefix-count table per event, table vote and assignment
    int pt_bpl;      // bins per lane of the table vote (n_phi / 64)
    int pt_row;      // entries per window-count row (n_phi + pt_bpl + 2, rounded up to 8)
    int pt_row8;     // bytes per 8-bit window-count row (n_phi + pt_bpl + 4, rounded up to 16); 0 = none
    bool stage;      // bin values fit 16 bits: the peak marker keeps each group's candidate values
};

namespace {

// ------------------------------------------------------------------ layout
struct WsLayout {
    size_t misc, phi32, lay, cell_start, tmp_phi, tmp_key, sorted_phi, sorted_h, ptab, gtab, gtab8;
    size_t flags, grp_count, grp_votes, grp_off, grp_voff, stage, peak_voff, total;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int peak_group_lanes(const hough_plan* p) {
    int strips = p->g.n_phi / kStrip;
    return strips < 64 ? strips : 64;
}

int64_t peak_groups(const hough_plan* p) {
    return p->n_bins / ((int64_t)kStrip * peak_group_lanes(p));
}

// Candidate values the peak marker keeps per group (16-bit, in candidate order): three per four
// strips; a group with more candidates is written from the accumulator instead.
__host__ __device__ __forceinline__ int stage_cap(int group_lanes) { return group_lanes * 3 / 4; }

// Workspace of one event.  `misc` holds the number of candidates listed by the peaks pass (int32).
WsLayout ws_layout(const hough_plan* p, int32_t max_peaks) {
    WsLayout L{};
    size_t o = 0;
    const size_t maxh = (size_t)p->g.max_hits_per_event;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.misc = take(256);  // first: its offset must not depend on max_peaks
    L.phi32 = take(4 * maxh);
    L.lay = take(maxh);
    L.cell_start = take(4 * ((size_t)p->n_cells + 1));
    L.tmp_phi = take(4 * maxh);
    L.tmp_key = take(4 * maxh);
    L.sorted_phi = take(4 * maxh);
    L.sorted_h = take(4 * maxh);
    L.ptab = take(p->pt ? (size_t)p->n_layers * ((size_t)1 << p->F) * p->g.n_phi * 2 : 0);
    L.gtab = take(p->pt ? (size_t)p->n_layers * ((size_t)1 << p->F) * p->pt_row * 2 : 0);
    L.gtab8 = take(p->pt ? (size_t)p->n_layers * ((size_t)1 << p->F) * p->pt_row8 : 0);
    L.flags = take((size_t)(p->n_bins / kStrip));
    L.grp_count = take(4 * (size_t)(peak_groups(p) + 1));
    L.grp_votes = take(4 * (size_t)(peak_groups(p) + 1));
    L.grp_off = take(4 * (size_t)(peak_groups(p) + 1));
    L.grp_voff = take(8 * (size_t)(peak_groups(p) + 1));
    L.stage = take(p->stage ? 2 * (size_t)peak_groups(p) * stage_cap(peak_group_lanes(p)) : 0);
    L.peak_voff = take(8 * (size_t)(max_peaks > 0 ? max_peaks : 1));  // last: sized by max_peaks
    L.total = o;
    return L;
}

// Batch header in front of the per-event workspaces: work-queue counter and event order.
size_t batch_header_bytes(int32_t n_events) { return align_up(256 + 4 * (size_t)n_events, 256); }

// XCD-aware placement of a batch's events.  Workgroups are dispatched to the 8 XCDs round-robin by
// their linear index, and each XCD has its own L2, so the per-event tables the vote and the
// assignment look up (window counts, prefix counts, sorted hits: a few MB per event) are fetched
// once per XCD that works on the event.  The batched kernels therefore keep all the work of one
// event on one XCD: XCD x takes the events of size rank 8g + x for even g and 8g + 7 - x for odd g
// (a snake over the size order, which balances the XCDs' totals).
constexpr int kXcds = 8;
constexpr int kXcdMinEvents = 4 * kXcds;  // fewer events would leave XCDs idle: they are spread instead
__host__ __device__ __forceinline__ int xcd_rank(int g, int x) { return kXcds * g + ((g & 1) ? kXcds - 1 - x : x); }

template <typename T>
__device__ __host__ __forceinline__ T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

__device__ __forceinline__ void event_hits(const Events& ev, int e, int& h0, int& n) {
    if (ev.hit_off) {
        h0 = ev.hit_off[e];
        n = ev.hit_off[e + 1] - h0;
    } else {
        h0 = 0;
        n = ev.n_single;
    }
}

__device__ __forceinline__ char* event_ws(char* ws, const Events& ev, int e) { return ws + (size_t)e * ev.ws_stride; }

// ------------------------------------------------------------------ device helpers
__device__ __forceinline__ uint32_t cordic_azimuth(int32_t X, int32_t Y, const CordicTable& T) {
    int64_t x = X, y = Y;
    uint32_t quarter = 0;
    while (!(x > 0 && y >= 0)) {  // turn by -90 degrees (at most three times)
        int64_t t = x;
        x = y;
        y = -t;
        ++quarter;
    }
    x *= 65536;
    y *= 65536;
    int64_t theta = 0;
#pragma unroll
    for (int i = 0; i < kCordicSteps; ++i) {
        int64_t dx = x >> i, dy = y >> i;
        if (y >= 0) {
            x += dy;
            y -= dx;
            theta += T.t[i];
        } else {
            x -= dy;
            y += dx;
            theta -= T.t[i];
        }
    }
    return quarter * 1073741824u + (uint32_t)theta;
}

// Inclusive scan of one int64 value per thread over a workgroup of kScanThreads threads.
// `wsum` is LDS scratch of kScanThreads / 64 entries.  Returns the inclusive prefix; *total = sum.
__device__ __forceinline__ int64_t block_inclusive_scan(int64_t v, int64_t* wsum, int64_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        int64_t t = lane < kScanThreads / 64 ? wsum[lane] : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t u = __shfl_up(t, o, 64);
            if (lane >= o) t += u;
        }
        if (lane < kScanThreads / 64) wsum[lane] = t;
    }
    __syncthreads();
    const int64_t r = v + (w > 0 ? wsum[w - 1] : 0);
    *total = wsum[kScanThreads / 64 - 1];
    __syncthreads();
    return r;
}

// Sum of one int64 value per thread over a workgroup of kScanThreads threads (every thread gets it).
// `wsum` is LDS scratch of kScanThreads / 64 entries.
__device__ __forceinline__ int64_t block_reduce_sum(int64_t v, int64_t* wsum) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; ++i) t += wsum[i];
    __syncthreads();
    return t;
}

struct WsOff {
    size_t misc, phi32, lay, cell_start, tmp_phi, tmp_key, sorted_phi, sorted_h, ptab, gtab, gtab8;
    size_t flags, grp_count, grp_votes, grp_off, grp_voff, stage, peak_voff;
};

WsOff ws_off(const WsLayout& L) {
    return WsOff{L.misc,  L.phi32, L.lay,   L.cell_start, L.tmp_phi,   L.tmp_key,  L.sorted_phi, L.sorted_h,
                 L.ptab,  L.gtab,  L.gtab8, L.flags,      L.grp_count, L.grp_votes, L.grp_off,   L.grp_voff,
                 L.stage, L.peak_voff};
}

// misc words of an event's workspace: [0] listed candidates, [1] sorted by the bucketing pass (slab
// path), [2] some window of the table path holds more than 255 hits (the vote then reads the
// 16-bit window counts instead of the 8-bit ones)
constexpr int kMiscWide = 2;

// ------------------------------------------------------------------ batch set-up
// One workgroup: order the events by decreasing hit count (ties by index) for the vote's work
// queue, and reset the queue counter.
__global__ __launch_bounds__(1024) void k_batch_init(const int32_t* __restrict__ hit_off, int32_t n_events,
                                                    int32_t* __restrict__ queue, int32_t* __restrict__ order) {
    for (int e = threadIdx.x; e < n_events; e += blockDim.x) {
        const int ne = hit_off[e + 1] - hit_off[e];
        int rank = 0;
        for (int j = 0; j < n_events; ++j) {
            const int nj = hit_off[j + 1] - hit_off[j];
            rank += (nj > ne || (nj == ne && j < e)) ? 1 : 0;
        }
        order[rank] = e;
    }
    if (threadIdx.x < kXcds) queue[threadIdx.x] = 0;  // one work-queue counter per XCD
}

// ------------------------------------------------------------------ prep kernels
// One thread per hit (grid.y = event): validity, Q16.16, CORDIC azimuth.  No atomics.
__global__ __launch_bounds__(256) void k_prep_hits(Events ev, const float* __restrict__ hx,
                                                   const float* __restrict__ hy, const uint8_t* __restrict__ hl,
                                                   int n_layers, CordicTable T, char* __restrict__ ws, WsOff O,
                                                   uint32_t* __restrict__ phi_out) {
    const int e = blockIdx.y;
    int h0, n;
    event_hits(ev, e, h0, n);
    if (n > ev.max_hits) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    char* w = event_ws(ws, ev, e);
    if (h == 0) at<int32_t>(w, O.misc)[kMiscWide] = 0;  // set again by k_prep_fine if a window is wide
    if (h >= n) return;
    const float x = hx[h0 + h], y = hy[h0 + h];
    const uint8_t L = hl[h0 + h];
    bool ok = (int)L < n_layers && isfinite(x) && isfinite(y) && fabsf(x) < 32768.0f && fabsf(y) < 32768.0f;
    uint32_t phi = 0;
    if (ok) {
        // x * 2^16 is exact in float; round half to even
        const int32_t X = __float2int_rn(x * 65536.0f);
        const int32_t Y = __float2int_rn(y * 65536.0f);
        ok = !(X == 0 && Y == 0);
        if (ok) phi = cordic_azimuth(X, Y, T);
    }
    at<uint32_t>(w, O.phi32)[h] = phi;
    at<uint8_t>(w, O.lay)[h] = ok ? L : (uint8_t)0xFF;
    if (phi_out) phi_out[h0 + h] = phi;
}

// Bucket the valid hits of an event by cell (layer, top `cell_bits` bits of the angle), sort them
// by (layer, angle, hit index) and reset the event's status.  grid = (n_layers, events).
// An event of at most cap_h hits (one pass in registers) is split by layer: workgroup L reads all
// hits, counts those of earlier layers (its base) with wave ballots, histograms its layer's hits
// over the layer's cells in LDS, scans the histogram -> cell_start, scatters its hits into LDS,
// ranks each inside its cell by (angle, hit index) -- kRankBatch hits of a thread at a time, the
// first 8 entries of their cells loaded together -- and writes sorted_phi / sorted_h nearly in
// order; workgroup 0 also writes the status and flags the event sorted (misc word 1).
// A larger event is bucketed by workgroup 0 alone: LDS histogram over all cells, scan, scatter
// into cell order (arbitrary inside a cell) -> tmp_phi, tmp_key = (layer << 24) | hit index, for
// k_prep_rank (a scatter of single words to random addresses from one workgroup is slow, which
// is why small events do not take this path).
// An event with more than max_hits hits is treated as empty and flagged.
constexpr int kBucketUnroll = 16;  // hits per thread and pass: events up to 16384 hits stay in registers
constexpr int kRankBatch = 4;      // hits a thread ranks inside their cells at once

__global__ __launch_bounds__(kScanThreads) void k_prep_bucket(Events ev, int n_layers, int cell_bits, int M,
                                                              LayerTable LT, char* __restrict__ ws, WsOff O,
                                                              hough_status_t* __restrict__ st_base, int cap_h) {
    // LDS: cursors (all cells, or one layer's), then (per-layer path) angles [cap_h + 8] and hit
    // indices [cap_h + 8]
    extern __shared__ int32_t cur[];
    __shared__ int64_t wsum[kScanThreads / 64];
    __shared__ int32_t layer_n[kMaxLayers];
    const int e = blockIdx.y;
    int h0, n;
    event_hits(ev, e, h0, n);
    const int n_given = n;
    if (n > ev.max_hits) n = 0;
    char* w = event_ws(ws, ev, e);
    const uint32_t* phi32 = at<uint32_t>(w, O.phi32);
    const uint8_t* lay = at<uint8_t>(w, O.lay);
    int32_t* cell_start = at<int32_t>(w, O.cell_start);
    hough_status_t* st = st_base + e;
    const int tid = threadIdx.x;
    const int n_cells = n_layers << cell_bits;
    const int cpl = 1 << cell_bits;  // cells per layer (<= 1024)
    const int cshift = 32 - cell_bits;
    const bool per_layer = n <= kScanThreads * kBucketUnroll && n <= cap_h;
    if (!per_layer && blockIdx.x != 0) return;
    int32_t* sorted_flag = at<int32_t>(w, O.misc) + 1;
    uint8_t L[kBucketUnroll];
    uint32_t ph[kBucketUnroll];
    auto load = [&](int base) {
#pragma unroll
        for (int j = 0; j < kBucketUnroll; ++j) {
            const int h = base + j * kScanThreads + tid;
            L[j] = h < n ? lay[h] : (uint8_t)0xFE;  // 0xFE: no hit, 0xFF: bad hit
            ph[j] = h < n ? phi32[h] : 0u;
        }
    };
    auto write_status = [&](int64_t bad_tot) {  // thread 0; layer_n holds every layer's count
        int64_t votes = 0;
        for (int Ly = 0; Ly < n_layers; ++Ly) votes += (int64_t)layer_n[Ly] * LT.valid_cols[Ly];
        st->n_hits = n_given;
        st->n_bad_hits = (int32_t)bad_tot;
        st->n_votes = votes;
        st->n_peaks = 0;
        st->flags = n_given > ev.max_hits ? HOUGH_F_EVENT_TOO_LARGE : 0;
        st->n_pairs = 0;
    };
    if (per_layer) {
        const int myL = blockIdx.x;
        for (int i = tid; i < cpl; i += kScanThreads) cur[i] = 0;
        if (tid < kMaxLayers) layer_n[tid] = 0;
        load(0);
        __syncthreads();
        int before = 0, bad = 0;
#pragma unroll
        for (int j = 0; j < kBucketUnroll; ++j) {
            const int l = L[j];
            bad += l == 0xFF ? 1 : 0;
            before += l < myL ? 1 : 0;  // valid layers are < n_layers <= 32 < 0xFE
            if (l == myL) atomicAdd(&cur[ph[j] >> cshift], 1);
            if (blockIdx.x == 0 && l < n_layers) atomicAdd(&layer_n[l], 1);
        }
        __syncthreads();
        // both counts in one workgroup sum (each < 2^31)
        int64_t t_packed;
        block_inclusive_scan((int64_t)before | ((int64_t)bad << 32), wsum, &t_packed);
        const int64_t t_before = t_packed & 0xFFFFFFFFll, t_bad = t_packed >> 32;
        // exclusive scan of the layer's histogram (one cell per thread) -> local cursors, cell_start
        const int v = tid < cpl ? cur[tid] : 0;
        int64_t t_mine;
        const int excl = (int)(block_inclusive_scan(v, wsum, &t_mine) - v);
        const int base = (int)t_before;
        if (tid < cpl) {
            cur[tid] = excl;
            cell_start[myL * cpl + tid] = base + excl;
        }
        if (tid == 0 && myL == n_layers - 1) cell_start[n_cells] = base + (int)t_mine;
        if (tid == 0 && blockIdx.x == 0) {
            write_status(t_bad);
            *sorted_flag = 1;
        }
        __syncthreads();
        // scatter the layer's hits into LDS (positions relative to the layer's start)
        uint32_t* s_phi = reinterpret_cast<uint32_t*>(cur + ((cpl + 3) & ~3));
        int32_t* s_h = reinterpret_cast<int32_t*>(s_phi + cap_h + 8);
#pragma unroll
        for (int j = 0; j < kBucketUnroll; ++j) {
            if (L[j] != myL) continue;
            const int pos = atomicAdd(&cur[ph[j] >> cshift], 1);
            s_phi[pos] = ph[j] >> (32 - M);
            s_h[pos] = j * kScanThreads + tid;
        }
        __syncthreads();
        // every cursor now holds the end of its cell, i.e. the start of the next one
        uint32_t* sorted_phi = at<uint32_t>(w, O.sorted_phi) + base;
        int32_t* sorted_h = at<int32_t>(w, O.sorted_h) + base;
        const int nt = (int)t_mine;
        const int lshift = M - cell_bits;
        for (int q0 = tid; q0 < nt; q0 += kRankBatch * kScanThreads) {
            uint32_t a[kRankBatch];
            int32_t hh[kRankBatch], c0[kRankBatch], n_in[kRankBatch], rank[kRankBatch];
#pragma unroll
            for (int u = 0; u < kRankBatch; ++u) {
                const int q = min(q0 + u * kScanThreads, nt - 1);
                a[u] = s_phi[q];
                hh[u] = s_h[q];
            }
#pragma unroll
            for (int u = 0; u < kRankBatch; ++u) {
                const int c = (int)(a[u] >> lshift);
                c0[u] = c > 0 ? cur[c - 1] : 0;
                n_in[u] = cur[c] - c0[u];
            }
#pragma unroll
            for (int u = 0; u < kRankBatch; ++u) {
                uint32_t b[8];
                int32_t k2[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    b[i] = s_phi[c0[u] + i];
                    k2[i] = s_h[c0[u] + i];
                }
                int r = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    r += (int)((i < n_in[u]) & ((b[i] < a[u]) | ((b[i] == a[u]) & (k2[i] < hh[u]))));
                rank[u] = r;
            }
#pragma unroll
            for (int u = 0; u < kRankBatch; ++u) {
                for (int j = 8; j < n_in[u]; ++j) {
                    const uint32_t b = s_phi[c0[u] + j];
                    rank[u] += (b < a[u] || (b == a[u] && s_h[c0[u] + j] < hh[u])) ? 1 : 0;
                }
                if (q0 + u * kScanThreads < nt) {
                    sorted_phi[c0[u] + rank[u]] = a[u];
                    sorted_h[c0[u] + rank[u]] = hh[u];
                }
            }
        }
        return;
    }
    // one workgroup for a larger event
    uint32_t* tmp_phi = at<uint32_t>(w, O.tmp_phi);
    int32_t* tmp_key = at<int32_t>(w, O.tmp_key);
    const bool resident = n <= kScanThreads * kBucketUnroll;  // one pass holds every hit
    for (int i = tid; i < n_cells; i += kScanThreads) cur[i] = 0;
    if (resident) load(0);
    __syncthreads();
    int32_t bad = 0;
    for (int base = 0; base < n; base += kScanThreads * kBucketUnroll) {
        if (!resident) load(base);
#pragma unroll
        for (int j = 0; j < kBucketUnroll; ++j) {
            if (L[j] == 0xFF) ++bad;
            else if (L[j] != 0xFE) atomicAdd(&cur[((int)L[j] << cell_bits) | (int)(ph[j] >> cshift)], 1);
        }
    }
    __syncthreads();
    // exclusive scan of the histogram: each thread owns a contiguous chunk
    const int per = (n_cells + kScanThreads - 1) / kScanThreads;
    const int lo = min(n_cells, tid * per), hi = min(n_cells, lo + per);
    int64_t s = 0;
    for (int i = lo; i < hi; ++i) s += cur[i];
    int64_t tot;
    int64_t run = block_inclusive_scan(s, wsum, &tot) - s;
    int64_t bad_tot;
    block_inclusive_scan(bad, wsum, &bad_tot);
    for (int i = lo; i < hi; ++i) {
        const int32_t c = cur[i];
        cur[i] = (int32_t)run;
        cell_start[i] = (int32_t)run;
        run += c;
    }
    if (tid == 0) cell_start[n_cells] = (int32_t)tot;
    __syncthreads();
    if (tid < n_layers) {
        const int a = cur[tid << cell_bits];
        const int z = tid + 1 < n_layers ? cur[(tid + 1) << cell_bits] : (int32_t)tot;
        layer_n[tid] = z - a;
    }
    __syncthreads();
    if (tid == 0) {
        write_status(bad_tot);
        *sorted_flag = 0;
    }
    // scatter into cell order
    for (int base = 0; base < n; base += kScanThreads * kBucketUnroll) {
        if (!resident) load(base);
#pragma unroll
        for (int j = 0; j < kBucketUnroll; ++j) {
            if (L[j] >= 0xFE) continue;
            const int h = base + j * kScanThreads + tid;
            const int pos = atomicAdd(&cur[((int)L[j] << cell_bits) | (int)(ph[j] >> cshift)], 1);
            tmp_phi[pos] = ph[j] >> (32 - M);
            tmp_key[pos] = ((int32_t)L[j] << 24) | h;
        }
    }
}

// One thread per bucketed hit (grid.y = event): rank inside its cell by (angle, hit index).
__global__ __launch_bounds__(256) void k_prep_rank(Events ev, int n_cells, int cell_bits, int M,
                                                   char* __restrict__ ws, WsOff O) {
    char* w = event_ws(ws, ev, blockIdx.y);
    if (at<int32_t>(w, O.misc)[1]) return;  // sorted by the bucketing pass
    const int32_t* cell_start = at<int32_t>(w, O.cell_start);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cell_start[n_cells]) return;
    const uint32_t* tmp_phi = at<uint32_t>(w, O.tmp_phi);
    const int32_t* tmp_key = at<int32_t>(w, O.tmp_key);
    const uint32_t a = tmp_phi[q];
    const int32_t key = tmp_key[q];
    const int32_t h = key & 0xFFFFFF;
    const int c = ((key >> 24) << cell_bits) | (int)(a >> (M - cell_bits));
    const int c0 = cell_start[c], c1 = cell_start[c + 1];
    int rank = 0;
    for (int j = c0; j < c1; ++j) {
        const uint32_t b = tmp_phi[j];
        rank += (b < a || (b == a && (tmp_key[j] & 0xFFFFFF) < h)) ? 1 : 0;
    }
    at<uint32_t>(w, O.sorted_phi)[c0 + rank] = a;
    at<int32_t>(w, O.sorted_h)[c0 + rank] = h;
}

// ------------------------------------------------------------------ prep for the window tables
// Plans with the window tables (see below) sort the hits and build both tables in one pass over a
// fine histogram: one workgroup per (event, layer L, chunk of R consecutive phi0 rows of the
// layer), R = the plan's prep_rows (tuned).  With W = 2^F angles per row, the workgroup counts the
// layer's hits of every M-bit angle of its rows and of the row after them (the next chunk's first
// row, or the turn's first row) in LDS (16-bit counters, two per word, rows padded to W/2 + 1 words so that
// reads of one phase down consecutive rows hit distinct banks), scans the counts into prefix
// counts P_L(x) (relative to the layer's first sorted hit; the layer's hits below the chunk come
// from a count over all hits), writes PT and GT for its rows and every phase, and places each of
// its hits at sorted position P_L(angle) (+ its rank among the hits of the same angle by hit
// index: tied hits are collected in LDS and ranked there).  Chunk 0 also writes the window-count
// entries past n_phi (the turn repeated) and the layer's start; workgroup 0 of the event writes the
// status.  Every workgroup reads the event's prepared hits (k_prep_hits) from L2 (once for events
// of at most 16384 hits, which stay in registers; twice otherwise).
constexpr int kFineRows = 128;     // phi0 rows per chunk
constexpr int kFineTieCap = 1024;  // tied hits a workgroup ranks in LDS (more: all tied hits ranked from memory)
constexpr int kFineUnroll = 16;    // hits per thread loaded at once

__global__ __launch_bounds__(kScanThreads) void k_prep_fine(Events ev, int n_layers, int cell_bits, int M, int F,
                                                            int n_phi, int row, int row8, int R, int n_chunks,
                                                            LayerTable LT,
                                                            char* __restrict__ ws, WsOff O,
                                                            hough_status_t* __restrict__ st_base) {
    extern __shared__ uint32_t fine_lds[];
    __shared__ int64_t wsum[kScanThreads / 64];
    __shared__ int32_t s_vc[kMaxLayers];  // valid (l, k) columns per layer: votes of one of its hits
    __shared__ int32_t n_tie;
    const int e = blockIdx.y;
    const int L = blockIdx.x / n_chunks;
    const int c = blockIdx.x - L * n_chunks;
    int h0, n;
    event_hits(ev, e, h0, n);
    const int n_given = n;
    if (n > ev.max_hits) n = 0;
    char* w = event_ws(ws, ev, e);
    const uint32_t* phi32 = at<uint32_t>(w, O.phi32);
    const uint8_t* lay = at<uint8_t>(w, O.lay);
    const int tid = threadIdx.x;
    const int W = 1 << F;
    const int wpr = W / 2 + 1;  // words per padded row
    const int nwords = (R + 1) * wpr;
    uint32_t* hist = fine_lds;
    uint32_t* ties = fine_lds + nwords;  // (chunk angle << 16) | hit
    const int row0 = c * R;
    const uint32_t a_lo = (uint32_t)row0 << F;
    const uint32_t a_hi = a_lo + ((uint32_t)R << F);
    const uint32_t next_row = (uint32_t)((row0 + R) & (n_phi - 1));  // the row after the chunk
    const int sh = 32 - M;
    const bool counter = blockIdx.x == 0;
    for (int i = tid; i < nwords; i += kScanThreads) hist[i] = 0u;
    if (tid < kMaxLayers) s_vc[tid] = tid < n_layers ? LT.valid_cols[tid] : 0;
    if (tid == 0) n_tie = 0;
    __syncthreads();
    // a thread reads kFineUnroll (16) consecutive hits at a time: their layers as one 16-byte load,
    // their azimuths as four (the regions are 256-byte aligned and padded, so a last partial group
    // stays inside them); an event of at most kScanThreads * kFineUnroll hits stays in registers
    // for the placing pass
    static_assert(kFineUnroll == 16, "one 16-byte load of layer bytes per thread");
    uint8_t lh[kFineUnroll];
    uint32_t ah[kFineUnroll];
    auto load_hits = [&](int hb) {
        const int h0 = hb + kFineUnroll * tid;
        uint4 lv = make_uint4(0xFEFEFEFEu, 0xFEFEFEFEu, 0xFEFEFEFEu, 0xFEFEFEFEu);  // 0xFE: no hit
        uint4 pv[4] = {};
        if (h0 < n) {
            lv = *reinterpret_cast<const uint4*>(lay + h0);
#pragma unroll
            for (int q = 0; q < 4; ++q) pv[q] = *reinterpret_cast<const uint4*>(phi32 + h0 + 4 * q);
        }
        const uint32_t lw[4] = {lv.x, lv.y, lv.z, lv.w};
#pragma unroll
        for (int j = 0; j < kFineUnroll; ++j) {
            const bool in = h0 + j < n;
            const uint32_t pj = j % 4 == 0 ? pv[j / 4].x : j % 4 == 1 ? pv[j / 4].y : j % 4 == 2 ? pv[j / 4].z : pv[j / 4].w;
            lh[j] = in ? (uint8_t)(lw[j / 4] >> (8 * (j % 4))) : (uint8_t)0xFE;  // 0xFF: bad hit
            ah[j] = in ? pj >> sh : 0u;
        }
    };
    const bool resident = n <= kScanThreads * kFineUnroll;
    int before = 0, bad = 0, below = 0, mine = 0;
    int64_t votes = 0;  // workgroup 0: the event's hit-votes, one table lookup per hit (no atomics)
    for (int hb = 0; hb < n; hb += kScanThreads * kFineUnroll) {
        load_hits(hb);
#pragma unroll
        for (int j = 0; j < kFineUnroll; ++j) {
            const int lj = lh[j];
            bad += lj == 0xFF ? 1 : 0;
            before += lj < L ? 1 : 0;
            if (counter && lj < n_layers) votes += s_vc[lj];
            if (lj != L) continue;
            ++mine;
            const uint32_t a = ah[j];
            below += a < a_lo ? 1 : 0;
            const uint32_t col = a & (uint32_t)(W - 1);
            const uint32_t inc = 1u << (16 * (col & 1u));
            if (a >= a_lo && a < a_hi) atomicAdd(&hist[(int)((a - a_lo) >> F) * wpr + (int)(col >> 1)], inc);
            if ((a >> F) == next_row) atomicAdd(&hist[R * wpr + (int)(col >> 1)], inc);
        }
    }
    // the four counts in 16-bit fields of one sum (each is at most the event's hits, <= 65535 here)
    const uint64_t tot4 = (uint64_t)block_reduce_sum(
        (int64_t)((uint64_t)before | ((uint64_t)bad << 16) | ((uint64_t)below << 32) | ((uint64_t)mine << 48)), wsum);
    const int64_t t_votes = counter ? block_reduce_sum(votes, wsum) : 0;  // uniform per workgroup
    const int base = (int)(tot4 & 0xFFFFu), n_bad = (int)((tot4 >> 16) & 0xFFFFu);
    const int cbase = (int)((tot4 >> 32) & 0xFFFFu), n_L = (int)(tot4 >> 48);
    // exclusive scan of the counts in angle order -> prefix counts (16 bits: differences stay exact)
    const int T = (R + 1) << F;
    const int k = ((T + kScanThreads - 1) / kScanThreads + 1) & ~1;
    const int lo = min(T, tid * k), hi = min(T, lo + k);
    int32_t sum = 0;
    for (int i = lo; i < hi; i += 2) {
        const uint32_t v = hist[(i >> F) * wpr + ((i & (W - 1)) >> 1)];
        sum += (int32_t)(v & 0xFFFFu) + (int32_t)(v >> 16);
    }
    int64_t tot;
    uint32_t pre = (uint32_t)(cbase + (block_inclusive_scan(sum, wsum, &tot) - sum));
    for (int i = lo; i < hi; i += 2) {
        const int wi = (i >> F) * wpr + ((i & (W - 1)) >> 1);
        const uint32_t v = hist[wi];
        const uint32_t c0 = v & 0xFFFFu, c1 = v >> 16;
        hist[wi] = (pre & 0xFFFFu) | ((pre + c0) << 16);
        pre += c0 + c1;
    }
    __syncthreads();
    auto P16 = [&](int rl, int cl) -> uint32_t {
        const uint32_t v = hist[rl * wpr + (cl >> 1)];
        return (cl & 1) ? v >> 16 : v & 0xFFFFu;
    };
    // tables: PT[L][r][j] = P(jW + r), GT[L][r][j] = P((j + 1)W + r) - P(jW + r), two rows per store
    uint32_t* pt = reinterpret_cast<uint32_t*>(at<uint16_t>(w, O.ptab) + (size_t)L * W * n_phi);
    uint32_t* gt = reinterpret_cast<uint32_t*>(at<uint16_t>(w, O.gtab) + (size_t)L * W * row);
    const int RP = R / 2;
    for (int t = tid; t < W * RP; t += kScanThreads) {
        const int r = t / RP, jp = t - r * RP;
        const uint32_t p0 = P16(2 * jp, r), p1 = P16(2 * jp + 1, r), p2 = P16(2 * jp + 2, r);
        pt[((size_t)r * n_phi + row0) / 2 + jp] = (p0 & 0xFFFFu) | (p1 << 16);
        gt[((size_t)r * row + row0) / 2 + jp] = ((p1 - p0) & 0xFFFFu) | ((p2 - p1) << 16);
    }
    if (c == 0) {  // window counts past the turn repeat its first rows
        const int EP = (row - n_phi) / 2;
        for (int t = tid; t < W * EP; t += kScanThreads) {
            const int r = t / EP, jp = t - r * EP;
            const uint32_t p0 = P16(2 * jp, r), p1 = P16(2 * jp + 1, r), p2 = P16(2 * jp + 2, r);
            gt[((size_t)r * row + n_phi) / 2 + jp] = ((p1 - p0) & 0xFFFFu) | ((p2 - p1) << 16);
        }
    }
    // the same window counts as bytes, four per store (the vote's table while no window of the event
    // holds more than 255 hits; a wider one sets the event's flag and the vote reads the 16-bit rows)
    if (row8 > 0) {
        uint32_t* gt8 = reinterpret_cast<uint32_t*>(at<uint8_t>(w, O.gtab8) + (size_t)L * W * row8);
        bool wide = false;
        auto quad = [&](int j0, int r) -> uint32_t {  // counts of local rows j0 .. j0 + 3 at phase r
            uint32_t word = 0, prev = P16(j0, r);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t next = P16(j0 + u + 1, r), cnt = (next - prev) & 0xFFFFu;
                wide = wide || cnt > 255u;
                word |= (cnt > 255u ? 255u : cnt) << (8 * u);
                prev = next;
            }
            return word;
        };
        const int RQ = R / 4;
        for (int t = tid; t < W * RQ; t += kScanThreads) {
            const int r = t / RQ, jq = t - r * RQ;
            gt8[((size_t)r * row8 + row0) / 4 + jq] = quad(4 * jq, r);
        }
        if (c == 0) {
            const int EQ = (row8 - n_phi) / 4;
            for (int t = tid; t < W * EQ; t += kScanThreads) {
                const int r = t / EQ, jq = t - r * EQ;
                gt8[((size_t)r * row8 + n_phi) / 4 + jq] = quad(4 * jq, r);
            }
        }
        if (wide) atomicOr(at<int32_t>(w, O.misc) + kMiscWide, 1);
    }
    // sorted positions of the chunk's hits
    int32_t* sorted_h = at<int32_t>(w, O.sorted_h) + base;
    for (int hb = 0; hb < n; hb += kScanThreads * kFineUnroll) {
        if (!resident) load_hits(hb);
#pragma unroll
        for (int j = 0; j < kFineUnroll; ++j) {
            const uint32_t a = ah[j];
            if (lh[j] != L || a < a_lo || a >= a_hi) continue;
            const int h = hb + kFineUnroll * tid + j;
            const uint32_t x = a - a_lo;
            const int rl = (int)(x >> F), cl = (int)(x & (uint32_t)(W - 1));
            const uint32_t p = P16(rl, cl);
            const uint32_t pn = cl + 1 < W ? P16(rl, cl + 1) : P16(rl + 1, 0);
            if (((pn - p) & 0xFFFFu) == 1u) {
                sorted_h[p] = h;
            } else {
                const int q = atomicAdd(&n_tie, 1);
                if (q < kFineTieCap) ties[q] = (x << 16) | (uint32_t)h;
            }
        }
    }
    __syncthreads();
    const int nt = n_tie;
    if (nt <= kFineTieCap) {
        for (int i = tid; i < nt; i += kScanThreads) {
            const uint32_t me = ties[i];
            const uint32_t x = me >> 16, hh = me & 0xFFFFu;
            int rank = 0;
            for (int j = 0; j < nt; ++j) {
                const uint32_t o = ties[j];
                rank += ((o >> 16) == x && (o & 0xFFFFu) < hh) ? 1 : 0;
            }
            sorted_h[P16((int)(x >> F), (int)(x & (uint32_t)(W - 1))) + rank] = (int32_t)hh;
        }
    } else {  // too many tied hits for LDS: each ranks itself against the event's hits
        for (int h = tid; h < n; h += kScanThreads) {
            if (lay[h] != L) continue;
            const uint32_t a = phi32[h] >> sh;
            if (a < a_lo || a >= a_hi) continue;
            const uint32_t x = a - a_lo;
            const int rl = (int)(x >> F), cl = (int)(x & (uint32_t)(W - 1));
            const uint32_t p = P16(rl, cl);
            const uint32_t pn = cl + 1 < W ? P16(rl, cl + 1) : P16(rl + 1, 0);
            if (((pn - p) & 0xFFFFu) == 1u) continue;
            int rank = 0;
            for (int j = 0; j < h; ++j) rank += (lay[j] == L && (phi32[j] >> sh) == a) ? 1 : 0;
            sorted_h[p + rank] = h;
        }
    }
    if (tid == 0 && c == 0) {
        int32_t* cell_start = at<int32_t>(w, O.cell_start);
        cell_start[L << cell_bits] = base;
        if (L == n_layers - 1) cell_start[n_layers << cell_bits] = base + n_L;
    }
    if (counter && tid == 0) {
        hough_status_t* st = st_base + e;
        st->n_hits = n_given;
        st->n_bad_hits = n_bad;
        st->n_votes = t_votes;
        st->n_peaks = 0;
        st->flags = n_given > ev.max_hits ? HOUGH_F_EVENT_TOO_LARGE : 0;
        st->n_pairs = 0;
    }
}

// ------------------------------------------------------------------ window tables
// Prefix counts of an event's sorted hits at every angle the vote and the assignment ask about.
// With W = 2^F and P_L(x) = the number of valid hits of layer L whose M-bit angle is < x, extended
// past the full turn by P_L(x + 2^M) = P_L(x) + n_L, for every phase r in [0, W):
//     PT[L][r][j] = P_L(j W + r)                          j in [0, n_phi)   (assignment)
//     GT[L][r][j] = P_L((j + 1) W + r) - P_L(j W + r)     j in [0, row)     (vote)
// GT[L][r][j] is the number of the layer's hits in the cyclic angle window [j W + r, (j + 1) W + r)
// (at most 65535: 16 bits), and for j < n_phi - 1 the window's hits are the sorted positions
// [PT[L][r][j], PT[L][r][j + 1]) of the layer.  A sample value E and a bin b of a column select the
// window x = (E mod 2^M) + b W: the same phase r = E mod W for every bin, at j = (E mod 2^M) div W + b.
// Window-count rows run `row` entries (past n_phi they repeat the turn) so that a lane of the vote
// reads its bins without a wrap.  Both tables are written by k_prep_fine.

// ------------------------------------------------------------------ vote
__device__ __forceinline__ void lds_vote(uint32_t phi, uint32_t e, uint32_t mask, uint32_t lanebits,
                                         uint32_t data) {
    const uint32_t t = phi - e;
    uint32_t a;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a) : "v"(t), "s"(mask), "v"(lanebits));
    asm volatile("ds_add_u32 %0, %1" ::"v"(a), "v"(data) : "memory");
}

// Four votes at once: the four addresses live in four registers, so no atomic waits for the one
// before it to have read its address register before the next address can be formed.
__device__ __forceinline__ void lds_vote4(uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3, uint32_t e,
                                          uint32_t mask, uint32_t lanebits, uint32_t data) {
    uint32_t a0, a1, a2, a3;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a0) : "v"(p0 - e), "s"(mask), "v"(lanebits));
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a1) : "v"(p1 - e), "s"(mask), "v"(lanebits));
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a2) : "v"(p2 - e), "s"(mask), "v"(lanebits));
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a3) : "v"(p3 - e), "s"(mask), "v"(lanebits));
    asm volatile(
        "ds_add_u32 %0, %4\n\t"
        "ds_add_u32 %1, %4\n\t"
        "ds_add_u32 %2, %4\n\t"
        "ds_add_u32 %3, %4" ::"v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(data) : "memory");
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

// SLAB16 = false: slab dword (b * 64 + c), one 32-bit counter per (bin, column), F = 8.
// SLAB16 = true : slab dword (b * 32 + c % 32), 16-bit halves for columns c and c + 32, F = 7
//                 (half the LDS, so two workgroups share a CU and one's store overlaps the
//                 other's votes; a half never carries: a column counts at most max_hits <= 65535).
// OUT16: the accumulator in HBM is int16 (else int32).
// Work items are (event, slab) pairs, item = rank * n_slabs + slab where rank orders the events
// (order == nullptr: identity).  Items 0 .. gridDim.x-1 are taken by block index; with a queue the
// next items come from an atomic counter (which must start at 0), otherwise by a stride of gridDim.x.
template <bool SLAB16, bool OUT16>
__global__ __launch_bounds__(kVoteMaxThreads) void k_vote(Events ev, const int32_t* __restrict__ E, int n_layers,
                                                          int cell_bits, int n_cols, int n_phi, int F,
                                                          char* __restrict__ ws, WsOff O,
                                                          char* __restrict__ acc_base, size_t acc_stride,
                                                          int n_events, const int32_t* __restrict__ order,
                                                          int32_t* __restrict__ queue, hough_status_t* st_base) {
    // LDS: [slab_dwords] counters, the queue broadcast word, then (16-bit slabs) the store tile
    extern __shared__ uint32_t slab[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_waves = blockDim.x >> 6;
    const int n_slabs = n_cols / kVoteCols;
    const int total = n_events * n_slabs;
    const int slab_dwords = SLAB16 ? n_phi * 32 : n_phi * 64;

    // The vote addresses LDS by byte offset from 0: the slab must be the kernel's only LDS object
    // (no static __shared__ variables in this kernel).
    const uint32_t lds_base = (uint32_t)(uintptr_t)(lds_u32*)slab;
    if (lds_base != 0) {
        if (tid == 0 && blockIdx.x == 0) atomicOr(&st_base->flags, 0x40000000);
        return;
    }
    const uint32_t mask = (uint32_t)(n_phi - 1) << F;
    const uint32_t lanebits = SLAB16 ? (uint32_t)(lane & 31) << 2 : (uint32_t)lane << 2;
    const uint32_t data = SLAB16 ? (lane >= 32 ? 0x10000u : 1u) : 1u;
    uint4* s4 = reinterpret_cast<uint4*>(slab);

    int item = blockIdx.x;
    while (item < total) {
        const int rank = item / n_slabs;
        const int e = order ? order[rank] : rank;
        const int slab_id = item - rank * n_slabs;
        const int col = slab_id * kVoteCols + lane;
        char* w = event_ws(ws, ev, e);
        const int32_t* cell_start = at<int32_t>(w, O.cell_start);
        const uint32_t* sorted_phi = at<uint32_t>(w, O.sorted_phi);

        for (int i = tid; i < slab_dwords / 4; i += blockDim.x) s4[i] = make_uint4(0, 0, 0, 0);
        __syncthreads();
        // The hits of each layer are cut into chunks of 64; chunk g (counted over all layers, layer
        // by layer) goes to wave g % n_waves.  Lane L holds layer L's hit range and the index of its
        // first chunk, so the layer of a chunk is one ballot away.  A wave loads a chunk with one
        // coalesced load (one hit per lane) together with its lane's sample value for that layer,
        // keeps four chunks in flight across layer boundaries, and broadcasts hit j with
        // v_readlane: the hit values travel in VGPRs, so waiting for them never waits for the LDS
        // atomics (scalar loads would share the LDS wait counter).
        int lo_L = 0, hi_L = 0;
        if (lane < n_layers) {
            lo_L = cell_start[lane << cell_bits];
            hi_L = cell_start[(lane + 1) << cell_bits];
        }
        const int nch_L = (hi_L - lo_L + 63) >> 6;
        int end_L = nch_L;  // inclusive prefix over the layers
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(end_L, o, 64);
            if (lane >= o) end_L += u;
        }
        const int cs_L = end_L - nch_L;
        const int total_chunks = __builtin_amdgcn_readlane(end_L, 63);
        // Branch-free: every fetch issues its two loads (clamped in bounds), so the wait before a
        // chunk's votes covers that chunk only; a chunk past the end has cnt = 0 and votes nothing.
        auto fetch = [&](int g, uint32_t& phi, int32_t& ev, int& cnt) {
            const int L = min((int)__popcll(__ballot(end_L <= g)), n_layers - 1);
            const int lo = __builtin_amdgcn_readlane(lo_L, L);
            const int hi = __builtin_amdgcn_readlane(hi_L, L);
            const int h = lo + ((g - __builtin_amdgcn_readlane(cs_L, L)) << 6);
            cnt = g < total_chunks ? min(64, hi - h) : 0;
            phi = sorted_phi[min(h + lane, max(hi - 1, 0))];
            ev = E[(size_t)L * n_cols + col];
        };
        auto vote_chunk = [&](uint32_t phi, int32_t ev, int cnt) {
            if (ev != INT32_MIN) {
                const uint32_t ue = (uint32_t)ev;
                if (cnt == 64) {
#pragma unroll
                    for (int j = 0; j < 64; j += 4)
                        lds_vote4((uint32_t)__builtin_amdgcn_readlane((int)phi, j),
                                  (uint32_t)__builtin_amdgcn_readlane((int)phi, j + 1),
                                  (uint32_t)__builtin_amdgcn_readlane((int)phi, j + 2),
                                  (uint32_t)__builtin_amdgcn_readlane((int)phi, j + 3), ue, mask, lanebits, data);
                } else {
                    for (int j = 0; j < cnt; ++j)
                        lds_vote((uint32_t)__builtin_amdgcn_readlane((int)phi, j), ue, mask, lanebits, data);
                }
            }
        };
        uint32_t p0, p1, p2, p3;
        int32_t e0, e1, e2, e3;
        int n0, n1, n2, n3;
        fetch(wave, p0, e0, n0);
        fetch(wave + n_waves, p1, e1, n1);
        fetch(wave + 2 * n_waves, p2, e2, n2);
        fetch(wave + 3 * n_waves, p3, e3, n3);
        for (int g = wave; g < total_chunks; g += 4 * n_waves) {
            vote_chunk(p0, e0, n0);
            fetch(g + 4 * n_waves, p0, e0, n0);
            vote_chunk(p1, e1, n1);
            fetch(g + 5 * n_waves, p1, e1, n1);
            vote_chunk(p2, e2, n2);
            fetch(g + 6 * n_waves, p2, e2, n2);
            vote_chunk(p3, e3, n3);
            fetch(g + 7 * n_waves, p3, e3, n3);
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        __syncthreads();

        // store the slab: acc[col][b], b fastest
        const int col0 = slab_id * kVoteCols;
        char* acc_e = acc_base + (size_t)e * acc_stride;
        if (!SLAB16) {
            int32_t* acc = reinterpret_cast<int32_t*>(acc_e);
            const int quads = n_phi / 4;
            for (int i = tid; i < quads * kVoteCols; i += blockDim.x) {
                const int c = i & 63, q = i >> 6;
                uint4 v;
                v.x = slab[(4 * q + 0) * 64 + c];
                v.y = slab[(4 * q + 1) * 64 + c];
                v.z = slab[(4 * q + 2) * 64 + c];
                v.w = slab[(4 * q + 3) * 64 + c];
                *reinterpret_cast<uint4*>(acc + (size_t)(col0 + c) * n_phi + 4 * q) = v;
            }
        } else {
            // Tiles of TB bins (a column's share of a tile is one 128-byte line of the accumulator)
            // go through a padded LDS tile T[64][TB + 1] of 32-bit words: read row by row from the
            // slab (conflict-free), written back column by column, so that eight lanes store one
            // column's line and a wave stores eight whole lines per instruction.
            const int TB = min(OUT16 ? 64 : 32, n_phi);  // n_phi >= 16 is a power of two
            const int TP = TB + 1;
            constexpr int CH = OUT16 ? 8 : 4;  // bins per 16-byte store
            const int NCH = TB / CH;           // stores per column and tile
            uint32_t* T = slab + slab_dwords + 64;
            for (int b0 = 0; b0 < n_phi; b0 += TB) {
                for (int i = tid; i < TB * 32; i += blockDim.x) {
                    const int r = i >> 5, d = i & 31;
                    const uint32_t w = slab[(b0 + r) * 32 + d];
                    T[d * TP + r] = w & 0xFFFFu;
                    T[(d + 32) * TP + r] = w >> 16;
                }
                __syncthreads();
                for (int i = tid; i < kVoteCols * NCH; i += blockDim.x) {
                    const int c = i / NCH, p = i % NCH;
                    const uint32_t* t = T + c * TP + p * CH;
                    uint4 v;
                    if (OUT16) {
                        v.x = t[0] | (t[1] << 16);
                        v.y = t[2] | (t[3] << 16);
                        v.z = t[4] | (t[5] << 16);
                        v.w = t[6] | (t[7] << 16);
                        int16_t* acc = reinterpret_cast<int16_t*>(acc_e);
                        *reinterpret_cast<uint4*>(acc + (size_t)(col0 + c) * n_phi + b0 + p * CH) = v;
                    } else {
                        v = make_uint4(t[0], t[1], t[2], t[3]);
                        int32_t* acc = reinterpret_cast<int32_t*>(acc_e);
                        *reinterpret_cast<uint4*>(acc + (size_t)(col0 + c) * n_phi + b0 + p * CH) = v;
                    }
                }
                __syncthreads();
            }
        }
        if (queue) {
            int* next_item = reinterpret_cast<int*>(slab + slab_dwords);
            if (tid == 0) *next_item = (int)gridDim.x + atomicAdd(queue, 1);
            __syncthreads();  // also: the slab reads above are done before the next zeroing
            item = *next_item;
            __syncthreads();
        } else {
            __syncthreads();
            item += gridDim.x;
        }
    }
}

// The vote from the window tables (plans with at most 65535 hits per event and n_phi >= 128).
// Column (l, k) gets, from each layer L whose sample E is valid, the layer's hits in the windows
// [x_b, x_b + W), x_b = (E mod 2^M) + b W: with r = E mod W and s = (E mod 2^M) div W, bin b
// receives GT[L][r][s + b] (index taken mod n_phi; the row's entries past n_phi repeat the turn).
// So the accumulator column is the sum over layers of one window-count row each, rotated by s: no
// atomics, and every read is a run of consecutive entries.
// One wave per column at a time: lane i owns the BPL bins [i BPL, (i + 1) BPL), the entries
// [i0, i0 + BPL) with i0 = (s + i BPL) mod n_phi.  A lane loads the BPL/2 dwords from the dword
// boundary at or below i0 with 16-byte loads (consecutive lanes read consecutive bytes of the row,
// so a wave reads one contiguous stretch per layer); when i0 is odd (the parity of s, the same for
// the whole wave) its last pair also needs the dword after them, which is the first dword of lane
// i + 1 (mod 64): the row repeats the turn past n_phi, and lane 63's next entry is lane 0's first.
// A byte permute with a wave-uniform selector aligns the pairs.  Counts are kept as 16-bit pairs in 32-bit words: a plain
// add never carries between the halves, since no bin exceeds the event's hit count (<= 65535).
// A layer without a valid sample reads a row of zeros (every load is issued unconditionally).
// Work items are (event, block of `cpi` columns) as in k_vote: item = rank * blocks + block;
// the 4 waves of a workgroup take `cpi` / 4 consecutive columns each.
constexpr int kVotePtThreads = 256;

template <int BPL, bool OUT16>
__global__ __launch_bounds__(kVotePtThreads) void k_vote_pt(Events ev, const int32_t* __restrict__ Et, int et_stride,
                                                           int n_layers,
                                                           int n_cols, int n_phi, int M, int F, int row, int row8,
                                                           const uint32_t* __restrict__ zero_row,
                                                           char* __restrict__ ws, WsOff O,
                                                           char* __restrict__ acc_base, size_t acc_stride,
                                                           int n_events, const int32_t* __restrict__ order,
                                                           int32_t* __restrict__ queue, int cpi) {
    constexpr int NP = BPL / 2;                       // bin pairs per lane (= dwords loaded per layer)
    constexpr int ND = NP + 1;                        // with the dword of the next lane
    constexpr int LG = ND * 10 <= 60 ? 10 : (60 / ND > 0 ? 60 / ND : 1);  // layers per load group
    const int next4 = ((threadIdx.x + 1) & 63) * 4;   // byte address of lane + 1 (mod 64) for ds_bpermute
    __shared__ int next_item;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n_blocks = n_cols / cpi;
    const int total = n_events * n_blocks;
    const int cpw = cpi / (kVotePtThreads / 64);     // columns per wave
    const uint32_t mmask = (1u << M) - 1u;
    const uint32_t wmask = (1u << F) - 1u;
    const int row2 = row / 2;                        // row length in dwords
    // with a queue (batches): the workgroups of XCD x = blockIdx.x % 8 take the (event, column
    // block) items of that XCD's events (xcd_rank) from the XCD's own queue counter
    const bool by_xcd = queue != nullptr && gridDim.x % kXcds == 0 && n_events >= kXcdMinEvents;
    const int xcd = (int)(blockIdx.x % kXcds);
    const int xcd_wgs = (int)gridDim.x / kXcds;
    const int xcd_total = ((n_events + kXcds - 1) / kXcds) * n_blocks;
    int item = by_xcd ? (int)blockIdx.x / kXcds : (int)blockIdx.x;
    while (item < (by_xcd ? xcd_total : total)) {
        int rank, blk;
        if (by_xcd) {
            const int g = item / n_blocks;
            rank = xcd_rank(g, xcd);
            blk = item - g * n_blocks;
        } else {
            rank = item / n_blocks;
            blk = item - rank * n_blocks;
        }
        if (rank >= n_events) {  // the last group of eight ranks is short: no such event on this XCD
            item = by_xcd ? xcd_total : total;
            continue;
        }
        const int e = order ? order[rank] : rank;
        const uint32_t* gt = at<const uint32_t>(event_ws(ws, ev, e), O.gtab);
        const uint8_t* gt8 = at<const uint8_t>(event_ws(ws, ev, e), O.gtab8);
        // the 8-bit window counts unless a window of this event holds more than 255 hits
        const bool use8 = row8 > 0 && at<const int32_t>(event_ws(ws, ev, e), O.misc)[kMiscWide] == 0;
        char* acc_e = acc_base + (size_t)e * acc_stride;
        // The column's samples (layer-major, padded with invalid ones past the last layer) come in
        // one vector load, lane L holding layer L, read out with v_readlane: one load per column
        // instead of a scalar load and wait per layer; the next column's load is issued before the
        // current column is summed.
        const int col_first = blk * cpi + wave * cpw;
        const int lane_l = lane < et_stride ? lane : 0;
        int32_t ev_next = Et[(size_t)col_first * et_stride + lane_l];
        for (int ci = 0; ci < cpw; ++ci) {
            const int col = col_first + ci;
            const int32_t ev_lane = ev_next;
            if (ci + 1 < cpw) ev_next = Et[(size_t)(col + 1) * et_stride + lane_l];
            uint32_t acc[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) acc[q] = 0u;
            if constexpr (BPL >= 4) {
                if (use8) {
                    // a lane's BPL bytes from the dword holding its first entry on: sh = the entry's byte
                    // in that dword (the same for every lane, BPL being a multiple of 4); the bytes past
                    // the lane's dwords are the next lane's first dword (ds_bpermute), and
                    // v_alignbyte/v_perm spread each run of four counts into two 16-bit pairs
                    constexpr int NQ = BPL / 4;
                    constexpr int LG8 = (NQ + 1) * 10 <= 60 ? 10 : (60 / (NQ + 1) > 0 ? 60 / (NQ + 1) : 1);
                    for (int L0 = 0; L0 < n_layers; L0 += LG8) {
                        uint32_t d[LG8][NQ + 1];
                        uint32_t sh[LG8];
#pragma unroll
                        for (int u = 0; u < LG8; ++u) {
                            const int L = L0 + u;
                            const int32_t ev_l = __builtin_amdgcn_readlane(ev_lane, L);
                            const uint32_t ep = (uint32_t)ev_l & mmask;
                            const uint32_t r = ep & wmask, sft = ep >> F;
                            const uint32_t i0 = (sft + (uint32_t)(lane * BPL)) & (uint32_t)(n_phi - 1);
                            // the row offset fits 32 bits (fewer than 2^31 table bytes per event): one
                            // scalar multiply instead of a 64-bit one
                            const uint32_t* src =
                                ev_l != INT32_MIN
                                    ? reinterpret_cast<const uint32_t*>(gt8 + ((((uint32_t)L << F) | r) * (uint32_t)row8))
                                    : zero_row;
                            sh[u] = __builtin_amdgcn_readfirstlane(sft) & 3u;
                            __builtin_memcpy(&d[u][0], src + (i0 >> 2), 4 * NQ);  // dword-aligned loads
                        }
#pragma unroll
                        for (int u = 0; u < LG8; ++u) {
                            d[u][NQ] = sh[u] ? (uint32_t)__builtin_amdgcn_ds_bpermute(next4, (int)d[u][0]) : 0u;
#pragma unroll
                            for (int k = 0; k < NQ; ++k) {
                                const uint32_t x = __builtin_amdgcn_alignbyte(d[u][k + 1], d[u][k], sh[u]);
                                acc[2 * k] += __builtin_amdgcn_perm(x, x, 0x0c010c00u);
                                acc[2 * k + 1] += __builtin_amdgcn_perm(x, x, 0x0c030c02u);
                            }
                        }
                    }
                }
            }
            for (int L0 = 0; L0 < ((BPL >= 4 && use8) ? 0 : n_layers); L0 += LG) {
                uint32_t d[LG][ND];
                uint32_t sel[LG];
                bool odd[LG];
#pragma unroll
                for (int u = 0; u < LG; ++u) {
                    const int L = L0 + u;
                    const int32_t ev_l = __builtin_amdgcn_readlane(ev_lane, L);
                    const uint32_t ep = (uint32_t)ev_l & mmask;
                    const uint32_t r = ep & wmask, sft = ep >> F;
                    const uint32_t i0 = (sft + (uint32_t)(lane * BPL)) & (uint32_t)(n_phi - 1);
                    const uint32_t* src = ev_l != INT32_MIN ? gt + ((((uint32_t)L << F) | r) * (uint32_t)row2) : zero_row;
                    // byte selector: the pair starting at an odd entry spans two dwords
                    odd[u] = (__builtin_amdgcn_readfirstlane(sft) & 1u) != 0u;
                    sel[u] = odd[u] ? 0x05040302u : 0x03020100u;
                    __builtin_memcpy(&d[u][0], src + (i0 >> 1), 4 * NP);  // dword-aligned 16-byte loads
                }
#pragma unroll
                for (int u = 0; u < LG; ++u) {
                    d[u][NP] = odd[u] ? (uint32_t)__builtin_amdgcn_ds_bpermute(next4, (int)d[u][0]) : 0u;
#pragma unroll
                    for (int q = 0; q < NP; ++q) acc[q] += __builtin_amdgcn_perm(d[u][q + 1], d[u][q], sel[u]);
                }
            }
            // store the column's bins [lane * BPL, (lane + 1) * BPL)
            if (OUT16) {
                uint32_t* dst = reinterpret_cast<uint32_t*>(acc_e + ((size_t)col * n_phi + (size_t)lane * BPL) * 2);
#pragma unroll
                for (int q = 0; q < NP; q += 4) {
                    if (q + 4 <= NP) *reinterpret_cast<uint4*>(dst + q) = make_uint4(acc[q], acc[q + 1], acc[q + 2], acc[q + 3]);
                    else if (q + 2 <= NP) *reinterpret_cast<uint2*>(dst + q) = make_uint2(acc[q], acc[q + 1]);
                    else dst[q] = acc[q];
                }
            } else {
                uint32_t* dst = reinterpret_cast<uint32_t*>(acc_e + ((size_t)col * n_phi + (size_t)lane * BPL) * 4);
#pragma unroll
                for (int q = 0; q < NP; q += 2) {
                    if (q + 2 <= NP)
                        *reinterpret_cast<uint4*>(dst + 2 * q) = make_uint4(acc[q] & 0xFFFFu, acc[q] >> 16,
                                                                            acc[q + 1] & 0xFFFFu, acc[q + 1] >> 16);
                    else
                        *reinterpret_cast<uint2*>(dst + 2 * q) = make_uint2(acc[q] & 0xFFFFu, acc[q] >> 16);
                }
            }
        }
        if (by_xcd) {
            __syncthreads();
            if (threadIdx.x == 0) next_item = xcd_wgs + atomicAdd(queue + xcd, 1);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(next_item);
        } else if (queue) {
            __syncthreads();
            if (threadIdx.x == 0) next_item = (int)gridDim.x + atomicAdd(queue, 1);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(next_item);
        } else {
            item += gridDim.x;
        }
    }
}

// ------------------------------------------------------------------ peaks
// The cyclic phi0 neighbours of a strip (its edge bins) are the last bin of the strip before and
// the first bin of the strip after.  Consecutive lanes hold consecutive strips of a row, so the
// edge bins come from neighbouring lanes (ds_bpermute) instead of two narrow loads per row; only
// when a row is wider than a wave (more than 64 strips) do its first and last lanes load the
// bin beyond the wave from memory.
struct EdgeLanes {
    int left4, right4;  // byte addresses (lane * 4) of the lanes holding strips s-1 and s+1
    bool mem_l, mem_r;  // this lane loads its left / right edge bin from memory
};

__device__ __forceinline__ EdgeLanes edge_lanes(int strips) {
    const int lane = threadIdx.x & 63;
    const int g = strips < 64 ? strips : 64;  // strips of one row inside a wave (powers of two)
    const int row0 = lane & ~(g - 1);
    EdgeLanes e;
    e.left4 = (row0 | ((lane - 1) & (g - 1))) * 4;
    e.right4 = (row0 | ((lane + 1) & (g - 1))) * 4;
    e.mem_l = strips > 64 && lane == 0;
    e.mem_r = strips > 64 && lane == 63;
    return e;
}

// One strip of kStrip bins of a column row as 32-bit words (int16 rows: two bins per word); with
// rows wider than a wave (WIDE), the first and last lanes also load their outer edge bin.
template <typename T>
struct PlaneRaw {
    static constexpr int kW = sizeof(T) == 4 ? kStrip : kStrip / 2;
    uint32_t a[kW], m[kW], c[kW];  // columns k-1, k, k+1
    int32_t ea[2], em[2], ec[2];   // edge bins from memory (WIDE only)
};

template <typename T, bool WIDE>
__device__ __forceinline__ void load_strip(const T* __restrict__ row, int s, int n_phi, const EdgeLanes& el,
                                           uint32_t (&w)[PlaneRaw<T>::kW], int32_t (&e)[2]) {
    const int b0 = s * kStrip;
    const uint4 x = *reinterpret_cast<const uint4*>(row + b0);
    w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
    if (sizeof(T) == 4) {
        const uint4 y = *reinterpret_cast<const uint4*>(row + b0 + 4);
        w[4 % PlaneRaw<T>::kW] = y.x; w[5 % PlaneRaw<T>::kW] = y.y;
        w[6 % PlaneRaw<T>::kW] = y.z; w[7 % PlaneRaw<T>::kW] = y.w;
    }
    if (WIDE) {
        e[0] = 0;
        e[1] = 0;
        if (el.mem_l) e[0] = (int32_t)row[(b0 - 1) & (n_phi - 1)];
        if (el.mem_r) e[1] = (int32_t)row[(b0 + kStrip) & (n_phi - 1)];
    }
}

// The strip's bins v[1..8] and its edge bins v[0], v[9] (from the neighbouring lanes; every lane
// of the wave is active).
template <typename T, bool WIDE>
__device__ __forceinline__ void row_values(const uint32_t (&w)[PlaneRaw<T>::kW], const int32_t (&e)[2],
                                           const EdgeLanes& el, int32_t v[kStrip + 2]) {
#pragma unroll
    for (int i = 0; i < kStrip; ++i) {
        if (sizeof(T) == 4) v[i + 1] = (int32_t)w[i % PlaneRaw<T>::kW];
        else v[i + 1] = (int32_t)(int16_t)(w[(i >> 1) % PlaneRaw<T>::kW] >> (16 * (i & 1)));
    }
    const int l = __builtin_amdgcn_ds_bpermute(el.left4, v[kStrip]);
    const int r = __builtin_amdgcn_ds_bpermute(el.right4, v[1]);
    v[0] = WIDE && el.mem_l ? e[0] : l;
    v[kStrip + 1] = WIDE && el.mem_r ? e[1] : r;
}

// Raw loads of one d0 plane (columns k-1, k, k+1) in flight.  A neighbour outside the grid (d0 plane
// or q/pT column) is read from a row of zeros: accumulator values are >= 0 and candidates need
// >= threshold >= 1 votes, so a zero neighbour never decides a comparison, and every load is
// issued without a branch.
template <typename T, bool WIDE>
__device__ __forceinline__ void load_plane_raw(const T* __restrict__ acc, const T* __restrict__ zero_row, int l,
                                               int k, int s, int n_d0, int n_qpt, int n_phi, const EdgeLanes& el,
                                               PlaneRaw<T>& r) {
    const bool ok_plane = l >= 0 && l < n_d0;
    const T* base = acc + ((size_t)(ok_plane ? l : 0) * n_qpt + k) * n_phi;
    load_strip<T, WIDE>(ok_plane && k > 0 ? base - n_phi : zero_row, s, n_phi, el, r.a, r.ea);
    load_strip<T, WIDE>(ok_plane ? base : zero_row, s, n_phi, el, r.m, r.em);
    load_strip<T, WIDE>(ok_plane && k + 1 < n_qpt ? base + n_phi : zero_row, s, n_phi, el, r.c, r.ec);
}

// 3-wide maxima along phi0 of a strip with its two edge bins: m[i] = max(v[i], v[i+1], v[i+2])
__device__ __forceinline__ void max3(const int32_t v[kStrip + 2], int32_t m[kStrip]) {
#pragma unroll
    for (int i = 0; i < kStrip; ++i) m[i] = max(max(v[i], v[i + 1]), v[i + 2]);
}

struct PlaneWin {
    int32_t mid[kStrip + 2];  // the column itself, with edge bins
    int32_t lo[kStrip];       // 3-wide max of column k-1
    int32_t hi[kStrip];       // 3-wide max of column k+1
    int32_t all[kStrip];      // 3x3 max over columns k-1..k+1
};

template <typename T, bool WIDE>
__device__ __forceinline__ void finish_plane(const PlaneRaw<T>& r, const EdgeLanes& el, PlaneWin& w) {
    int32_t v[kStrip + 2], m0[kStrip];
    row_values<T, WIDE>(r.a, r.ea, el, v);
    max3(v, w.lo);
    row_values<T, WIDE>(r.c, r.ec, el, v);
    max3(v, w.hi);
    row_values<T, WIDE>(r.m, r.em, el, w.mid);
    max3(w.mid, m0);
#pragma unroll
    for (int i = 0; i < kStrip; ++i) w.all[i] = max(max(w.lo[i], m0[i]), w.hi[i]);
}

// grid.y = event.  Each thread walks `planes` (<= kMaxPeakPlanes) d0 planes of one strip, keeping
// the planes l-1, l, l+1 reduced in registers and the loads of plane l+2 in flight.  Its outputs
// (flag bytes, vote sums) are kept in LDS and stored after the walk: a global store inside the
// walk would make every wait for the next plane's loads also wait for that store.  The group sums
// are formed once after the walk from the per-strip flags and vote sums in LDS (16-byte reads),
// not by lane shuffles at every plane.
constexpr int kMaxPeakPlanes = 32;
constexpr int kMarkThreads = 256;

// Dynamic LDS of one marker workgroup: per plane the flag bytes and vote sums of its strips, the
// group counts and (staging on) the groups' candidate values.
__host__ __device__ __forceinline__ size_t mark_lds_bytes(int planes, int group_lanes, bool stage_on) {
    const size_t G = (size_t)(kMarkThreads / group_lanes);
    return (size_t)planes * (5 * (size_t)kMarkThreads + 4 * G + (stage_on ? 2 * G * (size_t)stage_cap(group_lanes) : 0));
}

// ROWW: rows of at least 64 strips, so that the 64 lanes of a wave hold strips of one row (one
// column and plane range per wave): the row addresses are then computed once per wave, in scalar
// registers.
template <typename T, bool WIDE, bool ROWW>
__global__ __launch_bounds__(kMarkThreads) void k_peaks_mark(Events ev, const char* __restrict__ acc_base,
                                                             size_t acc_stride, const T* __restrict__ zero_row,
                                                             int32_t thr, int n_d0, int n_qpt, int n_phi,
                                                             int group_lanes, int planes, bool stage_on,
                                                             char* __restrict__ ws, WsOff O) {
    // [planes][256] flag bytes | [planes][256] vote sums | [planes][G] group counts | [planes][G][capg] values
    extern __shared__ uint32_t mk_lds[];
    const int G = kMarkThreads / group_lanes;  // groups per workgroup
    uint8_t* s_flags = reinterpret_cast<uint8_t*>(mk_lds);
    int32_t* s_vl = reinterpret_cast<int32_t*>(mk_lds) + planes * (kMarkThreads / 4);
    int32_t* s_cnt = s_vl + planes * kMarkThreads;
    uint16_t* s_val = reinterpret_cast<uint16_t*>(s_cnt + planes * G);
    const int e = blockIdx.y;
    const T* acc = reinterpret_cast<const T*>(acc_base + (size_t)e * acc_stride);
    char* w = event_ws(ws, ev, e);
    uint8_t* flags = at<uint8_t>(w, O.flags);
    int32_t* grp_count = at<int32_t>(w, O.grp_count);
    int32_t* grp_votes = at<int32_t>(w, O.grp_votes);
    uint16_t* stage = at<uint16_t>(w, O.stage);
    const int capg = stage_cap(group_lanes);
    const int gi = threadIdx.x / group_lanes;          // group of this thread inside the workgroup
    const int gq = threadIdx.x & (group_lanes - 1);    // its strip inside the group
    const uint64_t gmask = group_lanes == 64 ? ~0ull
                                             : ((1ull << group_lanes) - 1ull) << ((threadIdx.x & 63) & ~(group_lanes - 1));
    const int strips = n_phi / kStrip;
    // Workgroups go to the 8 XCDs round-robin and each XCD has its own L2: block b works on tile
    // (b % 8) * (gridDim.x / 8) + b / 8 (gridDim.x is a multiple of 8), so the neighbouring q/pT
    // columns one tile re-reads are mostly loaded by tiles on the same XCD.
    const unsigned tile = (blockIdx.x % 8u) * (gridDim.x / 8u) + blockIdx.x / 8u;
    const int64_t t = (int64_t)tile * blockDim.x + threadIdx.x;
    const int s = (int)(t % strips);
    int k = (int)((t / strips) % n_qpt);
    int lr = (int)(t / ((int64_t)strips * n_qpt));
    if constexpr (ROWW) {
        k = __builtin_amdgcn_readfirstlane(k);
        lr = __builtin_amdgcn_readfirstlane(lr);
    }
    const int l0 = lr * planes;
    if (l0 >= n_d0) return;  // whole waves exit together (strips * n_qpt is a multiple of 64)
    const int l1 = min(n_d0, l0 + planes);
    PlaneRaw<T> raw;
    PlaneWin wa, wb, wc;  // planes l-1, l, l+1 rotate through these (no copies between planes)
    const EdgeLanes el = edge_lanes(strips);
    load_plane_raw<T, WIDE>(acc, zero_row, l0 - 1, k, s, n_d0, n_qpt, n_phi, el, raw);
    finish_plane<T, WIDE>(raw, el, wa);
    load_plane_raw<T, WIDE>(acc, zero_row, l0, k, s, n_d0, n_qpt, n_phi, el, raw);
    finish_plane<T, WIDE>(raw, el, wb);
    load_plane_raw<T, WIDE>(acc, zero_row, l0 + 1, k, s, n_d0, n_qpt, n_phi, el, raw);
    // test plane l (cur) against prev and next, with the loads of plane l + 2 in flight
    auto test_plane = [&](int l, const PlaneWin& prev, const PlaneWin& cur, PlaneWin& next) {
        finish_plane<T, WIDE>(raw, el, next);
        load_plane_raw<T, WIDE>(acc, zero_row, l + 2, k, s, n_d0, n_qpt, n_phi, el, raw);
        uint32_t bits = 0;
        int32_t vsum = 0;
#pragma unroll
        for (int i = 0; i < kStrip; ++i) {
            const int32_t v = cur.mid[i + 1];
            // neighbours that precede (l-1 plane, column k-1 of this plane, bin b-1) must be < v,
            // neighbours that follow must be <= v
            const int32_t P = max(max(prev.all[i], cur.lo[i]), cur.mid[i]);
            const int32_t Q = max(max(next.all[i], cur.hi[i]), cur.mid[i + 2]);
            if (v >= thr && v > P && v >= Q) {
                bits |= 1u << i;
                vsum += v;
            }
        }
        s_flags[(l - l0) * kMarkThreads + threadIdx.x] = (uint8_t)bits;
        s_vl[(l - l0) * kMarkThreads + threadIdx.x] = vsum;
        if (stage_on) {
            const int32_t cnt = __popc(bits);  // the group's candidate values in candidate order, while they are in registers
            // a strip holds at most 4 candidates (two adjacent bins cannot both win the tie rule):
            // the group's exclusive prefix of the counts from three ballots of their bits
            const uint64_t b0 = __ballot(cnt & 1), b1 = __ballot(cnt & 2), b2 = __ballot(cnt & 4);
            const uint64_t below = gmask & ((1ull << (threadIdx.x & 63)) - 1ull);
            int pos = __popcll(b0 & below) + 2 * __popcll(b1 & below) + 4 * __popcll(b2 & below);
            uint16_t* sv = s_val + ((l - l0) * G + gi) * capg;
#pragma unroll
            for (int i = 0; i < kStrip; ++i) {
                if ((bits >> i) & 1u) {
                    if (pos < capg) sv[pos] = (uint16_t)cur.mid[i + 1];
                    ++pos;
                }
            }
        }
    };
    for (int l = l0; l < l1; l += 3) {
        test_plane(l, wa, wb, wc);
        if (l + 1 >= l1) break;
        test_plane(l + 1, wb, wc, wa);
        if (l + 2 >= l1) break;
        test_plane(l + 2, wc, wa, wb);
    }
    // Group sums (a group is `group_lanes` consecutive strips of one column, inside one wave): lane x
    // of the wave takes its (plane, group) pairs x, x + 64, ..., adding the group's vote sums and
    // counting its flag bits in LDS.  The LDS written by the wave's other lanes is read after a wave
    // barrier (a wave's LDS operations complete in order).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
        const int np = l1 - l0;
        const int gw = 64 / group_lanes;  // groups per wave
        const int wave_t0 = (int)threadIdx.x & ~63;
        for (int x = (int)threadIdx.x & 63; x < np * gw; x += 64) {
            const int p = x / gw, g = x - p * gw;
            const int tid0 = wave_t0 + g * group_lanes;  // the group's first thread
            const int32_t* vl = s_vl + p * kMarkThreads + tid0;
            const uint8_t* fl = s_flags + p * kMarkThreads + tid0;
            int32_t vs = 0, cn = 0;
            if (group_lanes >= 4) {
                for (int i = 0; i < group_lanes; i += 4) {
                    const int4 v4 = *reinterpret_cast<const int4*>(vl + i);
                    vs += v4.x + v4.y + v4.z + v4.w;
                    cn += __popc(*reinterpret_cast<const uint32_t*>(fl + i));
                }
            } else {
                for (int i = 0; i < group_lanes; ++i) {
                    vs += vl[i];
                    cn += __popc((uint32_t)fl[i]);
                }
            }
            s_cnt[p * G + tid0 / group_lanes] = cn;
            const int64_t t0 = (int64_t)tile * blockDim.x + tid0;
            const int64_t sid0 = ((int64_t)(l0 + p) * n_qpt + (int)((t0 / strips) % n_qpt)) * strips + (int)(t0 % strips);
            grp_count[sid0 / group_lanes] = cn;
            grp_votes[sid0 / group_lanes] = vs;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int l = l0; l < l1; ++l) {
        const int64_t strip_id = ((int64_t)l * n_qpt + k) * strips + s;
        flags[strip_id] = s_flags[(l - l0) * kMarkThreads + threadIdx.x];
        if (stage_on && gq < min(s_cnt[(l - l0) * G + gi], capg))
            stage[(strip_id / group_lanes) * capg + gq] = s_val[((l - l0) * G + gi) * capg + gq];
    }
}

// Exclusive scans of the per-group candidate counts and vote sums into grp_off / grp_voff (the
// CSR base of each group), the candidate total into the status and the number of listed
// candidates into `misc`.  grid = (chunks, events): workgroup x scans the x-th of `chunks` equal
// ranges of the event's groups, starting from the sum of all groups before its range (loaded at
// once and reduced; a single event spreads over many CUs this way, a large batch uses one
// workgroup per event).  Each thread owns kPScanPer consecutive groups of a tile (vector loads and
// stores); the next tile's loads are issued before the current tile is scanned.
constexpr int kPScanPer = 8;
constexpr int kPScanThreads = 512;  // (1024 would cap the registers at 128 and spill)
constexpr int kPScanPrefixUnroll = 8;  // 16-byte loads per thread and round of the carry-in sum

__device__ __forceinline__ void load_groups(const int32_t* __restrict__ src, int64_t i0, int64_t n,
                                            int32_t (&v)[kPScanPer]) {
    if (i0 + kPScanPer <= n) {
        const int4* p = reinterpret_cast<const int4*>(src + i0);
#pragma unroll
        for (int q = 0; q < kPScanPer / 4; ++q) {
            const int4 t = p[q];
            v[4 * q] = t.x;
            v[4 * q + 1] = t.y;
            v[4 * q + 2] = t.z;
            v[4 * q + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kPScanPer; ++j) v[j] = i0 + j < n ? src[i0 + j] : 0;
    }
}

__global__ __launch_bounds__(kPScanThreads) void k_peaks_scan(Events ev, int64_t n_groups, int32_t cap,
                                                             char* __restrict__ ws, WsOff O,
                                                             hough_status_t* __restrict__ st_base) {
    __shared__ int64_t wsum_c[kPScanThreads / 64];
    __shared__ int64_t wsum_v[kPScanThreads / 64];
    const int e = blockIdx.y;
    char* w = event_ws(ws, ev, e);
    const int32_t* grp_count = at<int32_t>(w, O.grp_count);
    const int32_t* grp_votes = at<int32_t>(w, O.grp_votes);
    int32_t* grp_off = at<int32_t>(w, O.grp_off);
    int64_t* grp_voff = at<int64_t>(w, O.grp_voff);
    hough_status_t* st = st_base + e;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    constexpr int64_t tile = (int64_t)kPScanThreads * kPScanPer;
    // this workgroup's range [g0, g1) (a multiple of kPScanPer long, so vector loads stay aligned)
    const int64_t per = ((n_groups + gridDim.x - 1) / gridDim.x + kPScanPer - 1) / kPScanPer * kPScanPer;
    const int64_t g0 = min(n_groups, (int64_t)blockIdx.x * per);
    const int64_t g1 = min(n_groups, g0 + per);
    int32_t c[kPScanPer], v[kPScanPer];
    load_groups(grp_count, g0 + (int64_t)tid * kPScanPer, g1, c);
    load_groups(grp_votes, g0 + (int64_t)tid * kPScanPer, g1, v);
    // carry in: the sums over [0, g0), every load issued before the reduction
    int64_t carry_c = 0, carry_v = 0;
    if (g0 > 0) {
        int64_t pc = 0, pv = 0;
        for (int64_t i0 = 4 * (int64_t)tid; i0 < g0; i0 += 4 * kPScanThreads * kPScanPrefixUnroll) {
            int4 a[kPScanPrefixUnroll], b[kPScanPrefixUnroll];
#pragma unroll
            for (int u = 0; u < kPScanPrefixUnroll; ++u) {
                const int64_t j = min(i0 + 4 * (int64_t)kPScanThreads * u, g0 - 4);  // g0 is a multiple of 4
                a[u] = *reinterpret_cast<const int4*>(grp_count + j);
                b[u] = *reinterpret_cast<const int4*>(grp_votes + j);
            }
#pragma unroll
            for (int u = 0; u < kPScanPrefixUnroll; ++u) {
                if (i0 + 4 * (int64_t)kPScanThreads * u < g0) {
                    pc += (int64_t)a[u].x + a[u].y + a[u].z + a[u].w;
                    pv += (int64_t)b[u].x + b[u].y + b[u].z + b[u].w;
                }
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            pc += __shfl_xor(pc, o, 64);
            pv += __shfl_xor(pv, o, 64);
        }
        if (lane == 0) {
            wsum_c[wv] = pc;
            wsum_v[wv] = pv;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPScanThreads / 64; ++k) {
            carry_c += wsum_c[k];
            carry_v += wsum_v[k];
        }
        __syncthreads();  // wsum is reused by the scan
    }
    for (int64_t base = g0; base < g1; base += tile) {
        const int64_t i0 = base + (int64_t)tid * kPScanPer;
        int32_t sc = 0, sv = 0;  // a thread's groups hold < 2^31 candidates and votes
#pragma unroll
        for (int j = 0; j < kPScanPer; ++j) {
            sc += c[j];
            sv += v[j];
        }
        // inclusive scans of (sc, sv) over the workgroup
        int32_t ic = sc;
        int64_t iv = sv;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t uc = __shfl_up(ic, o, 64);
            const int64_t uv = __shfl_up(iv, o, 64);
            if (lane >= o) {
                ic += uc;
                iv += uv;
            }
        }
        if (lane == 63) {
            wsum_c[wv] = ic;
            wsum_v[wv] = iv;
        }
        __syncthreads();
        int64_t pc = 0, pv = 0, tc = 0, tv = 0;
#pragma unroll
        for (int k = 0; k < kPScanThreads / 64; ++k) {
            const int64_t a = wsum_c[k], b = wsum_v[k];
            pc += k < wv ? a : 0;
            pv += k < wv ? b : 0;
            tc += a;
            tv += b;
        }
        __syncthreads();  // wsum is rewritten by the next tile
        int64_t rc = carry_c + pc + ic - sc;
        int64_t rv = carry_v + pv + iv - sv;
        if (i0 + kPScanPer <= g1) {
#pragma unroll
            for (int q = 0; q < kPScanPer / 4; ++q) {
                int4 o4;
                longlong2 va, vb;
                o4.x = (int32_t)min(rc, (int64_t)INT32_MAX); va.x = rv; rc += c[4 * q]; rv += v[4 * q];
                o4.y = (int32_t)min(rc, (int64_t)INT32_MAX); va.y = rv; rc += c[4 * q + 1]; rv += v[4 * q + 1];
                o4.z = (int32_t)min(rc, (int64_t)INT32_MAX); vb.x = rv; rc += c[4 * q + 2]; rv += v[4 * q + 2];
                o4.w = (int32_t)min(rc, (int64_t)INT32_MAX); vb.y = rv; rc += c[4 * q + 3]; rv += v[4 * q + 3];
                reinterpret_cast<int4*>(grp_off + i0)[q] = o4;
                reinterpret_cast<longlong2*>(grp_voff + i0)[2 * q] = va;
                reinterpret_cast<longlong2*>(grp_voff + i0)[2 * q + 1] = vb;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kPScanPer; ++j) {
                if (i0 + j < g1) {
                    grp_off[i0 + j] = (int32_t)min(rc, (int64_t)INT32_MAX);
                    grp_voff[i0 + j] = rv;
                }
                rc += c[j];
                rv += v[j];
            }
        }
        carry_c += tc;
        carry_v += tv;
        if (base + tile < g1) {  // the next tile
            load_groups(grp_count, i0 + tile, g1, c);
            load_groups(grp_votes, i0 + tile, g1, v);
        }
    }
    if (tid == 0 && g1 == n_groups && (g0 < g1 || g0 == 0)) {  // the workgroup holding the last group
        grp_off[n_groups] = (int32_t)min(carry_c, (int64_t)INT32_MAX);
        grp_voff[n_groups] = carry_v;
        st->n_peaks = (int32_t)min(carry_c, (int64_t)INT32_MAX);
        *at<int32_t>(w, O.misc) = (int32_t)min(carry_c, (int64_t)cap);
        if (carry_c > cap) atomicOr(&st->flags, HOUGH_F_PEAK_OVERFLOW);
    }
}

// grid.y = event.  One thread per kWriteStrips consecutive strips (64 bins) of one group (fewer
// when a group is smaller): it loads their flag bytes and the values of the flagged bins, takes
// its candidates' position and vote prefix from the group's CSR bases plus an in-group scan over
// the group's threads, and writes its candidates and their CSR offsets in linear order.
constexpr int kWriteStrips = 8;
constexpr int kWriteFirst = 4;  // candidates per thread whose values are loaded together
constexpr int kWriteThreads = 256;

// The flagged bins of one thread's strips and the values of its first kWriteFirst candidates
// (their loads go out together; a bin with no candidate loads bin 0 of the range, unused).
template <typename T>
struct WriteItem {
    bool live;
    uint64_t bits, rest;
    int64_t row;
    int s0;
    const T* r;
    int32_t cnt, vsum;
    int idx[kWriteFirst];
    int32_t val[kWriteFirst];
};

template <typename T>
__device__ __forceinline__ void write_load(const T* acc, const uint8_t* flags, int64_t t, int64_t n_thr, int sp,
                                           int strips, int n_phi, WriteItem<T>& it) {
    it.live = t < n_thr;
    const int64_t strip0 = (it.live ? t : n_thr - 1) * sp;
    it.bits = 0;
    if (it.live) {
        if (sp == kWriteStrips) {
            it.bits = *reinterpret_cast<const uint64_t*>(flags + strip0);
        } else {
            for (int i = 0; i < sp; ++i) it.bits |= (uint64_t)flags[strip0 + i] << (8 * i);
        }
    }
    it.row = strip0 / strips;
    it.s0 = (int)(strip0 - it.row * strips);
    it.r = acc + it.row * n_phi + it.s0 * kStrip;
    it.cnt = __popcll(it.bits);
    it.rest = it.bits;
#pragma unroll
    for (int j = 0; j < kWriteFirst; ++j) {
        it.idx[j] = it.rest ? __ffsll((long long)it.rest) - 1 : 0;
        it.rest &= it.rest - 1;
    }
#pragma unroll
    for (int j = 0; j < kWriteFirst; ++j) it.val[j] = (int32_t)it.r[it.idx[j]];
    it.vsum = 0;
#pragma unroll
    for (int j = 0; j < kWriteFirst; ++j) it.vsum += j < it.cnt ? it.val[j] : 0;
    for (uint64_t b = it.rest; b; b &= b - 1) it.vsum += (int32_t)it.r[__ffsll((long long)b) - 1];
}

// In-group prefix over the group's tpg threads (consecutive lanes, all active), then the
// thread's candidates written from the group's CSR bases.
template <typename T>
__device__ __forceinline__ void write_emit(const WriteItem<T>& it, int32_t g_off, int64_t g_voff, int tpg, int n_qpt,
                                           hough_peak_t* peaks, int64_t* peak_voff, int32_t cap) {
    const int gl = threadIdx.x & (tpg - 1);
    int32_t inc = it.cnt, vinc = it.vsum;
    for (int o = 1; o < tpg; o <<= 1) {
        const int32_t a = __shfl_up(inc, o, tpg);
        const int32_t c = __shfl_up(vinc, o, tpg);
        if (gl >= o) {
            inc += a;
            vinc += c;
        }
    }
    if (!it.live || it.bits == 0) return;
    int32_t pos = g_off + inc - it.cnt;
    int64_t voff = g_voff + vinc - it.vsum;
    const int k = (int)(it.row % n_qpt);
    const int l = (int)(it.row / n_qpt);
    auto emit = [&](int i, int32_t v) {
        if (pos < cap) {
            hough_peak_t pk;
            pk.l = l;
            pk.k = k;
            pk.b = it.s0 * kStrip + i;
            pk.votes = v;
            peaks[pos] = pk;
            peak_voff[pos] = voff;
        }
        ++pos;
        voff += v;
    };
#pragma unroll
    for (int j = 0; j < kWriteFirst; ++j)
        if (j < it.cnt) emit(it.idx[j], it.val[j]);
    for (uint64_t b = it.rest; b; b &= b - 1) {
        const int i = __ffsll((long long)b) - 1;
        emit(i, (int32_t)it.r[i]);
    }
}

// The writer with the values the marker staged: a thread's first candidate inside its group comes
// from a scan of the strips' counts over the group's threads, its values from the stage (a group
// with more candidates than the stage holds reads them from the accumulator), then a scan of the
// vote sums gives their CSR offsets.  Every thread of the workgroup takes part in the scans.
template <typename T>
struct StagedItem {
    bool live, staged;
    uint64_t bits, rest;
    int cnt, pos0, s0;
    int64_t row;
    const T* r;
    const uint16_t* sv;
    int32_t val[kWriteFirst];
    int32_t vsum, vpre;
};

template <typename T>
__device__ __forceinline__ void staged_load(const T* acc, const uint8_t* flags, const uint16_t* stage, int capg,
                                            int64_t t, int64_t n_thr, int sp, int tpg, int strips, int n_phi,
                                            StagedItem<T>& it) {
    it.live = t < n_thr;
    const int64_t tc = it.live ? t : n_thr - 1;
    const int64_t strip0 = tc * sp;
    it.bits = 0;
    if (it.live) {
        if (sp == kWriteStrips) {
            it.bits = *reinterpret_cast<const uint64_t*>(flags + strip0);
        } else {
            for (int i = 0; i < sp; ++i) it.bits |= (uint64_t)flags[strip0 + i] << (8 * i);
        }
    }
    it.cnt = __popcll(it.bits);
    const int gl = threadIdx.x & (tpg - 1);
    int inc = it.cnt;
    for (int o = 1; o < tpg; o <<= 1) {
        const int a = __shfl_up(inc, o, tpg);
        if (gl >= o) inc += a;
    }
    const int gtot = __shfl(inc, tpg - 1, tpg);
    it.pos0 = inc - it.cnt;
    it.staged = gtot <= capg;
    it.row = strip0 / strips;
    it.s0 = (int)(strip0 - it.row * strips);
    it.r = acc + it.row * n_phi + it.s0 * kStrip;
    it.sv = stage + (tc / tpg) * capg + it.pos0;
    it.rest = it.bits;
    int idx[kWriteFirst];
#pragma unroll
    for (int j = 0; j < kWriteFirst; ++j) {
        idx[j] = it.rest ? __ffsll((long long)it.rest) - 1 : 0;
        it.rest &= it.rest - 1;
    }
#pragma unroll
    for (int j = 0; j < kWriteFirst; ++j)
        it.val[j] = j < it.cnt ? (it.staged ? (int32_t)it.sv[j] : (int32_t)it.r[idx[j]]) : 0;
    it.vsum = 0;
#pragma unroll
    for (int j = 0; j < kWriteFirst; ++j) it.vsum += it.val[j];
    int j = kWriteFirst;
    for (uint64_t b = it.rest; b; b &= b - 1, ++j)
        it.vsum += it.staged ? (int32_t)it.sv[j] : (int32_t)it.r[__ffsll((long long)b) - 1];
    int32_t vinc = it.vsum;
    for (int o = 1; o < tpg; o <<= 1) {
        const int32_t c = __shfl_up(vinc, o, tpg);
        if (gl >= o) vinc += c;
    }
    it.vpre = vinc - it.vsum;
}

template <typename T>
__device__ __forceinline__ void staged_emit(const StagedItem<T>& it, int32_t g_off, int64_t g_voff, int n_qpt,
                                            hough_peak_t* peaks, int64_t* peak_voff, int32_t cap) {
    if (!it.live || it.bits == 0) return;
    int32_t pos = g_off + it.pos0;
    int64_t voff = g_voff + it.vpre;
    const int k = (int)(it.row % n_qpt);
    const int l = (int)(it.row / n_qpt);
    int j = 0;
    for (uint64_t b = it.bits; b; b &= b - 1, ++j) {
        const int i = __ffsll((long long)b) - 1;
        const int32_t v = j < kWriteFirst ? it.val[j] : (it.staged ? (int32_t)it.sv[j] : (int32_t)it.r[i]);
        if (pos < cap) {
            hough_peak_t pk;
            pk.l = l;
            pk.k = k;
            pk.b = it.s0 * kStrip + i;
            pk.votes = v;
            peaks[pos] = pk;
            peak_voff[pos] = voff;
        }
        ++pos;
        voff += v;
    }
}

template <typename T>
__global__ __launch_bounds__(kWriteThreads) void k_peaks_write(Events ev, const char* __restrict__ acc_base,
                                                               size_t acc_stride, int64_t n_groups, int n_qpt,
                                                               int n_phi, int group_lanes, int64_t n_strips,
                                                               bool stage_on, char* __restrict__ ws, WsOff O,
                                                               hough_peak_t* __restrict__ peaks_base, int32_t cap) {
    const int e = blockIdx.y;
    const T* acc = reinterpret_cast<const T*>(acc_base + (size_t)e * acc_stride);
    char* w = event_ws(ws, ev, e);
    const uint8_t* flags = at<uint8_t>(w, O.flags);
    const int32_t* grp_off = at<int32_t>(w, O.grp_off);
    const int64_t* grp_voff = at<int64_t>(w, O.grp_voff);
    const int strips = n_phi / kStrip;
    const int sp = min(kWriteStrips, group_lanes);  // strips per thread (both powers of two)
    const int tpg = group_lanes / sp;              // threads per group (1..8)
    const int64_t n_thr = n_strips / sp;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the group's CSR bases do not depend on the flags: load them together
    const int64_t g = (t < n_thr ? t : n_thr - 1) / tpg;
    const int32_t g_off = grp_off[g];
    const int64_t g_voff = grp_voff[g];
    if (stage_on) {
        StagedItem<T> it;
        staged_load(acc, flags, at<const uint16_t>(w, O.stage), stage_cap(group_lanes), t, n_thr, sp, tpg, strips,
                    n_phi, it);
        staged_emit(it, g_off, g_voff, n_qpt, peaks_base + (size_t)e * cap, at<int64_t>(w, O.peak_voff), cap);
        return;
    }
    WriteItem<T> it;
    write_load(acc, flags, t, n_thr, sp, strips, n_phi, it);
    write_emit(it, g_off, g_voff, tpg, n_qpt, peaks_base + (size_t)e * cap, at<int64_t>(w, O.peak_voff), cap);
}

// The CSR scan and the writer in one pass for a single event or a small batch (grid as the
// writer's): a workgroup owns kWriteThreads / tpg whole groups; it sums the candidate counts
// and votes of every group before its own (all loads issued at once, then one workgroup
// reduction), scans its own groups in LDS, and writes their candidates.  The workgroup holding
// the last group sets the event's totals.  Every workgroup re-reads the counts before it, which
// is cheap for one event and not for hundreds, so large batches use the two kernels above.
constexpr int kCarryUnroll = 8;         // 16-byte loads per thread and round of the carry-in sum
constexpr int kScanWriteMaxEvents = 4;  // batches up to this size take the one-pass form
constexpr int64_t kScanWriteMaxGroups = 32768;  // groups of a 512x256x64 grid: 16384; of 1024x512x128: 131072

template <typename T>
__global__ __launch_bounds__(kWriteThreads) void k_peaks_scan_write(Events ev, const char* __restrict__ acc_base,
                                                                    size_t acc_stride, int64_t n_groups, int n_qpt,
                                                                    int n_phi, int group_lanes, int64_t n_strips,
                                                                    bool stage_on, char* __restrict__ ws, WsOff O,
                                                                    hough_peak_t* __restrict__ peaks_base,
                                                                    int32_t cap, hough_status_t* __restrict__ st_base) {
    __shared__ int64_t red_c[kWriteThreads / 64], red_v[kWriteThreads / 64];
    __shared__ int32_t s_off[kWriteThreads];
    __shared__ int64_t s_voff[kWriteThreads];
    const int e = blockIdx.y;
    const T* acc = reinterpret_cast<const T*>(acc_base + (size_t)e * acc_stride);
    char* w = event_ws(ws, ev, e);
    const uint8_t* flags = at<uint8_t>(w, O.flags);
    const int32_t* grp_count = at<int32_t>(w, O.grp_count);
    const int32_t* grp_votes = at<int32_t>(w, O.grp_votes);
    const int strips = n_phi / kStrip;
    const int sp = min(kWriteStrips, group_lanes);
    const int tpg = group_lanes / sp;
    const int64_t n_thr = n_strips / sp;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int gpb = kWriteThreads / tpg;                 // groups per workgroup (a multiple of 32)
    const int64_t gb = (int64_t)blockIdx.x * gpb;        // first group of this workgroup
    const int64_t t = (int64_t)blockIdx.x * kWriteThreads + tid;
    WriteItem<T> it;
    StagedItem<T> si;
    if (stage_on)
        staged_load(acc, flags, at<const uint16_t>(w, O.stage), stage_cap(group_lanes), t, n_thr, sp, tpg, strips,
                    n_phi, si);
    else
        write_load(acc, flags, t, n_thr, sp, strips, n_phi, it);
    // own groups' counts, and the carry-in over [0, gb) (gb is a multiple of 4)
    const bool own = tid < gpb && gb + tid < n_groups;
    const int32_t oc = own ? grp_count[gb + tid] : 0;
    const int32_t ov = own ? grp_votes[gb + tid] : 0;
    int64_t pc = 0, pv = 0;
    for (int64_t i0 = 4 * (int64_t)tid; i0 < gb; i0 += 4 * kWriteThreads * kCarryUnroll) {
        int4 a[kCarryUnroll], b[kCarryUnroll];
#pragma unroll
        for (int u = 0; u < kCarryUnroll; ++u) {
            const int64_t j = min(i0 + 4 * (int64_t)kWriteThreads * u, gb - 4);
            a[u] = *reinterpret_cast<const int4*>(grp_count + j);
            b[u] = *reinterpret_cast<const int4*>(grp_votes + j);
        }
#pragma unroll
        for (int u = 0; u < kCarryUnroll; ++u) {
            if (i0 + 4 * (int64_t)kWriteThreads * u < gb) {
                pc += (int64_t)a[u].x + a[u].y + a[u].z + a[u].w;
                pv += (int64_t)b[u].x + b[u].y + b[u].z + b[u].w;
            }
        }
    }
    // inclusive scans of the own counts inside each wave, totals of the carry per wave
    int32_t ic = oc;
    int64_t iv = ov;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t uc = __shfl_up(ic, o, 64);
        const int64_t uv = __shfl_up(iv, o, 64);
        if (lane >= o) {
            ic += uc;
            iv += uv;
        }
        pc += __shfl_xor(pc, o, 64);
        pv += __shfl_xor(pv, o, 64);
    }
    __shared__ int64_t wown_c[kWriteThreads / 64], wown_v[kWriteThreads / 64];
    if (lane == 63) {
        wown_c[wv] = ic;
        wown_v[wv] = iv;
    }
    if (lane == 0) {
        red_c[wv] = pc;
        red_v[wv] = pv;
    }
    __syncthreads();
    int64_t carry_c = 0, carry_v = 0, pre_c = 0, pre_v = 0, tot_c = 0, tot_v = 0;
#pragma unroll
    for (int k = 0; k < kWriteThreads / 64; ++k) {
        carry_c += red_c[k];
        carry_v += red_v[k];
        pre_c += k < wv ? wown_c[k] : 0;
        pre_v += k < wv ? wown_v[k] : 0;
        tot_c += wown_c[k];
        tot_v += wown_v[k];
    }
    if (tid < gpb) {
        s_off[tid] = (int32_t)min(carry_c + pre_c + ic - oc, (int64_t)INT32_MAX);
        s_voff[tid] = carry_v + pre_v + iv - ov;
    }
    if (tid == 0 && gb < n_groups && gb + gpb >= n_groups) {  // the workgroup holding the last group
        const int64_t total = carry_c + tot_c;
        hough_status_t* st = st_base + e;
        st->n_peaks = (int32_t)min(total, (int64_t)INT32_MAX);
        *at<int32_t>(w, O.misc) = (int32_t)min(total, (int64_t)cap);
        if (total > cap) atomicOr(&st->flags, HOUGH_F_PEAK_OVERFLOW);
    }
    __syncthreads();
    const int gi = (int)(((t < n_thr ? t : n_thr - 1) / tpg) - gb);  // this thread's group, local
    const int gl = min(max(gi, 0), gpb - 1);
    if (stage_on)
        staged_emit(si, s_off[gl], s_voff[gl], n_qpt, peaks_base + (size_t)e * cap, at<int64_t>(w, O.peak_voff), cap);
    else
        write_emit(it, s_off[gl], s_voff[gl], tpg, n_qpt, peaks_base + (size_t)e * cap, at<int64_t>(w, O.peak_voff),
                   cap);
}

// ------------------------------------------------------------------ assign
typedef __attribute__((address_space(3))) const uint32_t lds_cu32;
typedef __attribute__((address_space(3))) const int32_t lds_ci32;

// Views of the event's sorted hits (angle and hit index at a sorted position): two LDS arrays,
// one packed LDS word per hit (angle in the low 16 bits, hit index in the high 16 bits: plans with
// M <= 16 angle bits, whose events have at most 65535 hits), or the workspace arrays.
struct HitsSplit {
    lds_cu32* phi;
    lds_ci32* h;
    __device__ __forceinline__ uint32_t angle(int i) const { return phi[i]; }
    __device__ __forceinline__ int32_t hit(int i) const { return h[i]; }
};
struct HitsPacked {
    lds_cu32* w;
    __device__ __forceinline__ uint32_t angle(int i) const { return w[i] & 0xFFFFu; }
    __device__ __forceinline__ int32_t hit(int i) const { return (int32_t)(w[i] >> 16); }
};
struct HitsGlobal {
    const uint32_t* __restrict__ phi;
    const int32_t* __restrict__ h;
    __device__ __forceinline__ uint32_t angle(int i) const { return phi[i]; }
    __device__ __forceinline__ int32_t hit(int i) const { return h[i]; }
};

// The list of one candidate, layer by layer: the run(s) of sorted hits with angle in
// [lo, lo + 2^F) (mod 2^M), lo = E + b * 2^F, found from the cell table and a short scan, copied in
// order to the wave's LDS buffer (or straight to memory beyond it).
// First index of cell c (hits [cs[c], cs[c+1]) sorted by angle) whose angle is >= x.  SCAN8 (LDS
// views only): the first 8 entries of the cell are compared at once (independent loads, no
// divergent loop; the cells hold about two hits on average), a longer cell continues one by one.
template <bool SCAN8, typename View>
__device__ __forceinline__ int cell_lower_bound(const int32_t* cs, int c, const View& hv, uint32_t x) {
    const int a = cs[c];
    const int n_in = cs[c + 1] - a;
    if (!SCAN8) {
        int q = a;
        while (q < a + n_in && hv.angle(q) < x) ++q;
        return q;
    }
    // all eight loads are issued before any compare (a load under `i < n_in` would wait on its
    // own); the staged arrays leave room for reads up to 8 entries past the last hit
    uint32_t v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = hv.angle(a + i);
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) cnt += (int)((i < n_in) & (v[i] < x));
    if (n_in > 8 && cnt == 8)
        while (cnt < n_in && hv.angle(a + cnt) < x) ++cnt;
    return a + cnt;
}

template <bool SCAN8, typename View>
__device__ __forceinline__ void assign_candidate(const hough_peak_t& pk, int64_t off, int64_t o0, const int32_t* Ec,
                                                 int n_layers, int cell_bits, int n_cols, int M, int F,
                                                 const int32_t* cell_start, const View& hv,
                                                 int32_t* buf, int buf_words, int32_t* hit_idx, int32_t cap_pairs) {
    const uint32_t span = 1u << M;
    const uint32_t W = 1u << F;
    const int cshift = M - cell_bits;
    int32_t ev_l[kMaxLayers];
#pragma unroll
    for (int L = 0; L < kMaxLayers; ++L) ev_l[L] = L < n_layers ? Ec[(size_t)L * n_cols] : INT32_MIN;
    int64_t wpos = off;
#pragma unroll
    for (int L = 0; L < kMaxLayers; ++L) {
        if (L >= n_layers || wpos >= cap_pairs) break;
        if (ev_l[L] == INT32_MIN) continue;
        const uint32_t lo = ((uint32_t)ev_l[L] + ((uint32_t)pk.b << F)) & (span - 1u);
        const uint32_t hi = lo + W;  // may exceed 2^M: the window wraps
        // the window's first and last hits lie in the cells of its two ends: every hit of a later
        // cell has a larger angle than the window's start, every hit of an earlier cell a smaller one
        const int32_t* cs = cell_start + (L << cell_bits);
        const int lay_end = cs[1 << cell_bits];
        const int q = cell_lower_bound<SCAN8>(cs, (int)(lo >> cshift), hv, lo);
        const uint32_t he = hi <= span ? hi : span;
        const int z = he < span ? cell_lower_bound<SCAN8>(cs, (int)(he >> cshift), hv, he) : lay_end;
        int r = -1, z2 = -1;
        if (hi > span) {
            const uint32_t hw = hi - span;
            r = cs[0];
            z2 = cell_lower_bound<SCAN8>(cs, (int)(hw >> cshift), hv, hw);
        }
        // copy the run(s) four entries at a time: the four loads go out before the four stores
        for (int seg = 0; seg < 2; ++seg) {
            const int a0 = seg == 0 ? q : r;
            const int a1 = seg == 0 ? z : z2;
            for (int j = a0; j < a1; j += 4) {
                int32_t h[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) h[u] = hv.hit(min(j + u, a1 - 1));
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t wp = wpos + (j - a0) + u;
                    if (j + u < a1 && wp < cap_pairs) {
                        const int64_t rel = wp - o0;
                        if (rel < buf_words) buf[rel] = h[u];
                        else hit_idx[wp] = h[u];
                    }
                }
            }
            wpos += a1 > a0 ? a1 - a0 : 0;
        }
    }
}

// Copies the cell table (nc words) and, when staged, the event's nh sorted angles and hit indices
// from global memory to LDS: as two arrays, or (PACK) as one word per hit.  16 bytes per load,
// with all of a thread's loads of a round issued before its first store (a load-then-store loop
// would wait on memory once per element).  Sources and destinations are 16-byte aligned; a source
// is read up to the next multiple of four words (inside its 256-byte padded workspace array).
constexpr int kStageUnroll = 8;  // 16-byte loads per thread and round: 128 KiB per round at 1024 threads

template <bool PACK>
__device__ __forceinline__ void assign_stage(int32_t* d_cells, const int32_t* __restrict__ g_cells, int nc,
                                             uint32_t* d_stage, int stage_stride, const uint32_t* __restrict__ g_phi,
                                             const int32_t* __restrict__ g_h, int nh, int tid) {
    const int c4 = (nc + 3) >> 2;
    const int h4 = (nh + 3) >> 2;
    const int total = c4 + (PACK ? h4 : 2 * h4);
    for (int r0 = tid; r0 < total; r0 += kStageUnroll * kAssignThreads) {
        uint4 v[kStageUnroll], w[kStageUnroll];
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            const int c = min(r0 + u * kAssignThreads, total - 1);
            if (PACK) {
                const int k = c < c4 ? 0 : c - c4;
                v[u] = c < c4 ? reinterpret_cast<const uint4*>(g_cells)[c] : reinterpret_cast<const uint4*>(g_phi)[k];
                w[u] = reinterpret_cast<const uint4*>(g_h)[k];
            } else {
                const uint4* src = c < c4 ? reinterpret_cast<const uint4*>(g_cells) + c
                                 : c < c4 + h4 ? reinterpret_cast<const uint4*>(g_phi) + (c - c4)
                                               : reinterpret_cast<const uint4*>(g_h) + (c - c4 - h4);
                v[u] = *src;
            }
        }
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            const int c = r0 + u * kAssignThreads;
            if (c < total) {
                if (c < c4) {
                    reinterpret_cast<uint4*>(d_cells)[c] = v[u];
                } else if (PACK) {
                    uint4 o;
                    o.x = v[u].x | (w[u].x << 16);
                    o.y = v[u].y | (w[u].y << 16);
                    o.z = v[u].z | (w[u].z << 16);
                    o.w = v[u].w | (w[u].w << 16);
                    reinterpret_cast<uint4*>(d_stage)[c - c4] = o;
                } else {
                    const int k = c - c4;  // angles, then the hit indices stage_stride words later
                    reinterpret_cast<uint4*>(d_stage + (k < h4 ? 0 : stage_stride))[k < h4 ? k : k - h4] = v[u];
                }
            }
        }
    }
}

// One thread per listed candidate (the first min(listed, cap_peaks) written by the peaks pass;
// grid.y = event): CSR offset from the peaks pass, then its list (assign_candidate).  The 64
// candidates of a wave own one contiguous stretch of the CSR list: it is assembled in an LDS
// buffer of the wave and then written with coalesced stores.  Each workgroup lays out its LDS
// from its event's hit count: the cell table, the event's sorted hits when they fit (one word per
// hit with PACK, else two), and the 16 wave buffers in what is left, up to kAssignBufMax words
// each (a longer stretch goes on straight to memory); so the scans and copies do not wait on
// memory.  The per-layer sample values of a candidate are loaded together, and a wave's next 64
// candidates are loaded while it works on the current ones.
template <bool PACK>
__global__ __launch_bounds__(kAssignThreads) void k_assign_fill(
    Events ev, const hough_peak_t* __restrict__ peaks_base, int32_t peak_stride, int32_t cap_peaks,
    hough_status_t* __restrict__ st_base, const int32_t* __restrict__ E, int n_layers, int cell_bits, int n_cols,
    int n_qpt, int M, int F, char* __restrict__ ws, WsOff O, int32_t* __restrict__ offsets_base,
    int32_t* __restrict__ hit_idx_base, int32_t cap_pairs, int lds_words, int cells_words) {
    extern __shared__ int32_t sm_i32[];
    constexpr int kWaves = kAssignThreads / 64;
    const int e = blockIdx.y;
    char* w = event_ws(ws, ev, e);
    const hough_peak_t* peaks = peaks_base + (size_t)e * peak_stride;
    const int64_t* peak_voff = at<int64_t>(w, O.peak_voff);
    const int32_t* g_cell_start = at<int32_t>(w, O.cell_start);
    const uint32_t* sorted_phi = at<uint32_t>(w, O.sorted_phi);
    const int32_t* sorted_h = at<int32_t>(w, O.sorted_h);
    int32_t* offsets = offsets_base + (size_t)e * (cap_peaks + 1);
    int32_t* hit_idx = hit_idx_base + (size_t)e * cap_pairs;
    hough_status_t* st = st_base + e;
    const int n = min(*at<int32_t>(w, O.misc), cap_peaks);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (blockIdx.x == 0 && tid == 0) {
        const int64_t tot = n > 0 ? peak_voff[n - 1] + peaks[n - 1].votes : 0;
        offsets[n] = (int32_t)min(tot, (int64_t)INT32_MAX);
        st->n_pairs = tot;
        if (tot > cap_pairs) atomicOr(&st->flags, HOUGH_F_PAIR_OVERFLOW);
    }
    if ((int)blockIdx.x * kAssignThreads >= n) return;  // uniform per block
    const int n_cells = n_layers << cell_bits;
    const int n_valid = g_cell_start[n_cells];
    // LDS layout of this event: cells [cells_words] | staged hits [stage_words] | 16 buffers; the
    // staged arrays hold n_pad >= n_valid + 8 entries (the 8-entry scan reads past the last hit)
    const int n_pad = ((n_valid + 3) & ~3) + 8;
    const int stage_words = PACK ? n_pad : 2 * n_pad;
    int buf_words = min(kAssignBufMax, (lds_words - cells_words - stage_words) / kWaves) & ~63;
    const bool staged = buf_words >= kAssignBufMin;
    if (!staged) buf_words = min(kAssignBufMax, (lds_words - cells_words) / kWaves) & ~63;
    int32_t* cell_start = sm_i32;
    uint32_t* s_stage = reinterpret_cast<uint32_t*>(sm_i32 + cells_words);
    int32_t* buf = sm_i32 + cells_words + (staged ? stage_words : 0) + wave * buf_words;
    const int stride = gridDim.x * kAssignThreads;
    int base = blockIdx.x * kAssignThreads + wave * 64;
    // the wave's first candidates: their loads overlap the staging
    hough_peak_t pk{};
    int64_t off = 0;
    if (base < n) {
        const int i = min(base + lane, n - 1);
        pk = peaks[i];
        off = peak_voff[i];
    }
    assign_stage<PACK>(cell_start, g_cell_start, n_cells + 1, s_stage, n_pad, sorted_phi, sorted_h,
                       staged ? n_valid : 0, tid);
    __syncthreads();
    for (; base < n; base += stride) {
        const int i = base + lane;
        const int last = min(n, base + 64) - 1;
        // the wave's stretch of the list, [o0, o1): from the first and last lanes' candidates
        const int64_t o0 = __shfl(off, 0, 64);
        const int64_t o1 = __shfl(off, last - base, 64) + __shfl(pk.votes, last - base, 64);
        const hough_peak_t cur = pk;
        const int64_t cur_off = off;
        if (base + stride < n) {  // the wave's next candidates (wave-uniform)
            const int i2 = min(base + stride + lane, n - 1);
            pk = peaks[i2];
            off = peak_voff[i2];
        }
        if (i < n) {
            offsets[i] = (int32_t)min(cur_off, (int64_t)INT32_MAX);
            const int32_t* Ec = E + (size_t)cur.l * n_qpt + cur.k;
            if (staged && PACK)
                assign_candidate<true>(cur, cur_off, o0, Ec, n_layers, cell_bits, n_cols, M, F, cell_start,
                                       HitsPacked{(lds_cu32*)s_stage}, buf, buf_words, hit_idx, cap_pairs);
            else if (staged)
                assign_candidate<true>(cur, cur_off, o0, Ec, n_layers, cell_bits, n_cols, M, F, cell_start,
                                       HitsSplit{(lds_cu32*)s_stage, (lds_ci32*)(s_stage + n_pad)}, buf, buf_words,
                                       hit_idx, cap_pairs);
            else
                assign_candidate<false>(cur, cur_off, o0, Ec, n_layers, cell_bits, n_cols, M, F, cell_start,
                                        HitsGlobal{sorted_phi, sorted_h}, buf, buf_words, hit_idx, cap_pairs);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // coalesced flush of the buffered part of the stretch
        const int64_t fe = min(min(o1, o0 + buf_words), (int64_t)cap_pairs);
        for (int64_t wq = o0 + lane; wq < fe; wq += 64) hit_idx[wq] = buf[wq - o0];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Assignment from the window table (plans with the table, see k_prep_fine).  The hits of layer L in the
// window of candidate (l, k, b) are sorted positions: with x = (E mod 2^M) + b * W = r + j * W,
// the run [PT[L][r][j], PT[L][r][j + 1]) of the layer (relative to its first sorted hit); a window
// that passes the turn (j = n_phi - 1) is the run from PT[L][r][j] to the layer's end followed by
// [0, PT[L][r][0]) (the hits below angle r).  One 8-byte table load per layer (the dword pair
// holding entries j and j + 1; a wrapping window loads entry 0 as well) replaces the searches of
// k_assign_fill; the layers are taken ten at a time so that their loads are in flight together.
typedef __attribute__((address_space(3))) const uint16_t lds_cu16;

// hit_run(i, a1): entry i of a run ending at a1, read up to two entries past a1 (the staged LDS
// view reads them, as the LDS past the staged hits is the wave buffers; the global view clamps).
struct HitsU16 {
    lds_cu16* h;
    __device__ __forceinline__ int32_t hit(int i) const { return (int32_t)h[i]; }
    __device__ __forceinline__ int32_t hit_run(int i, int) const { return (int32_t)h[i]; }
};
struct HitsIdx {
    const int32_t* __restrict__ h;
    __device__ __forceinline__ int32_t hit(int i) const { return h[i]; }
    __device__ __forceinline__ int32_t hit_run(int i, int a1) const { return h[min(i, a1 - 1)]; }
};

constexpr int kAssignLayerChunk = 10;

// Copies entries [a0, a1) of the sorted hits to CSR positions from wpos on: the first n_buf of them
// into the wave's buffer (index rel), the rest straight to memory, none past cap_pairs (the counts are
// split once per run, so the copy loops carry no per-entry tests).  Reads may run up to two
// entries past a1 (inside the LDS, or clamped for the global view); whole quads of writes are
// unconditional.
template <typename View>
__device__ __forceinline__ void pt_copy_run(int a0, int a1, int32_t wpos, int32_t o0, const View& hv, int32_t* buf,
                                            int buf_words, int32_t* hit_idx, int32_t cap_pairs) {
    const int n_e = min(a1 - a0, cap_pairs - wpos);  // entries written (wpos <= cap_pairs here)
    if (n_e <= 0) return;
    const int rel = wpos - o0;
    const int n_buf = max(0, min(n_e, buf_words - rel));
    int t = 0;
    for (; t + 4 <= n_buf; t += 4) {
        int32_t h[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) h[v] = hv.hit_run(a0 + t + v, a1);
#pragma unroll
        for (int v = 0; v < 4; ++v) buf[rel + t + v] = h[v];
    }
    if (t < n_buf) {
        int32_t h[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) h[v] = hv.hit_run(a0 + t + v, a1);
#pragma unroll
        for (int v = 0; v < 3; ++v)
            if (t + v < n_buf) buf[rel + t + v] = h[v];
        t = n_buf;
    }
    for (; t < n_e; ++t) hit_idx[wpos + t] = hv.hit_run(a0 + t, a1);  // past the wave's buffer
}

// The samples of a candidate's column for the layers [L0, L0 + kAssignLayerChunk) from the column-major
// copy of the sample table (INT32_MIN past the last layer: no test per layer, contiguous loads).
__device__ __forceinline__ void col_samples(const int32_t* __restrict__ Ecol, int L0,
                                            int32_t (&ev)[kAssignLayerChunk]) {
    __builtin_memcpy(ev, Ecol + L0, sizeof(ev));
}

// ev0: the candidate's samples of its first kAssignLayerChunk layers (loaded ahead by the caller);
// Ecol: its column in the column-major sample table, for further layers.
template <typename View>
__device__ __forceinline__ void assign_candidate_pt(const hough_peak_t& pk, int64_t off, int64_t o0,
                                                    const int32_t* __restrict__ Ecol,
                                                    const int32_t (&ev0)[kAssignLayerChunk],
                                                    int n_layers, int M, int F, int n_phi, int row,
                                                    const uint16_t* __restrict__ pt, const int32_t* lay_start,
                                                    const View& hv, int32_t* buf, int buf_words, int32_t* hit_idx,
                                                    int32_t cap_pairs) {
    constexpr int LC = kAssignLayerChunk;
    const uint32_t mmask = (1u << M) - 1u, wmask = (1u << F) - 1u;
    if (off >= cap_pairs) return;
    // positions below cap_pairs fit 32 bits, and so does the wave's first position o0 <= off
    int32_t wpos = (int32_t)off;
    const int32_t o0_32 = (int32_t)o0;
    for (int L0 = 0; L0 < n_layers; L0 += LC) {
        if (wpos >= cap_pairs) break;
        int32_t ev_l[LC];
        if (L0 == 0) {
#pragma unroll
            for (int u = 0; u < LC; ++u) ev_l[u] = ev0[u];
        } else {
            col_samples(Ecol, L0, ev_l);
        }
        uint32_t lh[LC];  // lo | hi << 16: the run's first and end entries in the layer
        uint32_t wr = 0;  // layers whose window passes the turn
#pragma unroll
        for (int u = 0; u < LC; ++u) {
            // every load is in bounds (an invalid sample still gives an angle below 2^M; the pair of
            // a row's last entry reaches one dword past the row, into the next row or the window
            // counts that follow the table in the workspace)
            const uint32_t x = ((uint32_t)ev_l[u] + ((uint32_t)pk.b << F)) & mmask;
            const uint32_t r = x & wmask, j = x >> F;
            const int Lc = min(L0 + u, n_layers - 1);
            // the row offset fits 32 bits (fewer than 2^31 table entries per event)
            const uint32_t* rp = reinterpret_cast<const uint32_t*>(pt + ((((uint32_t)Lc << F) | r) * (uint32_t)n_phi));
            wr |= ((int)j == n_phi - 1 ? 1u : 0u) << u;
            uint2 v;
            __builtin_memcpy(&v, rp + (j >> 1), 8);
            // entries j and j + 1 of the row: the dword's halves for even j, else its high half and
            // the next dword's low half.  A byte shift rather than a select on the parity of j: with a
            // select the compiler would load the second dword only in the odd branch and wait for it
            // there, one layer after another, instead of keeping all the layers' loads in flight.
            lh[u] = __builtin_amdgcn_alignbyte(v.y, v.x, (j & 1u) * 2u);
        }
#pragma unroll
        for (int u = 0; u < LC; ++u) {
            if (wr & (1u << u)) {  // the window passes the turn: it ends at entry 0 of the row
                const uint32_t r = ((uint32_t)ev_l[u] + ((uint32_t)pk.b << F)) & wmask;
                const int Lc = min(L0 + u, n_layers - 1);
                lh[u] = (lh[u] & 0xFFFFu) | ((uint32_t)pt[(((uint32_t)Lc << F) | r) * (uint32_t)n_phi] << 16);
            }
        }
#pragma unroll
        for (int u = 0; u < LC; ++u) {
            const int L = L0 + u;
            if (L >= n_layers || ev_l[u] == INT32_MIN) continue;
            const int base = lay_start[L];
            const int lo_u = (int)(lh[u] & 0xFFFFu), hi_u = (int)(lh[u] >> 16);
            if (!(wr & (1u << u))) {
                const int a0 = base + lo_u, a1 = base + hi_u;
                pt_copy_run(a0, a1, wpos, o0_32, hv, buf, buf_words, hit_idx, cap_pairs);
                wpos = (int32_t)min((int64_t)wpos + (a1 - a0), (int64_t)cap_pairs);
            } else {  // the run to the layer's end, then the layer's first entries
                const int a0 = base + lo_u, a1 = lay_start[L + 1];
                pt_copy_run(a0, a1, wpos, o0_32, hv, buf, buf_words, hit_idx, cap_pairs);
                wpos = (int32_t)min((int64_t)wpos + (a1 - a0), (int64_t)cap_pairs);
                pt_copy_run(base, base + hi_u, wpos, o0_32, hv, buf, buf_words, hit_idx, cap_pairs);
                wpos = (int32_t)min((int64_t)wpos + hi_u, (int64_t)cap_pairs);
            }
        }
    }
}

// One thread per listed candidate (grid.y = event), as k_assign_fill: the 64 candidates of a wave
// own one contiguous stretch of the CSR list, assembled in the wave's LDS buffer and stored
// coalesced.  LDS: the layers' first sorted positions, then the event's sorted hit indices as 16-bit
// values (staged when they leave room for buffers of kAssignBufMin words), then THREADS / 64 wave
// buffers.  THREADS = 1024 with the whole LDS for a single event, 512 with half of it for batches.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_assign_pt(
    Events ev, const hough_peak_t* __restrict__ peaks_base, int32_t peak_stride, int32_t cap_peaks,
    hough_status_t* __restrict__ st_base, const int32_t* __restrict__ Et, int et_stride, int n_layers, int cell_bits,
    int n_cols,
    int n_qpt, int M, int F, int n_phi, int row, char* __restrict__ ws, WsOff O,
    int32_t* __restrict__ offsets_base, int32_t* __restrict__ hit_idx_base, int32_t cap_pairs, int lds_words,
    const int32_t* __restrict__ order, int n_events) {
    extern __shared__ int32_t sm_i32[];
    constexpr int kWaves = THREADS / 64;
    constexpr int kHead = 64;  // words for the layer starts (n_layers + 1 <= 33)
    // workgroup bx of event e; with `order` (batches, grid.y a multiple of 8), all workgroups of one
    // event run on one XCD (see xcd_rank): linear index L -> XCD L % 8, its (L / 8)-th workgroup
    int bx = (int)blockIdx.x, e = (int)blockIdx.y;
    if (order) {
        const int64_t L = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        const int64_t k = L / kXcds;
        const int rank = xcd_rank((int)(k / gridDim.x), (int)(L % kXcds));
        if (rank >= n_events) return;  // padding of the last group of eight events
        e = order[rank];
        bx = (int)(k % gridDim.x);
    }
    char* w = event_ws(ws, ev, e);
    const hough_peak_t* peaks = peaks_base + (size_t)e * peak_stride;
    const int64_t* peak_voff = at<int64_t>(w, O.peak_voff);
    const int32_t* g_cell_start = at<int32_t>(w, O.cell_start);
    const int32_t* sorted_h = at<int32_t>(w, O.sorted_h);
    const uint16_t* pt = at<const uint16_t>(w, O.ptab);
    int32_t* offsets = offsets_base + (size_t)e * (cap_peaks + 1);
    int32_t* hit_idx = hit_idx_base + (size_t)e * cap_pairs;
    hough_status_t* st = st_base + e;
    const int n = min(*at<int32_t>(w, O.misc), cap_peaks);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (bx == 0 && tid == 0) {
        const int64_t tot = n > 0 ? peak_voff[n - 1] + peaks[n - 1].votes : 0;
        offsets[n] = (int32_t)min(tot, (int64_t)INT32_MAX);
        st->n_pairs = tot;
        if (tot > cap_pairs) atomicOr(&st->flags, HOUGH_F_PAIR_OVERFLOW);
    }
    if (bx * THREADS >= n) return;  // uniform per block
    const int n_valid = g_cell_start[n_layers << cell_bits];
    const int h4 = (n_valid + 3) >> 2;          // 16-byte chunks of sorted hit indices
    const int stage_words = (2 * h4 + 3) & ~3;  // as 16-bit values
    int buf_words = min(kAssignBufMax, (lds_words - kHead - stage_words) / kWaves) & ~63;
    const bool staged = buf_words >= kAssignBufMin;
    if (!staged) buf_words = min(kAssignBufMax, (lds_words - kHead) / kWaves) & ~63;
    int32_t* lay_start = sm_i32;
    uint32_t* s16 = reinterpret_cast<uint32_t*>(sm_i32 + kHead);
    int32_t* buf = sm_i32 + kHead + (staged ? stage_words : 0) + wave * buf_words;
    const int stride = gridDim.x * THREADS;
    int base = bx * THREADS + wave * 64;
    // a two-deep pipeline over the wave's candidates: while a candidate copies its runs, the samples
    // of the next one and the row of the one after are in flight (a candidate then waits for its
    // table loads only, not for its samples first)
    // (n >= 1 here; the loads clamp to the last candidate and are issued without a condition, so
    // that no branch join makes the wave wait for them early)
    const int i1 = min(base + lane, n - 1), i2 = min(base + stride + lane, n - 1);
    hough_peak_t pk = peaks[i1], pk2 = peaks[i2];
    int64_t off = peak_voff[i1], off2 = peak_voff[i2];
    int32_t ev_n[kAssignLayerChunk];
    col_samples(Et + (size_t)(pk.l * n_qpt + pk.k) * et_stride, 0, ev_n);
    if (tid <= n_layers) lay_start[tid] = g_cell_start[tid << cell_bits];
    if (staged) {
        for (int c0 = tid; c0 < h4; c0 += kStageUnroll * THREADS) {
            uint4 v[kStageUnroll];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u)
                v[u] = reinterpret_cast<const uint4*>(sorted_h)[min(c0 + u * THREADS, h4 - 1)];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const int c = c0 + u * THREADS;
                if (c < h4)
                    reinterpret_cast<uint2*>(s16)[c] =
                        make_uint2((v[u].x & 0xFFFFu) | (v[u].y << 16), (v[u].z & 0xFFFFu) | (v[u].w << 16));
            }
        }
    }
    __syncthreads();
    for (; base < n; base += stride) {
        const int i = base + lane;
        const int last = min(n, base + 64) - 1;
        const int64_t o0 = __shfl(off, 0, 64);
        const int64_t o1 = __shfl(off, last - base, 64) + __shfl(pk.votes, last - base, 64);
        const hough_peak_t cur = pk;
        const int64_t cur_off = off;
        int32_t ev_c[kAssignLayerChunk];
#pragma unroll
        for (int u = 0; u < kAssignLayerChunk; ++u) ev_c[u] = ev_n[u];
        // the wave's next candidates: their samples, and the rows of the ones after
        pk = pk2;
        off = off2;
        col_samples(Et + (size_t)(pk.l * n_qpt + pk.k) * et_stride, 0, ev_n);
        const int i3 = min(base + 2 * stride + lane, n - 1);
        pk2 = peaks[i3];
        off2 = peak_voff[i3];
        if (i < n) {
            offsets[i] = (int32_t)min(cur_off, (int64_t)INT32_MAX);
            const int32_t* Ecol = Et + (size_t)(cur.l * n_qpt + cur.k) * et_stride;
            if (staged)
                assign_candidate_pt(cur, cur_off, o0, Ecol, ev_c, n_layers, M, F, n_phi, row, pt, lay_start,
                                    HitsU16{(lds_cu16*)s16}, buf, buf_words, hit_idx, cap_pairs);
            else
                assign_candidate_pt(cur, cur_off, o0, Ecol, ev_c, n_layers, M, F, n_phi, row, pt, lay_start,
                                    HitsIdx{sorted_h}, buf, buf_words, hit_idx, cap_pairs);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t fe = min(min(o1, o0 + buf_words), (int64_t)cap_pairs);
        for (int64_t wq = o0 + lane; wq < fe; wq += 64) hit_idx[wq] = buf[wq - o0];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ------------------------------------------------------------------ fit
// Track fit of each listed candidate (grid.y = event), one lane per candidate: the algebraic
// (Kasa) circle x^2 + y^2 + a x + b y + c = 0 through its hits in the least-squares sense.  The
// eight moments of the normal equations are summed over the candidate's hit list in list order
// (double), the 3x3 system is solved by Cramer's rule, and the
// row (xc, yc, R^2, n) = (-a/2, -b/2, xc^2 + yc^2 - c, n) is written; R^2 = -1 for fewer than 3 hits
// or a zero determinant, -2 for a list cut by the pair capacity.
// The moments of one list entry, added in the fixed order of a plain loop over the list.
struct FitSums {
    double sx = 0.0, sy = 0.0, sxx = 0.0, sxy = 0.0, syy = 0.0, sz = 0.0, sxz = 0.0, syz = 0.0;
    __device__ __forceinline__ void add(float xf, float yf) {
        const double X = (double)xf, Y = (double)yf;
        const double Z = X * X + Y * Y;
        sx += X;
        sy += Y;
        sxx += X * X;
        sxy += X * Y;
        syy += Y * Y;
        sz += Z;
        sxz += X * Z;
        syz += Y * Z;
    }
};

// Solve and store the row of a list [q0, q1) (cut when q1 > cap_pairs).
__device__ __forceinline__ void fit_store(double* o, int32_t q0, int32_t q1, int32_t cap_pairs, const FitSums& m) {
    const double N = (double)(q1 - q0);
    if (q1 > cap_pairs) {  // the list was cut: no fit
        o[0] = 0.0;
        o[1] = 0.0;
        o[2] = -2.0;
        o[3] = N;
        return;
    }
    const double sx = m.sx, sy = m.sy, sxx = m.sxx, sxy = m.sxy, syy = m.syy, sz = m.sz, sxz = m.sxz, syz = m.syz;
    // normal matrix [[sxx, sxy, sx], [sxy, syy, sy], [sx, sy, N]], right-hand side -(sxz, syz, sz)
    const double m_yy = syy * N - sy * sy;  // cofactors shared by the determinants
    const double m_xy = sxy * N - sy * sx;
    const double m_c = sxy * sy - syy * sx;
    const double det = sxx * m_yy - sxy * m_xy + sx * m_c;
    o[3] = N;
    if (N < 3.0 || det == 0.0) {
        o[0] = 0.0;
        o[1] = 0.0;
        o[2] = -1.0;
        return;
    }
    const double r0 = -sxz, r1 = -syz, r2 = -sz;
    const double a = (r0 * m_yy - sxy * (r1 * N - sy * r2) + sx * (r1 * sy - syy * r2)) / det;
    const double b = (sxx * (r1 * N - r2 * sy) - r0 * m_xy + sx * (sxy * r2 - r1 * sx)) / det;
    const double c = (sxx * (syy * r2 - sy * r1) - sxy * (sxy * r2 - r1 * sx) + r0 * m_c) / det;
    const double xc = -a / 2.0, yc = -b / 2.0;
    o[0] = xc;
    o[1] = yc;
    o[2] = xc * xc + yc * yc - c;
}

constexpr int kFitThreads = 256;
constexpr int kFitBuf = 1024;  // list entries staged per wave (coordinates, 8 KiB)

// A wave fits 64 consecutive candidates, whose lists are one contiguous stretch of the CSR list.
// The stretch is staged in pieces of kFitBuf entries: hit indices loaded coalesced, coordinates
// gathered (four per lane in flight) into the wave's LDS buffer; then every lane adds the entries of
// its own list that lie in the piece, in list order, so the sums are those of a plain loop over the
// list.
__global__ __launch_bounds__(kFitThreads) void k_fit(Events ev, const float* __restrict__ hx,
                                                    const float* __restrict__ hy,
                                                    const int32_t* __restrict__ offsets_base,
                                                    const int32_t* __restrict__ hit_idx_base, int32_t cap_peaks,
                                                    int32_t cap_pairs, const hough_status_t* __restrict__ st_base,
                                                    double* __restrict__ out_base) {
    __shared__ float2 stage[kFitThreads / 64][kFitBuf];
    const int e = blockIdx.y;
    const int n = min(st_base[e].n_peaks, cap_peaks);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pw = (blockIdx.x * (kFitThreads / 64) + wave) * 64;  // the wave's first candidate
    if (pw >= n) return;
    const int p = pw + lane;
    const bool valid = p < n;
    int h0, nh;
    event_hits(ev, e, h0, nh);
    const int32_t* offsets = offsets_base + (size_t)e * (cap_peaks + 1);
    const int32_t* hit_idx = hit_idx_base + (size_t)e * cap_pairs;
    const int32_t q0 = valid ? offsets[p] : 0, q1 = valid ? offsets[p + 1] : 0;
    const int32_t s0 = offsets[pw];
    const int32_t s1 = min(offsets[min(pw + 64, n)], cap_pairs);  // entries past the capacity were not written
    float2* buf = stage[wave];
    FitSums m;
    for (int ps = s0; ps < s1; ps += kFitBuf) {
        const int len = min(kFitBuf, s1 - ps);
        {  // all of a lane's indices, then all its gathers: two dependent memory steps per piece
            constexpr int kPer = kFitBuf / 64;
            int hh[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u)  // clamped, not skipped: a load under a branch waits on its own
                hh[u] = hit_idx[ps + min(lane + 64 * u, len - 1)];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const float xv = hx[h0 + hh[u]], yv = hy[h0 + hh[u]];
                if (lane + 64 * u < len) buf[lane + 64 * u] = make_float2(xv, yv);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int qa = max(q0, ps), qb = min(q1, ps + len);
        for (int q = qa; q < qb; q += 4) {  // four entries read at once, added in order
            float2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = buf[min(q + u, qb - 1) - ps];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (q + u < qb) m.add(v[u].x, v[u].y);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();  // every lane is done with the piece before it is overwritten
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (!valid) return;
    fit_store(out_base + ((size_t)e * cap_peaks + p) * 4, q0, q1, cap_pairs, m);
}

// Events of up to kFitResHits hits: the workgroup first copies all the event's coordinates into
// LDS, so the per-entry gathers are LDS reads (from global memory each lane's gather touched its own
// cache line, which bound the kernel above); the staged piece of the list holds hit indices only.
// Workgroups loop over the event's 64-candidate chunks.
constexpr int kFitResThreads = 1024;
constexpr int kFitResBuf = 512;  // list entries staged per wave
constexpr int kFitResIdxBytes = (kFitResThreads / 64) * kFitResBuf * 4;
constexpr int kFitResHits = (kLdsBytes - kFitResIdxBytes) / 8;

__global__ __launch_bounds__(kFitResThreads) void k_fit_res(Events ev, const float* __restrict__ hx,
                                                           const float* __restrict__ hy,
                                                           const int32_t* __restrict__ offsets_base,
                                                           const int32_t* __restrict__ hit_idx_base,
                                                           int32_t cap_peaks, int32_t cap_pairs,
                                                           const hough_status_t* __restrict__ st_base,
                                                           double* __restrict__ out_base, int32_t res_hits) {
    extern __shared__ float2 xy[];  // [res_hits] coordinates, then the waves' index pieces
    constexpr int kWaves = kFitResThreads / 64;
    const int e = blockIdx.y;
    const int n = min(st_base[e].n_peaks, cap_peaks);
    if (blockIdx.x * kWaves * 64 >= n) return;
    int h0, nh;
    event_hits(ev, e, h0, nh);
    if (nh > res_hits) return;  // (the launch sizes res_hits for every event it covers)
    // copy the coordinates with all of a thread's loads in flight at once (a plain strided loop
    // waits for each load before the next: a dozen round trips for a 12 000-hit event)
    constexpr int kCopy = 8;
    for (int i0 = threadIdx.x; i0 < nh; i0 += kCopy * kFitResThreads) {
        float xv[kCopy], yv[kCopy];
#pragma unroll
        for (int u = 0; u < kCopy; ++u) {
            const int i = min(i0 + u * kFitResThreads, nh - 1);
            xv[u] = hx[h0 + i];
            yv[u] = hy[h0 + i];
        }
#pragma unroll
        for (int u = 0; u < kCopy; ++u)
            if (i0 + u * kFitResThreads < nh) xy[i0 + u * kFitResThreads] = make_float2(xv[u], yv[u]);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t* ib = reinterpret_cast<int32_t*>(xy + res_hits) + wave * kFitResBuf;
    const int32_t* offsets = offsets_base + (size_t)e * (cap_peaks + 1);
    const int32_t* hit_idx = hit_idx_base + (size_t)e * cap_pairs;
    for (int chunk = blockIdx.x * kWaves + wave; chunk * 64 < n; chunk += gridDim.x * kWaves) {
        const int pw = chunk * 64, p = pw + lane;
        const bool valid = p < n;
        const int32_t q0 = valid ? offsets[p] : 0, q1 = valid ? offsets[p + 1] : 0;
        const int32_t s0 = offsets[pw];
        const int32_t s1 = min(offsets[min(pw + 64, n)], cap_pairs);
        FitSums m;
        for (int ps = s0; ps < s1; ps += kFitResBuf) {
            const int len = min(kFitResBuf, s1 - ps);
            constexpr int kPer = kFitResBuf / 64;
            int hh[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u)  // clamped, not skipped: a load under a branch waits on its own
                hh[u] = hit_idx[ps + min(lane + 64 * u, len - 1)];
#pragma unroll
            for (int u = 0; u < kPer; ++u)
                if (lane + 64 * u < len) ib[lane + 64 * u] = hh[u];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int qa = max(q0, ps) - ps, qb = min(q1, ps + len) - ps;
#pragma unroll 1
            for (int q = qa; q < qb; ++q) {
                const float2 v = xy[ib[q]];
                m.add(v.x, v.y);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();  // every lane is done with the piece before it is overwritten
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (valid) fit_store(out_base + ((size_t)e * cap_peaks + p) * 4, q0, q1, cap_pairs, m);
    }
}

// ------------------------------------------------------------------ per-hit radius vote
// The transform with each hit's own radius (a detector smeared in x and y): R = floor(sqrt(X^2 +
// Y^2)) in Q16.16, the sample's A in IEEE double as for the table, its arcsine in integers (A as
// Q2.30, b = floor(sqrt(2^60 - a^2)), the CORDIC angle of (b, a) as a signed 32-bit binary angle,
// rounded half up to M bits).  One thread per (hit, kCrCols columns); every sample is computed on
// the fly (ALU-bound: a 30-step CORDIC per sample) and voted with a global atomic.
constexpr int kCrThreads = 256;
constexpr int kCrCols = 16;

// floor(sqrt(v)) for v < 2^63: a double estimate corrected to the exact integer (at most a step or
// two: the estimate is within one of the root)
__device__ __forceinline__ uint64_t isqrt_u64(uint64_t v) {
    uint64_t s = (uint64_t)sqrt((double)v);
    while (s * s > v) --s;
    while ((s + 1) * (s + 1) <= v) ++s;
    return s;
}

struct CrGrid {
    int32_t n_layers, n_qpt, n_cols, n_phi, M, F;
    double qpt_min, qstep, d0_min, dstep, kappa;
};

__global__ __launch_bounds__(256) void k_cr_init(int32_t* __restrict__ acc, int64_t n_bins, int32_t n_hits,
                                                hough_status_t* __restrict__ st) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n_bins / 4) reinterpret_cast<int4*>(acc)[i] = make_int4(0, 0, 0, 0);
    if (i == 0) {
        for (int64_t j = n_bins / 4 * 4; j < n_bins; ++j) acc[j] = 0;
        st->n_hits = n_hits;
        st->n_bad_hits = 0;
        st->n_votes = 0;
        st->n_peaks = 0;
        st->flags = 0;
        st->n_pairs = 0;
    }
}

__global__ __launch_bounds__(kCrThreads) void k_vote_cr(const float* __restrict__ hx, const float* __restrict__ hy,
                                                        const uint8_t* __restrict__ hl, int32_t n, CrGrid g,
                                                        CordicTable T, int32_t* __restrict__ acc,
                                                        hough_status_t* __restrict__ st) {
    const int chunks = (g.n_cols + kCrCols - 1) / kCrCols;
    const int64_t t = (int64_t)blockIdx.x * kCrThreads + threadIdx.x;
    const int h = (int)(t / chunks), ch = (int)(t % chunks);
    uint32_t votes = 0, bad = 0;
    if (h < n) {
        const float x = hx[h], y = hy[h];
        const uint8_t L = hl[h];
        bool ok = (int)L < g.n_layers && isfinite(x) && isfinite(y) && fabsf(x) < 32768.0f && fabsf(y) < 32768.0f;
        int32_t X = 0, Y = 0;
        if (ok) {
            X = __float2int_rn(x * 65536.0f);  // exact scaling, round half to even
            Y = __float2int_rn(y * 65536.0f);
            ok = !(X == 0 && Y == 0);
        }
        if (!ok) {
            bad = ch == 0 ? 1u : 0u;
        } else {
            const int s = 32 - g.M;
            const uint32_t maskM = g.M >= 32 ? 0xFFFFFFFFu : ((1u << g.M) - 1u);
            const uint32_t phiM = cordic_azimuth(X, Y, T) >> s;
            const uint64_t R2 = (uint64_t)((int64_t)X * X) + (uint64_t)((int64_t)Y * Y);
            const double r = (double)isqrt_u64(R2) / 65536.0;
            const int c0 = ch * kCrCols;
            const int c1 = min(g.n_cols, c0 + kCrCols);
            for (int col = c0; col < c1; ++col) {
                const int l = col / g.n_qpt, k = col % g.n_qpt;
                const double q = g.qpt_min + ((double)k + 0.5) * g.qstep;
                const double c = -g.kappa * q;
                const double d = g.d0_min + ((double)l + 0.5) * g.dstep;
                const double num = c * (r * r + d * d) + 2.0 * d;
                const double den = 2.0 * r * (1.0 + c * d);
                if (!(den > 0.0)) continue;
                const double A = num / den;
                if (!(fabs(A) <= 1.0)) continue;
                const int64_t a = llrint(A * 1073741824.0);
                const int64_t b = (int64_t)isqrt_u64((uint64_t)(((int64_t)1 << 60) - a * a));
                const int64_t th = (int64_t)(int32_t)cordic_azimuth((int32_t)b, (int32_t)a, T);
                const int32_t E = (int32_t)((th + ((int64_t)1 << (s - 1))) >> s);
                const uint32_t bin = ((phiM - (uint32_t)E) & maskM) >> g.F;
                atomicAdd(acc + (size_t)col * g.n_phi + bin, 1);
                ++votes;
            }
        }
    }
    // one atomic per wave for each count
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        votes += __shfl_xor(votes, o, 64);
        bad += __shfl_xor(bad, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (votes) atomicAdd(reinterpret_cast<unsigned long long*>(&st->n_votes), (unsigned long long)votes);
        if (bad) atomicAdd(&st->n_bad_hits, (int)bad);
    }
}

// Background suppression inside each candidate's bin (refinement).  Per listed candidate (one
// thread): the angle inside the bin of each listed hit, rel = ((PhiM - E) mod 2^M) - b * 2^F with
// the sample of its layer at the candidate's (l, k); among the windows [c, c + w) that begin at a
// listed hit's rel, the one holding hits of the most distinct layers, then the most hits, then the
// lowest c; per layer present in it, the hit nearest the centre (smallest |2 rel - 2c - w|, ties by
// the lower hit index).  Lists of up to kRefineStage hits keep (rel, layer) in LDS (16 bits each,
// entry-major so that a wave's threads hit distinct banks); longer lists recompute them from the
// workspace.  out_layers = -1 for a list cut by the pair capacity.
constexpr int kRefineThreads = 256;
constexpr int kRefineStage = 64;

__global__ __launch_bounds__(kRefineThreads) void k_refine(
    const hough_peak_t* __restrict__ peaks, int32_t cap_peaks, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ hit_idx, int32_t cap_pairs, const char* __restrict__ ws, WsOff O,
    const hough_status_t* __restrict__ st, const int32_t* __restrict__ E, int n_layers, int n_cols, int n_qpt,
    int M, int F, int32_t w, int32_t* __restrict__ out_hits, int32_t* __restrict__ out_layers) {
    __shared__ uint16_t s_rl[kRefineStage * kRefineThreads];
    const int n = min(st->n_peaks, cap_peaks);
    const int p = blockIdx.x * kRefineThreads + threadIdx.x;
    if (p >= n) return;
    const hough_peak_t pk = peaks[p];
    const int32_t q0 = offsets[p], q1 = offsets[p + 1];
    int32_t* oh = out_hits + (size_t)p * n_layers;
    for (int L = 0; L < n_layers; ++L) oh[L] = -1;
    if (q1 > cap_pairs) {
        out_layers[p] = -1;
        return;
    }
    const int m = q1 - q0;
    const uint32_t* phi32 = at<const uint32_t>(const_cast<char*>(ws), O.phi32);
    const uint8_t* lay = at<const uint8_t>(const_cast<char*>(ws), O.lay);
    const int32_t* Ec = E + (size_t)pk.l * n_qpt + pk.k;
    const uint32_t mask = M >= 32 ? 0xFFFFFFFFu : ((1u << M) - 1u);
    const uint32_t bW = (uint32_t)pk.b << F;
    auto rel_of = [&](int j, int& L) -> int32_t {
        const int32_t h = hit_idx[q0 + j];
        L = lay[h];
        return (int32_t)(((phi32[h] >> (32 - M)) - (uint32_t)Ec[(size_t)L * n_cols]) & mask) - (int32_t)bW;
    };
    const bool staged = m <= kRefineStage;
    if (staged) {
        for (int j = 0; j < m; ++j) {
            int L;
            const int32_t r = rel_of(j, L);
            s_rl[j * kRefineThreads + threadIdx.x] = (uint16_t)((r << 5) | L);  // r < 2^F <= 256, L < 32
        }
    }
    auto get = [&](int j, int32_t& r, int& L) {
        if (staged) {
            const uint32_t v = s_rl[j * kRefineThreads + threadIdx.x];
            r = (int32_t)(v >> 5);
            L = (int)(v & 31u);
        } else {
            r = rel_of(j, L);
        }
    };
    int best_l = -1, best_n = -1;
    int32_t best_c = 0;
    for (int i = 0; i < m; ++i) {
        int32_t c0;
        int Li;
        get(i, c0, Li);
        uint32_t lm = 0;
        int cnt = 0;
        for (int j = 0; j < m; ++j) {
            int32_t r;
            int L;
            get(j, r, L);
            if (r >= c0 && r < c0 + w) {
                lm |= 1u << L;
                ++cnt;
            }
        }
        const int nl = __popc(lm);
        if (nl > best_l || (nl == best_l && cnt > best_n) || (nl == best_l && cnt == best_n && c0 < best_c)) {
            best_l = nl;
            best_n = cnt;
            best_c = c0;
        }
    }
    out_layers[p] = m > 0 ? best_l : 0;
    if (m == 0) return;
    for (int L = 0; L < n_layers; ++L) {
        int32_t pick = -1, pick_d = 0;
        for (int j = 0; j < m; ++j) {
            int32_t r;
            int Lj;
            get(j, r, Lj);
            if (Lj != L || !(r >= best_c && r < best_c + w)) continue;
            const int32_t h = hit_idx[q0 + j];
            const int32_t d = abs(2 * r - 2 * best_c - w);
            if (pick < 0 || d < pick_d || (d == pick_d && h < pick)) {
                pick = h;
                pick_d = d;
            }
        }
        oh[L] = pick;
    }
}

// Assignment under the per-hit radius: the lists of the candidates found in a per-hit-radius
// accumulator (hough_vote_cr, then hough_peaks on it).  Each hit's bin in a column follows its own
// radius, so the lists are collected by voting again: k_cra_init clears the bin -> candidate map
// and the per-candidate fill counters, k_cra_map marks every listed candidate's bin, k_cra_vote
// repeats the vote (same integer arithmetic as k_vote_cr) and appends, for a vote into a
// candidate's bin, the key (layer << 32) | (angle inside the bin << 24) | hit at the candidate's
// CSR offset plus an atomic slot, and k_cra_sort sorts each list's keys (the list order of the
// assignment: layer, angle inside the bin, hit index) and writes the hit indices.  A list that
// starts before the pair capacity is collected whole (its keys may run up to max_hits past it) so
// that its first entries are the right ones.
__global__ __launch_bounds__(256) void k_cra_init(int32_t* __restrict__ map, int64_t n_bins,
                                                 int32_t* __restrict__ fill, int32_t cap_peaks) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n_bins) map[i] = -1;
    if (i < cap_peaks) fill[i] = 0;
}

__global__ __launch_bounds__(256) void k_cra_map(const hough_peak_t* __restrict__ peaks, int32_t cap_peaks,
                                                const char* __restrict__ ws, WsOff O, int n_qpt, int n_phi,
                                                int32_t* __restrict__ map) {
    const int n = min(*at<const int32_t>(const_cast<char*>(ws), O.misc), cap_peaks);
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const hough_peak_t pk = peaks[p];
    map[((int64_t)pk.l * n_qpt + pk.k) * n_phi + pk.b] = p;
}

__global__ __launch_bounds__(kCrThreads) void k_cra_vote(const float* __restrict__ hx, const float* __restrict__ hy,
                                                        const uint8_t* __restrict__ hl, int32_t n, CrGrid g,
                                                        CordicTable T, const int32_t* __restrict__ map,
                                                        const int64_t* __restrict__ peak_voff,
                                                        int32_t* __restrict__ fill, uint64_t* __restrict__ keys,
                                                        int32_t cap_pairs) {
    const int chunks = (g.n_cols + kCrCols - 1) / kCrCols;
    const int64_t t = (int64_t)blockIdx.x * kCrThreads + threadIdx.x;
    const int h = (int)(t / chunks), ch = (int)(t % chunks);
    if (h >= n) return;
    const float x = hx[h], y = hy[h];
    const uint8_t L = hl[h];
    bool ok = (int)L < g.n_layers && isfinite(x) && isfinite(y) && fabsf(x) < 32768.0f && fabsf(y) < 32768.0f;
    int32_t X = 0, Y = 0;
    if (ok) {
        X = __float2int_rn(x * 65536.0f);
        Y = __float2int_rn(y * 65536.0f);
        ok = !(X == 0 && Y == 0);
    }
    if (!ok) return;
    const int s = 32 - g.M;
    const uint32_t maskM = g.M >= 32 ? 0xFFFFFFFFu : ((1u << g.M) - 1u);
    const uint32_t wmask = (1u << g.F) - 1u;
    const uint32_t phiM = cordic_azimuth(X, Y, T) >> s;
    const uint64_t R2 = (uint64_t)((int64_t)X * X) + (uint64_t)((int64_t)Y * Y);
    const double r = (double)isqrt_u64(R2) / 65536.0;
    const int c0 = ch * kCrCols;
    const int c1 = min(g.n_cols, c0 + kCrCols);
    for (int col = c0; col < c1; ++col) {
        const int l = col / g.n_qpt, k = col % g.n_qpt;
        const double q = g.qpt_min + ((double)k + 0.5) * g.qstep;
        const double c = -g.kappa * q;
        const double d = g.d0_min + ((double)l + 0.5) * g.dstep;
        const double num = c * (r * r + d * d) + 2.0 * d;
        const double den = 2.0 * r * (1.0 + c * d);
        if (!(den > 0.0)) continue;
        const double A = num / den;
        if (!(fabs(A) <= 1.0)) continue;
        const int64_t a = llrint(A * 1073741824.0);
        const int64_t b = (int64_t)isqrt_u64((uint64_t)(((int64_t)1 << 60) - a * a));
        const int64_t th = (int64_t)(int32_t)cordic_azimuth((int32_t)b, (int32_t)a, T);
        const int32_t E = (int32_t)((th + ((int64_t)1 << (s - 1))) >> s);
        const uint32_t rel = (phiM - (uint32_t)E) & maskM;
        const int32_t p = map[(size_t)col * g.n_phi + (rel >> g.F)];
        if (p < 0) continue;
        const int64_t base = peak_voff[p];
        if (base >= cap_pairs) continue;  // the list lies wholly past the capacity
        const int slot = atomicAdd(fill + p, 1);
        keys[base + slot] = ((uint64_t)L << 32) | ((uint64_t)(rel & wmask) << 24) | (uint64_t)h;
    }
}

__global__ __launch_bounds__(256) void k_cra_sort(const hough_peak_t* __restrict__ peaks, int32_t cap_peaks,
                                                 const char* __restrict__ ws, WsOff O, uint64_t* __restrict__ keys,
                                                 int32_t* __restrict__ offsets, int32_t* __restrict__ hit_idx,
                                                 int32_t cap_pairs, hough_status_t* __restrict__ st) {
    const int n = min(*at<const int32_t>(const_cast<char*>(ws), O.misc), cap_peaks);
    const int64_t* peak_voff = at<const int64_t>(const_cast<char*>(ws), O.peak_voff);
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p == 0) {
        const int64_t tot = n > 0 ? peak_voff[n - 1] + peaks[n - 1].votes : 0;
        offsets[n] = (int32_t)min(tot, (int64_t)INT32_MAX);
        st->n_pairs = tot;
        if (tot > cap_pairs) atomicOr(&st->flags, HOUGH_F_PAIR_OVERFLOW);
    }
    if (p >= n) return;
    const int64_t base = peak_voff[p];
    offsets[p] = (int32_t)min(base, (int64_t)INT32_MAX);
    if (base >= cap_pairs) return;
    const int nv = peaks[p].votes;
    uint64_t* kk = keys + base;
    for (int i = 1; i < nv; ++i) {  // insertion sort of the list's keys (a few to a few hundred)
        const uint64_t v = kk[i];
        int j = i - 1;
        while (j >= 0 && kk[j] > v) {
            kk[j + 1] = kk[j];
            --j;
        }
        kk[j + 1] = v;
    }
    const int m = (int)min((int64_t)nv, (int64_t)cap_pairs - base);
    for (int i = 0; i < m; ++i) hit_idx[base + i] = (int32_t)(kk[i] & 0xFFFFFFu);
}

// ------------------------------------------------------------------ zvote
// Per candidate p (grid.y = event): every hit h of its list with a usable z votes, for each
// cot(theta) row m, into z0 bin j(m) = (Z_h * 2^16 - S_h * C_m - z0min) >> shift, where S_h is the
// arc length from the origin to the hit's layer for the candidate's (d0, q/pT) centre; the output
// is the (m, j) with the most votes, lowest m * n_z0 + j on ties.  With A_h = Z_h * 2^16 - z0min -
// S_h * C_0 and B_h = S_h * dC, the value for row m is A_h - m * B_h (exact int64).
//
// A wave takes groups of kZvoteGroup consecutive candidates.  It first stages (Z_h, S_h) of all
// hits of the group in its LDS (one pass of independent loads for the whole group: hit index,
// then z and layer, then the arc length; A_h and B_h are formed when a lane fetches its hit), then
// votes the candidates one by one: with H <= 64 hits, R = min(kZvoteSlots, 64 / H) rows at once,
// one lane per (row slot, hit).  The row slots lie n_z0 + 1 words apart, so the same bin of
// different slots falls into different LDS banks.
//
// Each LDS word of a row histogram holds (count << 16) | (0xFFFF - j).  Adding 1 << 16 returns the
// old word, so old + 2^16 - m * n_z0 = (count << 16) | (0xFFFF - (m * n_z0 + j)) is a key whose
// maximum over all votes is the argmax with the lowest linear index (a bin's last vote returns its
// final count; counts < 2^16 and n_cot * n_z0 <= 2^16 are plan limits).  The voter then writes
// the word back to (0xFFFF - j): the atomics of one instruction complete before the next LDS
// instruction of the wave, so the row is clean for the next row voted in that slot.  A group
// holding a candidate of more than 64 hits is voted from memory instead, one row at a time in
// chunks of 64 hits, restoring the row after its last chunk.
constexpr int kZvoteGroup = 4;                    // candidates staged together by a wave
constexpr int kZvoteUnroll = 8;                   // rows voted before their returned words are used
constexpr int kZvoteStage = kZvoteGroup * 64;     // staged hits per wave (Z, S: 8 bytes each)

// Q16.16 z and arc length of a listed hit; S = -1 when the hit has no usable z or arc length
__device__ __forceinline__ int2 zvote_zs(int32_t h, const float* __restrict__ hz, const uint8_t* __restrict__ hl,
                                         int h0, const int32_t* __restrict__ Sc, int n_layers, size_t s_layer) {
    const float zf = hz[h0 + h];
    const int L = hl[h0 + h];
    bool ok = isfinite(zf) && fabsf(zf) < 32768.0f && L < n_layers;
    int32_t S = ok ? Sc[(size_t)L * s_layer] : -1;
    ok = ok && S >= 0;
    return make_int2(ok ? __float2int_rn(zf * 65536.0f) : 0, ok ? S : -1);
}

// an unusable hit gets A = -1, B = 0: its value is negative on every row and never votes
__device__ __forceinline__ void zvote_ab(int2 zs, const ZGrid& zg, int64_t& A, int64_t& B) {
    const bool ok = zs.y >= 0;
    A = ok ? (int64_t)zs.x * 65536 - zg.z0min - (int64_t)zs.y * zg.c0 : -1;
    B = ok ? (int64_t)zs.y * zg.dc : 0;
}

__device__ __forceinline__ void zvote_hit(int32_t h, const float* __restrict__ hz, const uint8_t* __restrict__ hl,
                                          int h0, const int32_t* __restrict__ Sc, int n_layers, size_t s_layer,
                                          const ZGrid& zg, int64_t& A, int64_t& B) {
    zvote_ab(zvote_zs(h, hz, hl, h0, Sc, n_layers, s_layer), zg, A, B);
}

// floor(65536 / H) + 1 for H = 1..64: slot = (lane * kInvH[H]) >> 16 equals lane / H for lane < 64.
struct InvTable {
    uint32_t v[65];
};
constexpr InvTable make_inv_table() {
    InvTable t{};
    for (int h = 1; h <= 64; ++h) t.v[h] = 65536u / (uint32_t)h + 1u;
    return t;
}
__constant__ InvTable kInvH = make_inv_table();

// Votes of one candidate of H (1..64) hits whose (A, B) the lane fetches with get(i), i < H.
// Lane = (row slot, hit); rows m = slot, slot + R, ...  For a z0 bin width 2^s with 28 <= s <= 32
// (FAST) the bin index j and the remainder below it (left-aligned in 32 bits) step by constant
// amounts from row to row: j - bH - borrow, an exact 64-bit subtraction done in two 32-bit halves.
// Otherwise the 64-bit value is stepped and shifted.  The vote's word is restored with an atomic
// subtract of the same amount (the adds of one instruction all precede it).
template <bool FAST, typename Get>
__device__ __forceinline__ uint32_t zvote_small(int H, int lane, uint32_t* region, const ZGrid& zg, Get get) {
    const int nz = zg.n_z0;
    const int R = min(kZvoteSlots, 64 / H);
    const int slot = (int)(((uint32_t)lane * kInvH.v[H]) >> 16);
    int64_t A = -1, B = 0;
    if (slot < R) get(lane - slot * H, A, B);
    uint32_t* row = region + slot * (nz + 1);
    const int64_t z0 = A - (int64_t)slot * B;
    const int64_t step = (int64_t)R * B;
    uint32_t kc = 0x10000u - (uint32_t)(slot * nz);
    const uint32_t kstep = (uint32_t)(R * nz);
    const int iters = (zg.n_cot + R - 1) / R;
    const uint32_t unit = 0x10000u;
    uint32_t best = 0;
    if (FAST) {
        const int sh = zg.shift;
        const uint64_t lowmask = (sh == 64) ? ~0ull : ((1ull << sh) - 1);
        int32_t j = (int32_t)(z0 >> sh);
        uint32_t low = (uint32_t)(((uint64_t)z0 & lowmask) << (32 - sh));
        const int32_t bH = (int32_t)(step >> sh);
        const uint32_t bL = (uint32_t)(((uint64_t)step & lowmask) << (32 - sh));
        // every row of all but the last iteration exists (m < n_cot); the last one is checked.
        // kZvoteUnroll rows are voted before their returned words are used: the add and restore
        // of one row precede those of the next in the wave's LDS order, so nothing waits per row.
        int it = 0;
        for (; it + kZvoteUnroll < iters; it += kZvoteUnroll) {
            uint32_t got[kZvoteUnroll];
            bool ok[kZvoteUnroll];
            uint32_t kcs[kZvoteUnroll];
#pragma unroll
            for (int u = 0; u < kZvoteUnroll; ++u) {
                ok[u] = (uint32_t)j < (uint32_t)nz;
                kcs[u] = kc;
                got[u] = 0;
                if (ok[u]) {
                    got[u] = __hip_atomic_fetch_add(row + j, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_sub(row + j, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                asm volatile("" ::: "memory");
                const uint32_t nl = low - bL;
                j = j - bH - (nl > low ? 1 : 0);
                low = nl;
                kc -= kstep;
            }
#pragma unroll
            for (int u = 0; u < kZvoteUnroll; ++u) best = max(best, ok[u] ? got[u] + kcs[u] : 0u);
        }
        for (; it + 1 < iters; ++it) {
            if ((uint32_t)j < (uint32_t)nz) {
                const uint32_t old = __hip_atomic_fetch_add(row + j, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                best = max(best, old + kc);
                __hip_atomic_fetch_sub(row + j, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            asm volatile("" ::: "memory");
            const uint32_t nl = low - bL;
            j = j - bH - (nl > low ? 1 : 0);
            low = nl;
            kc -= kstep;
        }
        if (slot + (iters - 1) * R < zg.n_cot && (uint32_t)j < (uint32_t)nz) {
            const uint32_t old = __hip_atomic_fetch_add(row + j, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            best = max(best, old + kc);
            __hip_atomic_fetch_sub(row + j, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        asm volatile("" ::: "memory");
    } else {
        int64_t z = z0;
        int m = slot;
        for (int it = 0; it < iters; ++it) {
            if (m < zg.n_cot && (uint64_t)z < zg.lim) {
                const uint32_t j = (uint32_t)((uint64_t)z >> zg.shift);
                const uint32_t old = __hip_atomic_fetch_add(row + j, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                best = max(best, old + kc);
                __hip_atomic_fetch_sub(row + j, unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            asm volatile("" ::: "memory");
            z -= step;
            m += R;
            kc -= kstep;
        }
    }
    return best;
}

__device__ __forceinline__ void zvote_write(int32_t* o, uint32_t best, int nz) {
    if (best == 0) {
        o[0] = -1;
        o[1] = -1;
        o[2] = 0;
    } else {
        const uint32_t lin = 0xFFFFu - (best & 0xFFFFu);
        o[0] = (int32_t)(lin / (uint32_t)nz);
        o[1] = (int32_t)(lin % (uint32_t)nz);
        o[2] = (int32_t)(best >> 16);
    }
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, 64));
    return v;
}

__global__ __launch_bounds__(kZvoteThreads) void k_zvote(
    Events ev, const float* __restrict__ hz, const uint8_t* __restrict__ hl, int n_layers,
    const hough_peak_t* __restrict__ peaks_base, int32_t cap_peaks, const int32_t* __restrict__ offsets_base,
    const int32_t* __restrict__ hit_idx_base, int32_t cap_pairs, const hough_status_t* __restrict__ st_base,
    const int32_t* __restrict__ S, int n_d0, int n_qpt, ZGrid zg, int32_t* __restrict__ out_base) {
    // LDS per wave: kZvoteSlots row histograms of n_z0 words (n_z0 + 1 apart), then kZvoteStage
    // staged (Z, S)
    extern __shared__ uint32_t zs_u32[];
    const int e = blockIdx.y;
    int h0, nh;
    event_hits(ev, e, h0, nh);
    const hough_peak_t* peaks = peaks_base + (size_t)e * cap_peaks;
    const int32_t* offsets = offsets_base + (size_t)e * ((size_t)cap_peaks + 1);
    const int32_t* hit_idx = hit_idx_base + (size_t)e * cap_pairs;
    int32_t* out = out_base + (size_t)e * 3 * cap_peaks;
    const int n = min(st_base[e].n_peaks, cap_peaks);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nz = zg.n_z0;
    const size_t s_layer = (size_t)n_d0 * n_qpt;
    const size_t slots_words = ((size_t)kZvoteSlots * (nz + 1) + 1) & ~(size_t)1;  // keeps the stage 8-byte aligned
    const size_t wave_words = slots_words + 2 * kZvoteStage;
    uint32_t* region = zs_u32 + (size_t)wave * wave_words;
    int2* stage = reinterpret_cast<int2*>(region + slots_words);  // [kZvoteStage] (Z, S)
    for (int i = lane; i < kZvoteSlots * (nz + 1); i += 64) region[i] = 0xFFFFu - (uint32_t)(i % (nz + 1));
    const int waves = kZvoteThreads / 64;
    const int n_groups = (n + kZvoteGroup - 1) / kZvoteGroup;
    const bool fast = zg.shift >= 28 && zg.shift <= 32;
    for (int grp = blockIdx.x * waves + wave; grp < n_groups; grp += gridDim.x * waves) {
        const int p0 = grp * kZvoteGroup;
        const int cnt = min(kZvoteGroup, n - p0);
        // lane c < cnt: candidate p0 + c (its list start, (l, k)); lane cnt: the end of the last list
        const int32_t my_off = lane <= cnt ? offsets[p0 + lane] : 0;
        const int32_t my_l = lane < cnt ? peaks[p0 + lane].l : 0;
        const int32_t my_k = lane < cnt ? peaks[p0 + lane].k : 0;
        const int32_t q0 = __builtin_amdgcn_readlane(my_off, 0);
        int32_t qe = __builtin_amdgcn_readlane(my_off, cnt);
        bool small = true;
        for (int c = 0; c < cnt; ++c) {
            const int32_t a = __builtin_amdgcn_readlane(my_off, c), b = __builtin_amdgcn_readlane(my_off, c + 1);
            small = small && b - a <= 64;
        }
        qe = min(qe, cap_pairs);
        if (small) {
            // stage (A, B) of every listed hit of the group: pair q -> candidate = number of list
            // starts <= q, minus one
#pragma unroll
            for (int i = 0; i < kZvoteStage / 64; ++i) {
                const int32_t q = q0 + i * 64 + lane;
                int c = 0;
                for (int j = 1; j < cnt; ++j) c += q >= __builtin_amdgcn_readlane(my_off, j) ? 1 : 0;
                // with every lane active: a lane shuffle reads nothing from inactive lanes
                const int32_t l = __shfl(my_l, c, 64), k = __shfl(my_k, c, 64);
                if (q < qe) stage[q - q0] = zvote_zs(hit_idx[q], hz, hl, h0, S + (size_t)l * n_qpt + k, n_layers, s_layer);
            }
            asm volatile("" ::: "memory");
            for (int c = 0; c < cnt; ++c) {
                const int32_t o0 = __builtin_amdgcn_readlane(my_off, c);
                const int32_t o1 = __builtin_amdgcn_readlane(my_off, c + 1);
                int32_t* o = out + 3 * (size_t)(p0 + c);
                if (o1 > cap_pairs) {  // hit list cut by the pair capacity: no result
                    if (lane == 0) {
                        o[0] = -1;
                        o[1] = -1;
                        o[2] = -1;
                    }
                    continue;
                }
                const int H = o1 - o0;
                uint32_t best = 0;
                if (H >= 1) {
                    const int2* st_c = stage + (o0 - q0);
                    auto get = [&](int i, int64_t& A, int64_t& B) { zvote_ab(st_c[i], zg, A, B); };
                    best = fast ? zvote_small<true>(H, lane, region, zg, get) : zvote_small<false>(H, lane, region, zg, get);
                }
                best = wave_max(best);
                if (lane == 0) zvote_write(o, best, nz);
            }
            asm volatile("" ::: "memory");
        } else {
            for (int c = 0; c < cnt; ++c) {
                const int32_t o0 = __builtin_amdgcn_readlane(my_off, c);
                const int32_t o1 = __builtin_amdgcn_readlane(my_off, c + 1);
                const int32_t pl = __builtin_amdgcn_readlane(my_l, c), pk = __builtin_amdgcn_readlane(my_k, c);
                int32_t* o = out + 3 * (size_t)(p0 + c);
                if (o1 > cap_pairs) {
                    if (lane == 0) {
                        o[0] = -1;
                        o[1] = -1;
                        o[2] = -1;
                    }
                    continue;
                }
                const int H = o1 - o0;
                const int32_t* Sc = S + (size_t)pl * n_qpt + pk;
                uint32_t best = 0;
                if (H >= 1 && H <= 64) {
                    auto get = [&](int i, int64_t& A, int64_t& B) {
                        zvote_hit(hit_idx[o0 + i], hz, hl, h0, Sc, n_layers, s_layer, zg, A, B);
                    };
                    best = fast ? zvote_small<true>(H, lane, region, zg, get) : zvote_small<false>(H, lane, region, zg, get);
                } else if (H > 64) {
                    for (int m = 0; m < zg.n_cot; ++m) {
                        const uint32_t kc = 0x10000u - (uint32_t)(m * nz);
                        for (int c0 = 0; c0 < H; c0 += 64) {
                            int64_t A = -1, B = 0;
                            if (c0 + lane < H) zvote_hit(hit_idx[o0 + c0 + lane], hz, hl, h0, Sc, n_layers, s_layer, zg, A, B);
                            const int64_t z0 = A - (int64_t)m * B;
                            if ((uint64_t)z0 < zg.lim) {
                                const uint32_t j = (uint32_t)((uint64_t)z0 >> zg.shift);
                                const uint32_t old = __hip_atomic_fetch_add(region + j, 0x10000u, __ATOMIC_RELAXED,
                                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
                                best = max(best, old + kc);
                            }
                            asm volatile("" ::: "memory");
                        }
                        for (int j = lane; j < nz; j += 64) region[j] = 0xFFFFu - (uint32_t)j;
                        asm volatile("" ::: "memory");
                    }
                }
                best = wave_max(best);
                if (lane == 0) zvote_write(o, best, nz);
            }
        }
    }
}

// ------------------------------------------------------------------ host helpers
int ilog2_exact(int v) {
    if (v <= 0 || (v & (v - 1))) return -1;
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

int launch_status() { return hipGetLastError() == hipSuccess ? HOUGH_OK : HOUGH_E_HIP; }

// Largest event (hits) the bucketing workgroup sorts in LDS: resident in one pass and with its
// angles and keys beside the cell cursors in the LDS (0: none).
int bucket_cap_hits(const hough_plan* p) {
    const int cpl_pad = ((1 << p->cell_bits) + 3) & ~3;
    const long room = ((long)kLdsBytes - 4L * cpl_pad - 1024) / 8 - 8;  // static LDS aside, 8 entries of slack
    long cap = room < (long)kScanThreads * kBucketUnroll ? room : (long)kScanThreads * kBucketUnroll;
    cap = cap < p->g.max_hits_per_event ? cap : p->g.max_hits_per_event;
    return cap >= 64 ? (int)cap : 0;
}

// phi0 rows per k_prep_fine workgroup: the tuned value (a power of two), else kFineRows; at most n_phi
int fine_rows(const hough_plan* p) {
    int R = p->tuning.prep_rows > 0 ? p->tuning.prep_rows : kFineRows;
    const int past = (p->pt_row > p->pt_row8 ? p->pt_row : p->pt_row8) - p->g.n_phi;
    while (R < past) R *= 2;  // chunk 0 writes the window counts past the turn from its rows
    return p->g.n_phi < R ? p->g.n_phi : R;
}

// Dynamic LDS of k_prep_fine: R + 1 padded rows of 16-bit counter pairs and the tied-hit list.
size_t fine_lds_bytes(const hough_plan* p) {
    const size_t R = (size_t)fine_rows(p);
    return 4 * ((R + 1) * (((size_t)1 << p->F) / 2 + 1) + kFineTieCap);
}

// Launchers shared by the single-event and batched entry points.
// The 8-bit window counts serve batches (where the vote's table reads bound it); a single event's
// vote waits on latency instead, and writing the second table would only lengthen its prep.  The
// prep and the vote of one chain see the same event count, so they agree on the table.
int pt_row8_for(const hough_plan* p, int n_events) { return n_events > 1 ? p->pt_row8 : 0; }

void launch_prep(const hough_plan* p, const Events& ev, int n_events, int max_n, const float* x, const float* y,
                 const uint8_t* layer, uint32_t* phi_out, char* ws, const WsOff& O, hough_status_t* st,
                 hipStream_t stream) {
    if (max_n > 0)
        hipLaunchKernelGGL(k_prep_hits, dim3((max_n + 255) / 256, n_events), dim3(256), 0, stream, ev, x, y, layer,
                           p->n_layers, p->cordic, ws, O, phi_out);
    if (p->pt) {
        const int R = fine_rows(p);
        const int n_chunks = p->g.n_phi / R;
        hipLaunchKernelGGL(k_prep_fine, dim3(p->n_layers * n_chunks, n_events), dim3(kScanThreads),
                           fine_lds_bytes(p), stream, ev, p->n_layers, p->cell_bits, p->M, p->F, p->g.n_phi,
                           p->pt_row, pt_row8_for(p, n_events), R, n_chunks, p->layers, ws, O, st);
        return;
    }
    // events of at most cap_h hits are sorted by one workgroup per layer (LDS); the rank pass
    // runs only if a larger event is possible
    const int cap_h = bucket_cap_hits(p);
    const size_t lds_layer = cap_h > 0 ? 4 * ((((size_t)1 << p->cell_bits) + 3) & ~(size_t)3) + 8 * ((size_t)cap_h + 8)
                                       : 0;
    const size_t lds_all = 4 * (size_t)p->n_cells;
    const size_t lds = lds_layer > lds_all ? lds_layer : lds_all;
    hipLaunchKernelGGL(k_prep_bucket, dim3(p->n_layers, n_events), dim3(kScanThreads), lds, stream, ev,
                       p->n_layers, p->cell_bits, p->M, p->layers, ws, O, st, cap_h);
    if (max_n > cap_h)
        hipLaunchKernelGGL(k_prep_rank, dim3((max_n + 255) / 256, n_events), dim3(256), 0, stream, ev, p->n_cells,
                           p->cell_bits, p->M, ws, O);
}

// LDS of one vote workgroup: the slab, the queue word (padded to 256 bytes) and, for 16-bit slabs,
// the store tile of 64 columns x (TB + 1) words (TB = 64 bins for int16 outputs, 32 for int32).
size_t vote_lds_bytes(const hough_plan* p) {
    const size_t slab = (size_t)p->g.n_phi * ((size_t)1 << p->F);
    if (p->F == 8) return slab + 16;
    const size_t tb = p->g.acc_bits == 16 ? 64 : 32;
    return slab + 256 + 64 * (tb + 1) * 4;
}

// Columns per work item of the table vote: a single event takes the largest block that still gives
// every CU four workgroups; a batch takes 64 (fewer queue atomics).
int pt_cols_per_item(const hough_plan* p, bool single) {
    int cpi = p->tuning.vote_cols > 0 ? p->tuning.vote_cols : 64;
    if (p->tuning.vote_cols <= 0)
        while (single && cpi > 4 && (int64_t)p->n_cols / cpi < 4 * (int64_t)p->n_cu) cpi /= 2;
    while (p->n_cols % cpi) cpi /= 2;
    return cpi;
}

template <int BPL>
void launch_vote_pt_bpl(const hough_plan* p, const Events& ev, int n_events, char* ws, const WsOff& O, char* a,
                        size_t acc_stride, const int32_t* order, int32_t* queue, int grid, int cpi,
                        hipStream_t stream) {
    const uint32_t* zr = static_cast<const uint32_t*>(p->d_zero);
    if (p->g.acc_bits == 16)
        hipExtLaunchKernelGGL((k_vote_pt<BPL, true>), dim3(grid), dim3(kVotePtThreads), 0, stream, p->vote_start,
                              p->vote_stop, 0, ev, p->d_Et, p->et_stride, p->n_layers, p->n_cols, p->g.n_phi, p->M, p->F,
                              p->pt_row, pt_row8_for(p, n_events), zr, ws, O, a, acc_stride, n_events, order, queue,
                              cpi);
    else
        hipExtLaunchKernelGGL((k_vote_pt<BPL, false>), dim3(grid), dim3(kVotePtThreads), 0, stream, p->vote_start,
                              p->vote_stop, 0, ev, p->d_Et, p->et_stride, p->n_layers, p->n_cols, p->g.n_phi, p->M, p->F,
                              p->pt_row, pt_row8_for(p, n_events), zr, ws, O, a, acc_stride, n_events, order, queue,
                              cpi);
}

void launch_vote_pt(const hough_plan* p, const Events& ev, int n_events, char* ws, const WsOff& O, void* acc,
                    size_t acc_stride, const int32_t* order, int32_t* queue, int grid, hipStream_t stream) {
    const int cpi = pt_cols_per_item(p, queue == nullptr);
    const int64_t items = (int64_t)n_events * (p->n_cols / cpi);
    if (queue != nullptr && grid <= 0) grid = 8 * p->n_cu;  // persistent: eight workgroups per CU
    if (queue == nullptr || grid > items) grid = (int)items;
    char* a = static_cast<char*>(acc);
    switch (p->pt_bpl) {
        case 2: launch_vote_pt_bpl<2>(p, ev, n_events, ws, O, a, acc_stride, order, queue, grid, cpi, stream); break;
        case 4: launch_vote_pt_bpl<4>(p, ev, n_events, ws, O, a, acc_stride, order, queue, grid, cpi, stream); break;
        case 8: launch_vote_pt_bpl<8>(p, ev, n_events, ws, O, a, acc_stride, order, queue, grid, cpi, stream); break;
        case 16: launch_vote_pt_bpl<16>(p, ev, n_events, ws, O, a, acc_stride, order, queue, grid, cpi, stream); break;
        case 32: launch_vote_pt_bpl<32>(p, ev, n_events, ws, O, a, acc_stride, order, queue, grid, cpi, stream); break;
        default: launch_vote_pt_bpl<64>(p, ev, n_events, ws, O, a, acc_stride, order, queue, grid, cpi, stream); break;
    }
}

void launch_vote(const hough_plan* p, const Events& ev, int n_events, char* ws, const WsOff& O, void* acc,
                 size_t acc_stride, const int32_t* order, int32_t* queue, int grid, hough_status_t* st,
                 hipStream_t stream) {
    if (p->pt) {
        launch_vote_pt(p, ev, n_events, ws, O, acc, acc_stride, order, queue, grid, stream);
        return;
    }
    int threads = p->tuning.vote_threads;
    char* a = static_cast<char*>(acc);
    const int32_t* E = p->d_E;
    size_t lds = vote_lds_bytes(p);
    if (grid <= p->n_cu) {
        // At most one workgroup per CU: the most waves per workgroup, and more than half the LDS
        // so that no CU gets two slabs while another idles (the dispatcher packs what fits).
        threads = kVoteMaxThreads;
        if (lds <= (size_t)kLdsBytes / 2) lds = (size_t)kLdsBytes / 2 + 256;
    }
    // with timing events set, the launch itself records them at the kernel's start and end
    if (p->F == 8)
        hipExtLaunchKernelGGL(k_vote<false, false>, dim3(grid), dim3(threads), lds, stream,
                              p->vote_start, p->vote_stop, 0, ev, E, p->n_layers, p->cell_bits, p->n_cols,
                              p->g.n_phi, p->F, ws, O, a, acc_stride, n_events, order, queue, st);
    else if (p->g.acc_bits == 32)
        hipExtLaunchKernelGGL(k_vote<true, false>, dim3(grid), dim3(threads), lds, stream,
                              p->vote_start, p->vote_stop, 0, ev, E, p->n_layers, p->cell_bits, p->n_cols,
                              p->g.n_phi, p->F, ws, O, a, acc_stride, n_events, order, queue, st);
    else
        hipExtLaunchKernelGGL(k_vote<true, true>, dim3(grid), dim3(threads), lds, stream,
                              p->vote_start, p->vote_stop, 0, ev, E, p->n_layers, p->cell_bits, p->n_cols,
                              p->g.n_phi, p->F, ws, O, a, acc_stride, n_events, order, queue, st);
}

void launch_peaks(const hough_plan* p, const Events& ev, int n_events, const void* acc, size_t acc_stride,
                  int32_t threshold, hough_peak_t* peaks, int32_t cap, char* ws, const WsOff& O,
                  hough_status_t* st, hipStream_t stream) {
    const int strips = p->g.n_phi / kStrip;
    const int gl = peak_group_lanes(p);
    // fewer planes per thread while the launch would give a CU fewer than two workgroups (a single
    // event or a small batch: one 4-wave workgroup per CU leaves the loads too few waves to hide in)
    int planes = p->tuning.peak_planes;
    auto mark_blocks = [&](int pl) {
        return ((int64_t)strips * p->g.n_qpt * ((p->g.n_d0 + pl - 1) / pl) + kMarkThreads - 1) / kMarkThreads;
    };
    while (planes > 1 && mark_blocks(planes) * n_events < 2 * (int64_t)p->n_cu) planes = (planes + 1) / 2;
    const int lranges = (p->g.n_d0 + planes - 1) / planes;
    const int64_t mark_threads = (int64_t)strips * p->g.n_qpt * lranges;
    const int64_t n_strips = p->n_bins / kStrip;
    const int64_t groups = peak_groups(p);
    const dim3 gm((unsigned)(((mark_threads + kMarkThreads - 1) / kMarkThreads + 7) / 8 * 8), n_events);  // multiple of 8: see k_peaks_mark
    const int wsp = gl < kWriteStrips ? gl : kWriteStrips;
    const dim3 gw((unsigned)((n_strips / wsp + kWriteThreads - 1) / kWriteThreads), n_events);
    const char* a = static_cast<const char*>(acc);
    const int16_t* z16 = static_cast<const int16_t*>(p->d_zero);
    const int32_t* z32 = static_cast<const int32_t*>(p->d_zero);
    const int nd = p->g.n_d0, nq = p->g.n_qpt, nph = p->g.n_phi;
    const dim3 mb(kMarkThreads);
    // the one-pass scan and writer serves single events and small batches
    const bool one_pass = n_events <= kScanWriteMaxEvents && groups <= kScanWriteMaxGroups;
    // staged values pay off where the writer is a pass of its own (its accumulator gathers would be
    // spread over the whole batch); the one-pass writer reads the values where they lie.  The marker
    // of rows wider than a wave (more than 512 bins) holds more registers, and staging there costs
    // it a wave per SIMD: its writer gathers instead.
    const bool stage_on = p->stage && !one_pass && strips <= 64;
    const size_t mlds = mark_lds_bytes(planes, gl, stage_on);
    if (p->g.acc_bits == 32 && strips > 64)
        hipLaunchKernelGGL((k_peaks_mark<int32_t, true, true>), gm, mb, mlds, stream, ev, a, acc_stride, z32, threshold,
                           nd, nq, nph, gl, planes, stage_on, ws, O);
    else if (p->g.acc_bits == 32 && strips == 64)
        hipLaunchKernelGGL((k_peaks_mark<int32_t, false, true>), gm, mb, mlds, stream, ev, a, acc_stride, z32, threshold,
                           nd, nq, nph, gl, planes, stage_on, ws, O);
    else if (p->g.acc_bits == 32)
        hipLaunchKernelGGL((k_peaks_mark<int32_t, false, false>), gm, mb, mlds, stream, ev, a, acc_stride, z32, threshold,
                           nd, nq, nph, gl, planes, stage_on, ws, O);
    else if (strips > 64)
        hipLaunchKernelGGL((k_peaks_mark<int16_t, true, true>), gm, mb, mlds, stream, ev, a, acc_stride, z16, threshold,
                           nd, nq, nph, gl, planes, stage_on, ws, O);
    else if (strips == 64)
        hipLaunchKernelGGL((k_peaks_mark<int16_t, false, true>), gm, mb, mlds, stream, ev, a, acc_stride, z16, threshold,
                           nd, nq, nph, gl, planes, stage_on, ws, O);
    else
        hipLaunchKernelGGL((k_peaks_mark<int16_t, false, false>), gm, mb, mlds, stream, ev, a, acc_stride, z16, threshold,
                           nd, nq, nph, gl, planes, stage_on, ws, O);
    // scan and writer in one pass: each writer workgroup re-reads the counts of all groups before
    // it, so only while that is cheaper than a separate scan (few events, not too many groups)
    if (one_pass) {
        if (p->g.acc_bits == 32)
            hipLaunchKernelGGL(k_peaks_scan_write<int32_t>, gw, dim3(kWriteThreads), 0, stream, ev, a, acc_stride,
                               groups, p->g.n_qpt, p->g.n_phi, gl, n_strips, false, ws, O, peaks, cap, st);
        else
            hipLaunchKernelGGL(k_peaks_scan_write<int16_t>, gw, dim3(kWriteThreads), 0, stream, ev, a, acc_stride,
                               groups, p->g.n_qpt, p->g.n_phi, gl, n_strips, false, ws, O, peaks, cap, st);
        return;
    }
    // workgroups per event: enough to spread a small batch over the CUs, each with >= one tile
    int64_t chunks = 2 * (int64_t)p->n_cu / n_events;
    const int64_t by_size = groups / ((int64_t)kPScanThreads * kPScanPer);
    chunks = chunks < by_size ? chunks : by_size;
    chunks = chunks < 16 ? chunks : 16;
    chunks = chunks > 1 ? chunks : 1;
    hipLaunchKernelGGL(k_peaks_scan, dim3((unsigned)chunks, n_events), dim3(kPScanThreads), 0, stream, ev, groups,
                       cap, ws, O, st);
    if (p->g.acc_bits == 32)
        hipLaunchKernelGGL(k_peaks_write<int32_t>, gw, dim3(kWriteThreads), 0, stream, ev, a, acc_stride, groups, p->g.n_qpt,
                           p->g.n_phi, gl, n_strips, stage_on, ws, O, peaks, cap);
    else
        hipLaunchKernelGGL(k_peaks_write<int16_t>, gw, dim3(kWriteThreads), 0, stream, ev, a, acc_stride, groups, p->g.n_qpt,
                           p->g.n_phi, gl, n_strips, stage_on, ws, O, peaks, cap);
}

void launch_assign(const hough_plan* p, const Events& ev, int n_events, const hough_peak_t* peaks,
                   int32_t peak_stride, int32_t cap_peaks, int32_t* offsets, int32_t* hit_idx, int32_t cap_pairs,
                   char* ws, const WsOff& O, hough_status_t* st, hipStream_t stream,
                   const int32_t* order = nullptr) {
    // batches of at least 8 events: 512-thread workgroups with half the LDS, so that two share a CU
    // and one's table loads and staging overlap the other's copying; fewer events: 1024 threads and
    // the whole LDS, as for a single event
    const bool half = n_events >= kXcds && p->pt;
    const int threads = half ? kAssignThreads / 2 : kAssignThreads;
    const int64_t want = ((int64_t)cap_peaks + threads - 1) / threads;
    int64_t per_event_cap = p->tuning.assign_blocks > 0 ? p->tuning.assign_blocks : n_events > 1 ? 64 : 2 * 256;
    // a small batch still fills every CU once (one 1024-thread or two 512-thread workgroups per CU)
    const int64_t fill = ((int64_t)p->n_cu * (kAssignThreads / threads) + n_events - 1) / n_events;
    if (n_events > 1 && per_event_cap < fill) per_event_cap = fill;
    const unsigned nblk = (unsigned)(want < per_event_cap ? want : per_event_cap);
    // the kernel lays out its LDS per event (cell table, staged hits, wave buffers)
    const int cells_words = (p->n_cells + 1 + 3) & ~3;
    const int lds_words = kLdsBytes / 4;
    if (p->pt) {
        // large batches with the size order: events grouped per XCD, grid.y padded to a multiple of 8
        const int32_t* ord = n_events >= kXcdMinEvents ? order : nullptr;
        const unsigned gy = ord ? (unsigned)((n_events + kXcds - 1) / kXcds * kXcds) : (unsigned)n_events;
        if (half)
            hipExtLaunchKernelGGL(k_assign_pt<kAssignThreads / 2>, dim3(nblk, gy), dim3(kAssignThreads / 2),
                                  kLdsBytes / 2, stream, p->assign_start, p->assign_stop, 0, ev, peaks, peak_stride,
                                  cap_peaks, st, p->d_Et, p->et_stride, p->n_layers, p->cell_bits, p->n_cols,
                                  p->g.n_qpt, p->M, p->F, p->g.n_phi, p->pt_row, ws, O, offsets, hit_idx, cap_pairs,
                                  lds_words / 2, ord, n_events);
        else
            hipExtLaunchKernelGGL(k_assign_pt<kAssignThreads>, dim3(nblk, gy), dim3(kAssignThreads), kLdsBytes, stream,
                                  p->assign_start, p->assign_stop, 0, ev, peaks, peak_stride, cap_peaks, st, p->d_Et,
                                  p->et_stride, p->n_layers, p->cell_bits, p->n_cols, p->g.n_qpt, p->M, p->F,
                                  p->g.n_phi, p->pt_row, ws, O, offsets, hit_idx, cap_pairs, lds_words, ord, n_events);
        return;
    }
    // one packed word per staged hit: angles of at most 16 bits and hit indices below 2^16
    if (p->M <= 16 && p->g.max_hits_per_event <= 65536)
        hipLaunchKernelGGL(k_assign_fill<true>, dim3(nblk, n_events), dim3(kAssignThreads), kLdsBytes, stream, ev,
                           peaks, peak_stride, cap_peaks, st, p->d_E, p->n_layers, p->cell_bits, p->n_cols,
                           p->g.n_qpt, p->M, p->F, ws, O, offsets, hit_idx, cap_pairs, lds_words, cells_words);
    else
        hipLaunchKernelGGL(k_assign_fill<false>, dim3(nblk, n_events), dim3(kAssignThreads), kLdsBytes, stream, ev,
                           peaks, peak_stride, cap_peaks, st, p->d_E, p->n_layers, p->cell_bits, p->n_cols,
                           p->g.n_qpt, p->M, p->F, ws, O, offsets, hit_idx, cap_pairs, lds_words, cells_words);
}

void launch_fit(const Events& ev, int n_events, int n_cu, const float* x, const float* y, const int32_t* offsets,
                const int32_t* hit_idx, int32_t cap_peaks, int32_t cap_pairs, const hough_status_t* st, double* out,
                hipStream_t stream) {
    const int max_hits = ev.hit_off ? ev.max_hits : ev.n_single;
    if (max_hits <= kFitResHits) {  // coordinates resident in LDS
        const int res = (max_hits + 1) & ~1;
        const int64_t chunks = ((int64_t)cap_peaks + kFitResThreads - 1) / kFitResThreads;
        int64_t per_event = (2 * (int64_t)n_cu + n_events - 1) / n_events;
        per_event = per_event < chunks ? per_event : chunks;
        const dim3 grid((unsigned)(per_event > 0 ? per_event : 1), n_events);
        const size_t lds = (size_t)res * 8 + kFitResIdxBytes;
        hipLaunchKernelGGL(k_fit_res, grid, dim3(kFitResThreads), lds, stream, ev, x, y, offsets, hit_idx, cap_peaks,
                           cap_pairs, st, out, res);
        return;
    }
    const dim3 grid((unsigned)(((int64_t)cap_peaks + kFitThreads - 1) / kFitThreads), n_events);
    hipLaunchKernelGGL(k_fit, grid, dim3(kFitThreads), 0, stream, ev, x, y, offsets, hit_idx, cap_peaks, cap_pairs,
                       st, out);
}

void launch_zvote(const hough_plan* p, const Events& ev, int n_events, const float* z, const uint8_t* layer,
                  const hough_peak_t* peaks, int32_t cap_peaks, const int32_t* offsets, const int32_t* hit_idx,
                  int32_t cap_pairs, const hough_status_t* st, int32_t* out, hipStream_t stream) {
    // enough waves to fill the chip several times over, split over the events; a wave takes groups
    // of kZvoteGroup candidates
    const int64_t want = ((int64_t)cap_peaks + 4 * kZvoteGroup - 1) / (4 * kZvoteGroup);
    int64_t per_event = (2560 + n_events - 1) / n_events;
    per_event = per_event < want ? per_event : want;
    const unsigned nblk = (unsigned)(per_event > 0 ? per_event : 1);
    const size_t slots_words = ((size_t)kZvoteSlots * (p->zg.n_z0 + 1) + 1) & ~(size_t)1;
    const size_t lds = (size_t)(kZvoteThreads / 64) * (slots_words * 4 + 8 * kZvoteStage);
    hipLaunchKernelGGL(k_zvote, dim3(nblk, n_events), dim3(kZvoteThreads), lds, stream, ev, z, layer, p->n_layers,
                       peaks, cap_peaks, offsets, hit_idx, cap_pairs, st, p->d_S, p->g.n_d0, p->g.n_qpt, p->zg, out);
}

// ------------------------------------------------------------------ second transform (vertices)
// Vertex space: rows j (radius centres) x n_vphi azimuth bins.  A first-stage candidate (l, k, b)
// votes, in every row whose sample T[l][k][j] is valid, for the azimuth bin of
// (b * 2^F + 2^(F-1) + T) mod 2^M, i.e. where its bin-centre helix meets the row's radius.
//
// k_vvote: workgroup (g, s) counts the votes of candidate range g into rows [64 s, 64 s + 64) in
// LDS, lane = row, exactly like the first transform's slab (16-bit halves: rows c and c + 32 share
// the dword (bin * 32 + c), so a 32-lane half of a ds_add touches 32 distinct dwords), and copies
// its slab to its own partial in ws.  A half never carries: a row counts at most one vote per
// candidate and a range holds at most 65535 candidates.  k_vreduce adds the partials.
constexpr int kVvoteThreads = 1024;
constexpr int kVvoteUnroll = 8;
constexpr int kVreduceThreads = 1024;
constexpr int kVertexMaxRange = 65535;  // candidates per partial (16-bit halves)

struct VGrid {
    int32_t n_d0, n_qpt, n_phi, n_vr, n_vphi, F, min_votes, groups;
    uint32_t mask_m;   // 2^M - 1
    int32_t shift;     // M - log2(n_vphi): bits of the M-bit angle below one vertex bin
};

// Candidates listed by the first stage and the split into ranges of the vertex vote; identical in
// both kernels so that the reduction reads exactly the partials that were written.
__device__ __forceinline__ void vertex_ranges(const hough_status_t* st, int32_t cap, int32_t groups, int& n,
                                              int& chunk, int& active) {
    n = min(st->n_peaks, cap);
    n = n > 0 ? n : 0;
    chunk = (n + groups - 1) / groups;
    active = chunk > 0 ? (n + chunk - 1) / chunk : 0;
}

__global__ __launch_bounds__(kVvoteThreads) void k_vvote(const hough_peak_t* __restrict__ peaks_base, int32_t cap,
                                                         const hough_status_t* __restrict__ st_base,
                                                         const int32_t* __restrict__ T, VGrid vg,
                                                         uint32_t* __restrict__ partial_base, size_t partial_stride,
                                                         hough_status_t* __restrict__ st_v_base) {
    extern __shared__ uint32_t slab[];
    const int g = blockIdx.x, s = blockIdx.y, e = blockIdx.z, tid = threadIdx.x;
    const hough_peak_t* peaks = peaks_base + (size_t)e * cap;
    const hough_status_t* st = st_base + e;
    uint32_t* partial = partial_base + (size_t)e * partial_stride;
    hough_status_t* st_v = st_v_base + e;
    int n, chunk, active;
    vertex_ranges(st, cap, vg.groups, n, chunk, active);
    if (g == 0 && s == 0 && tid == 0) {
        st_v->n_hits = n;
        st_v->n_bad_hits = 0;
        st_v->n_votes = 0;
        st_v->n_peaks = 0;
        st_v->flags = 0;
        st_v->n_pairs = 0;
    }
    if (g >= active) return;
    const int p0 = g * chunk, p1 = min(n, p0 + chunk);
    const int words = vg.n_vphi * 32;
    for (int i = tid; i < words / 4; i += kVvoteThreads) reinterpret_cast<uint4*>(slab)[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const uint32_t inc = lane < 32 ? 1u : 65536u;
    const int32_t* Trow = T + s * 64 + lane;
    const uint32_t half = 1u << (vg.F - 1);
    // Candidates come sorted by linear index, so runs of them share a (l, k) column and with it the
    // table row (lane = radius row).  A wave takes 64 candidates (lane = candidate), marks the first
    // of each run (a head), loads the rows of up to kVvoteUnroll heads at once and then votes every
    // candidate of those runs (lane = row again) with the candidate's angle broadcast by readlane.
    // The next 64 candidates are loaded after the rows, so waiting for a row never waits for them.
    // Angles are held left-aligned in 32 bits (M-bit angle << (32 - M)), so the angle sum wraps
    // mod 2^M by itself and the azimuth bin is its top log2(n_vphi) bits.  Per vote: readlane,
    // add, shift, and-or into the LDS byte address, ds_add; a row without a valid sample adds 0.
    constexpr int kStride = (kVvoteThreads / 64) * 64;
    const uint32_t lv = 32u - (uint32_t)__builtin_clz((uint32_t)vg.n_vphi) - 1u;  // log2 n_vphi
    const uint32_t lsh = 32u - (uint32_t)vg.shift - lv;                                // 32 - M (M = shift + lv)
    const uint32_t to_row = 25u - lv;   // (sum >> to_row) & ~127 = bin * 128 (a 128-byte slab row)
    const uint32_t loff = (uint32_t)(lane & 31) << 2;
    const uint32_t row_mask = __builtin_amdgcn_readfirstlane(0xFFFFFF80u);
    int base = p0 + wave * 64;
    int4 c4 = make_int4(0, 0, 0, 0);  // votes 0 < min_votes: lanes past the range cast nothing
    if (base + lane < p1) c4 = *reinterpret_cast<const int4*>(peaks + base + lane);
    for (; base < p1; base += kStride) {
        // a bin outside the first grid (not one the peak finder writes) casts nothing
        const bool on = c4.w >= vg.min_votes && (unsigned)c4.x < (unsigned)vg.n_d0 &&
                        (unsigned)c4.y < (unsigned)vg.n_qpt && (unsigned)c4.z < (unsigned)vg.n_phi;
        const int key = on ? c4.x * vg.n_qpt + c4.y : -1;
        const int prev = __shfl_up(key, 1, 64);
        uint64_t heads = __ballot(on && (lane == 0 || key != prev));
        const uint64_t onm = __ballot(on);
        // the candidate's phi0 centre, left-aligned
        const uint32_t ang = (((uint32_t)c4.z << vg.F) + half) << lsh;
        bool fetched = false;
        while (heads) {
            int h[kVvoteUnroll + 1];
            uint32_t e[kVvoteUnroll];
#pragma unroll
            for (int u = 0; u < kVvoteUnroll; ++u) {
                h[u] = heads ? (int)__builtin_ctzll(heads) : 64;
                heads &= heads - 1;  // (no-op once empty)
                const int kk = __builtin_amdgcn_readlane(key, h[u] < 64 ? h[u] : 0);
                e[u] = (uint32_t)Trow[(size_t)(h[u] < 64 ? kk : 0) * vg.n_vr];
            }
            h[kVvoteUnroll] = heads ? (int)__builtin_ctzll(heads) : 64;  // end of the last run
            if (!fetched) {
                fetched = true;
                const int nb = base + kStride;
                int4 t = make_int4(0, 0, 0, 0);
                if (nb + lane < p1) t = *reinterpret_cast<const int4*>(peaks + nb + lane);
                c4 = t;
            }
#pragma unroll
            for (int u = 0; u < kVvoteUnroll; ++u) {
                if (h[u] >= 64) break;
                const uint32_t data = e[u] != (uint32_t)INT32_MIN ? inc : 0u;
                const uint32_t el = e[u] << lsh;
                const int span = h[u + 1] - h[u];
                const uint64_t rmask = span >= 64 ? ~0ull : (((1ull << span) - 1ull) << h[u]);
                uint64_t m = onm & rmask;
                // one vote: the candidate's angle by readlane, the slab byte address (the slab starts at
                // LDS address 0: the kernel has no static LDS) by one and-or, the atomic
                auto vote = [&](int i) {
                    const uint32_t sum = (uint32_t)__builtin_amdgcn_readlane((int)ang, i) + el;
                    uint32_t off;  // one and-or (the compiler otherwise splits it into an and and an add)
                    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(off) : "v"(sum >> to_row), "s"(row_mask), "v"(loff));
                    asm volatile("ds_add_u32 %0, %1" ::"v"(off), "v"(data) : "memory");
                };
                if (m == rmask) {  // every candidate of the run votes (the usual case): a counted loop
                    const int i1 = h[u + 1];
                    int i = h[u];
                    for (; i + 1 < i1; i += 2) {
                        vote(i);
                        vote(i + 1);
                    }
                    if (i < i1) vote(i);
                } else {
                    while (m) {
                        const int i = (int)__builtin_ctzll(m);
                        m &= m - 1;
                        vote(i);
                    }
                }
            }
        }
        if (!fetched) {  // no candidate of this chunk votes
            const int nb = base + kStride;
            int4 t = make_int4(0, 0, 0, 0);
            if (nb + lane < p1) t = *reinterpret_cast<const int4*>(peaks + nb + lane);
            c4 = t;
        }
    }
    // the atomics above are inline asm, which the compiler's wait counting does not see
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __syncthreads();
    uint4* dst = reinterpret_cast<uint4*>(partial + ((size_t)s * vg.groups + g) * words);
    for (int i = tid; i < words / 4; i += kVvoteThreads) dst[i] = reinterpret_cast<const uint4*>(slab)[i];
}

// One workgroup per 64 dwords of the slab layout (all rows' partials of 32 rows x 2 bins); wave w
// adds ranges w, w + 16, ...; the sums are combined in LDS and split into the two rows of a dword.
__global__ __launch_bounds__(kVreduceThreads) void k_vreduce(const hough_status_t* __restrict__ st_base, int32_t cap,
                                                             VGrid vg, const uint32_t* __restrict__ partial_base,
                                                             size_t partial_stride, int32_t* __restrict__ acc_v_base,
                                                             hough_status_t* __restrict__ st_v_base) {
    __shared__ uint32_t lo_s[kVreduceThreads / 64][64], hi_s[kVreduceThreads / 64][64];
    const int e = blockIdx.y;
    const hough_status_t* st = st_base + e;
    const uint32_t* partial = partial_base + (size_t)e * partial_stride;
    int32_t* acc_v = acc_v_base + (size_t)e * vg.n_vr * vg.n_vphi;
    hough_status_t* st_v = st_v_base + e;
    int n, chunk, active;
    vertex_ranges(st, cap, vg.groups, n, chunk, active);
    const int words = vg.n_vphi * 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t d = (int64_t)blockIdx.x * 64 + lane;  // dword of all slabs: s * words + w
    const int s = (int)(d / words), w = (int)(d % words);
    const uint32_t* src = partial + (size_t)s * vg.groups * words + w;
    uint32_t lo = 0, hi = 0;
    constexpr int kW = kVreduceThreads / 64;
    int g = wave;
    for (; g + 3 * kW < active; g += 4 * kW) {
        const uint32_t a0 = src[(size_t)g * words], a1 = src[(size_t)(g + kW) * words];
        const uint32_t a2 = src[(size_t)(g + 2 * kW) * words], a3 = src[(size_t)(g + 3 * kW) * words];
        lo += (a0 & 0xFFFFu) + (a1 & 0xFFFFu) + (a2 & 0xFFFFu) + (a3 & 0xFFFFu);
        hi += (a0 >> 16) + (a1 >> 16) + (a2 >> 16) + (a3 >> 16);
    }
    for (; g < active; g += kW) {
        const uint32_t a = src[(size_t)g * words];
        lo += a & 0xFFFFu;
        hi += a >> 16;
    }
    lo_s[wave][lane] = lo;
    hi_s[wave][lane] = hi;
    __syncthreads();
    if (wave == 0) {
        uint32_t L = 0, H = 0;
#pragma unroll
        for (int i = 0; i < kW; ++i) {
            L += lo_s[i][lane];
            H += hi_s[i][lane];
        }
        const int bin = w >> 5, c = w & 31;
        acc_v[((size_t)s * 64 + c) * vg.n_vphi + bin] = (int32_t)L;
        acc_v[((size_t)s * 64 + c + 32) * vg.n_vphi + bin] = (int32_t)H;
        unsigned long long t = (unsigned long long)L + H;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&st_v->n_votes), t);
    }
}

// n_events events: candidate lists at peaks + e * cap, statuses st[e] and st_v[e], vertex spaces at
// acc_v + e * n_vr * n_vphi, partials at partial + e * (slabs * groups * n_vphi * 32) words.
void launch_vertex_vote(const VGrid& vg, int slabs, int n_events, const hough_peak_t* peaks, int32_t cap,
                        const hough_status_t* st, const int32_t* T, uint32_t* partial, int32_t* acc_v,
                        hough_status_t* st_v, hipStream_t stream) {
    const size_t lds = (size_t)vg.n_vphi * 128;
    const size_t pstride = (size_t)slabs * vg.groups * vg.n_vphi * 32;
    hipLaunchKernelGGL(k_vvote, dim3((unsigned)vg.groups, (unsigned)slabs, (unsigned)n_events), dim3(kVvoteThreads),
                       lds, stream, peaks, cap, st, T, vg, partial, pstride, st_v);
    const unsigned rblocks = (unsigned)((int64_t)slabs * vg.n_vphi * 32 / 64);
    hipLaunchKernelGGL(k_vreduce, dim3(rblocks, (unsigned)n_events), dim3(kVreduceThreads), 0, stream, st, cap, vg,
                       partial, pstride, acc_v, st_v);
}

int check_hits(const hough_plan* p, const hough_hits_t* hits) {
    if (!p || !hits) return HOUGH_E_INVAL;
    if (hits->n < 0 || hits->n > p->g.max_hits_per_event) return HOUGH_E_INVAL;
    if (hits->n > 0 && (!hits->x || !hits->y || !hits->layer)) return HOUGH_E_INVAL;
    return HOUGH_OK;
}

Events single_event(const hough_plan* p, int n) { return Events{nullptr, n, p->g.max_hits_per_event, 0}; }

}  // namespace

// Second transform (vertex space) of one first-stage plan.
struct hough_vertex_plan {
    const hough_plan* first;  // not owned
    hough_plan* grid;         // the vertex space as a (1 x n_vr x n_vphi) plan: its peak finder
    hough_vertex_grid_t vg;
    int32_t* d_T;             // [n_d0][n_qpt][n_vr] sample at each row radius, INT32_MIN = invalid
    int slabs;                // n_vr / 64
    int groups;               // candidate ranges (partials) per slab, at least
};

namespace {
// Candidate ranges per event: the plan's count spread over the events of a launch, and at least
// enough that no range holds more than kVertexMaxRange candidates.
int vertex_groups(const hough_vertex_plan* vp, int32_t cap, int32_t n_events = 1) {
    const int64_t need = ((int64_t)cap + kVertexMaxRange - 1) / kVertexMaxRange;
    const int64_t spread = ((int64_t)vp->groups + n_events - 1) / n_events;
    return (int)(need > spread ? need : spread);
}

size_t vertex_partial_bytes(const hough_vertex_plan* vp, int32_t cap, int32_t n_events = 1) {
    return (size_t)n_events * vp->slabs * vertex_groups(vp, cap, n_events) * vp->vg.n_vphi * 128;
}

VGrid vertex_vgrid(const hough_vertex_plan* vp, int32_t cap, int32_t n_events = 1) {
    const hough_plan* p = vp->first;
    VGrid v{};
    v.n_d0 = p->g.n_d0;
    v.n_qpt = p->g.n_qpt;
    v.n_phi = p->g.n_phi;
    v.n_vr = vp->vg.n_vr;
    v.n_vphi = vp->vg.n_vphi;
    v.F = p->F;
    v.min_votes = vp->vg.min_votes;
    v.groups = vertex_groups(vp, cap, n_events);
    v.mask_m = p->M >= 32 ? 0xFFFFFFFFu : ((1u << p->M) - 1u);
    v.shift = p->M - ilog2_exact(vp->vg.n_vphi);
    return v;
}
}  // namespace

// ====================================================================== C ABI
// Workspace of hough_run_batch_noalloc: one copy per GPU, held until the process ends.
static __device__ __align__(256) char scratch[HOUGH_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::atomic<void*> g_scratch_dev[kMaxScratchDevices];
std::mutex g_scratch_mu;

// With `device` current: look up the device address of that GPU's copy of `scratch` once and keep it.
int noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return HOUGH_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device].load(std::memory_order_acquire)) return HOUGH_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();  // a later launch check must not report this failure
        return HOUGH_E_HIP;
    }
    g_scratch_dev[device].store(ptr, std::memory_order_release);
    return HOUGH_OK;
}

void* noalloc_scratch_get(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    return g_scratch_dev[device].load(std::memory_order_acquire);
}

}  // namespace

extern "C" {

const char* hough_strerror(int code) {
    switch (code) {
        case HOUGH_OK: return "ok";
        case HOUGH_E_INVAL: return "invalid argument";
        case HOUGH_E_UNSUPPORTED: return "unsupported grid or geometry";
        case HOUGH_E_HIP: return "HIP runtime error";
        case HOUGH_E_NOMEM: return "out of device memory";
        case HOUGH_E_SMALL_WS: return "workspace too small";
        default: return "unknown error";
    }
}

int hough_plan_create(const hough_geometry_t* geom, const hough_grid_t* grid, hough_plan_t** out) {
    if (!geom || !grid || !out || !geom->r_cm) return HOUGH_E_INVAL;
    *out = nullptr;
    const hough_grid_t& g = *grid;
    if (geom->n_layers < 1 || geom->n_layers > kMaxLayers) return HOUGH_E_UNSUPPORTED;
    if (!std::isfinite(geom->B_tesla)) return HOUGH_E_INVAL;
    for (int L = 0; L < geom->n_layers; ++L)
        if (!(geom->r_cm[L] > 0.0) || !std::isfinite(geom->r_cm[L])) return HOUGH_E_INVAL;
    const int lp = ilog2_exact(g.n_phi);
    if (lp < 4 || lp > 12) return HOUGH_E_UNSUPPORTED;
    if (g.n_qpt < 1 || g.n_d0 < 1 || g.max_hits_per_event < 1) return HOUGH_E_INVAL;
    if (g.max_hits_per_event > (1 << 24) - 1) return HOUGH_E_UNSUPPORTED;
    if (g.n_qpt % kVoteCols) return HOUGH_E_UNSUPPORTED;
    // vote slab rows are 2^F bytes: F = 8 -> 32-bit counters, F = 7 -> 16-bit counters
    if (g.acc_bits != 32 && g.acc_bits != 16) return HOUGH_E_UNSUPPORTED;
    if (g.frac_bits == 8) {
        if (g.acc_bits != 32) return HOUGH_E_UNSUPPORTED;
    } else if (g.frac_bits == 7) {
        if (g.max_hits_per_event > (g.acc_bits == 16 ? 32767 : 65535)) return HOUGH_E_UNSUPPORTED;
    } else {
        return HOUGH_E_UNSUPPORTED;
    }
    // the slab of one vote workgroup (and its store tile) must fit the 160 KiB of LDS
    {
        const size_t slab = (size_t)g.n_phi * ((size_t)1 << g.frac_bits);
        const size_t tile = g.frac_bits == 8 ? 0 : 256 + 64 * (size_t)((g.acc_bits == 16 ? 64 : 32) + 1) * 4;
        if (slab + 16 + tile > (size_t)kLdsBytes) return HOUGH_E_UNSUPPORTED;
    }
    if (!(g.qpt_max >= g.qpt_min) || !(g.d0_max >= g.d0_min)) return HOUGH_E_INVAL;
    if ((int64_t)g.n_d0 * g.n_qpt * g.n_phi > ((int64_t)1 << 31)) return HOUGH_E_UNSUPPORTED;
    if ((geom->n_layers << (lp < 10 ? lp : 10)) > kMaxCells) return HOUGH_E_UNSUPPORTED;
    // second-stage r-z grid: cot(theta) centres on an exact Q16.16 progression, z0 bins of a
    // power-of-two width in Q32.32 (the integer forms the zvote kernel steps through)
    const bool zvote = g.n_cot != 0 || g.n_z0 != 0;
    ZGrid zg{};
    if (zvote) {
        if (g.n_cot < 1 || g.n_z0 < 1) return HOUGH_E_INVAL;
        if (g.n_z0 > kZvoteMaxZ0 || (int64_t)g.n_cot * g.n_z0 > 65536) return HOUGH_E_UNSUPPORTED;
        if (g.max_hits_per_event > 65535) return HOUGH_E_UNSUPPORTED;
        if (!std::isfinite(g.cot_min) || !std::isfinite(g.cot_max) || !(g.cot_max > g.cot_min) ||
            !std::isfinite(g.z0_min) || !std::isfinite(g.z0_max) || !(g.z0_max > g.z0_min))
            return HOUGH_E_INVAL;
        if (fabs(g.cot_min) > 1024.0 || fabs(g.cot_max) > 1024.0 || fabs(g.z0_min) > 32768.0 ||
            fabs(g.z0_max) > 32768.0)
            return HOUGH_E_UNSUPPORTED;
        const int64_t W = llrint(((g.z0_max - g.z0_min) / (double)g.n_z0) * 4294967296.0);
        if (W < 1 || (W & (W - 1))) return HOUGH_E_UNSUPPORTED;
        int shift = 0;
        while (((int64_t)1 << shift) < W) ++shift;
        zg.n_cot = g.n_cot;
        zg.n_z0 = g.n_z0;
        zg.shift = shift;
        zg.z0min = llrint(g.z0_min * 4294967296.0);
        zg.lim = (uint64_t)g.n_z0 << shift;
        const double cstep = (g.cot_max - g.cot_min) / (double)g.n_cot;
        for (int m = 0; m < g.n_cot; ++m) {
            const int64_t C = llrint((g.cot_min + ((double)m + 0.5) * cstep) * 65536.0);
            if (m == 0) zg.c0 = C;
            if (m == 1) zg.dc = C - zg.c0;
            if (C != zg.c0 + (int64_t)m * zg.dc) return HOUGH_E_UNSUPPORTED;
        }
    }

    hough_plan* p = new (std::nothrow) hough_plan();
    if (!p) return HOUGH_E_NOMEM;
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) {
        delete p;
        return HOUGH_E_HIP;
    }
    // set-up of the no-alloc entry point on this device (its failure only disables that entry point)
    (void)noalloc_scratch_init(p->device);
    p->n_layers = geom->n_layers;
    for (int L = 0; L < p->n_layers; ++L) {
        p->r[L] = geom->r_cm[L];
        p->halflen[L] = geom->halflen_cm ? geom->halflen_cm[L] : 0.0;
    }
    p->B = geom->B_tesla;
    p->g = g;
    p->zvote = zvote;
    p->zg = zg;
    p->log2_phi = lp;
    p->F = g.frac_bits;
    p->M = lp + g.frac_bits;
    // one azimuth cell per phi0 bin (at most 2^10 cells per layer): a bin's window spans <= 2 cells
    p->cell_bits = lp < 10 ? lp : 10;
    // window-table path: every window count fits 16 bits (at most 65535 hits per event) and a
    // column's bins split evenly over the 64 lanes of a wave in pairs
    p->pt = g.max_hits_per_event <= 65535 && g.n_phi >= 128;
    p->stage = g.max_hits_per_event <= 65535;  // a bin holds at most one vote per hit
    p->pt_bpl = g.n_phi / 64;
    p->pt_row = ((g.n_phi + p->pt_bpl + 2) + 7) & ~7;  // window-count rows: entries a lane reads past the turn
    // 8-bit window counts: a lane reads its bins as whole dwords (at least four bins per lane)
    p->pt_row8 = p->pt_bpl >= 4 ? ((g.n_phi + p->pt_bpl + 4) + 15) & ~15 : 0;
    p->n_cols = g.n_d0 * g.n_qpt;
    p->n_cells = p->n_layers << p->cell_bits;
    p->n_bins = (int64_t)p->n_cols * g.n_phi;
    p->tuning.vote_threads = 1024;
    p->tuning.vote_grid = 0;
    p->tuning.peak_planes = 8;
    p->tuning.vote_cols = 0;
    p->tuning.assign_blocks = 0;
    p->tuning.prep_rows = 0;
    for (int i = 0; i < kCordicSteps; ++i)
        p->cordic.t[i] = (int32_t)llrint(atan(ldexp(1.0, -i)) * (2147483648.0 / M_PI));

    // sample table E[L][l][k] in IEEE double (no contraction: built with -ffp-contract=off)
    const size_t ntab = (size_t)p->n_layers * p->n_cols;
    int32_t* E = (int32_t*)malloc(ntab * sizeof(int32_t));
    if (!E) {
        delete p;
        return HOUGH_E_NOMEM;
    }
    int32_t* Stab = nullptr;
    if (zvote) {
        Stab = (int32_t*)malloc(ntab * sizeof(int32_t));
        if (!Stab) {
            free(E);
            delete p;
            return HOUGH_E_NOMEM;
        }
    }
    bool s_range_ok = true;
    const double kappa = 0.299792458e-2 * p->B;
    const double K = ldexp(1.0, p->M - 1) / M_PI;
    for (int L = 0; L < p->n_layers; ++L) {
        int32_t nvalid = 0;
        const double r = p->r[L];
        for (int l = 0; l < g.n_d0; ++l) {
            const double d = g.d0_min + ((double)l + 0.5) * ((g.d0_max - g.d0_min) / (double)g.n_d0);
            for (int k = 0; k < g.n_qpt; ++k) {
                const double q = g.qpt_min + ((double)k + 0.5) * ((g.qpt_max - g.qpt_min) / (double)g.n_qpt);
                const double c = -kappa * q;
                const double num = c * (r * r + d * d) + 2.0 * d;
                const double den = 2.0 * r * (1.0 + c * d);
                int32_t v = INT32_MIN, sv = -1;
                if (den > 0.0) {
                    const double A = num / den;
                    if (fabs(A) <= 1.0) {
                        v = (int32_t)llrint(asin(A) * K);
                        ++nvalid;
                        if (Stab) {
                            // arc length in the transverse plane from the origin to the layer crossing:
                            // chord length, then the arc of curvature c over it
                            const double Lc2 = r * r + d * d - 2.0 * d * r * A;
                            const double Lc = sqrt(Lc2 > 0.0 ? Lc2 : 0.0);
                            double sl;
                            if (c == 0.0) {
                                sl = Lc;
                            } else {
                                double u = fabs(c) * Lc / 2.0;
                                if (u > 1.0) u = 1.0;
                                sl = (2.0 / fabs(c)) * asin(u);
                            }
                            const long long S = llrint(sl * 65536.0);
                            if (S > INT32_MAX) s_range_ok = false;
                            sv = (int32_t)(S > INT32_MAX ? INT32_MAX : S);
                        }
                    }
                }
                E[((size_t)L * g.n_d0 + l) * g.n_qpt + k] = v;
                if (Stab) Stab[((size_t)L * g.n_d0 + l) * g.n_qpt + k] = sv;
            }
        }
        p->layers.valid_cols[L] = nvalid;
    }
    if (!s_range_ok) {
        free(E);
        free(Stab);
        delete p;
        return HOUGH_E_UNSUPPORTED;
    }
    // the column-major copy for the table vote: every layer group it reads (up to ten layers from a
    // layer below n_layers) stays inside a column's et_stride entries
    p->et_stride = (p->n_layers + 9 + 15) & ~15;  // at most 64 (n_layers <= 32): one wave's lanes
    const size_t ntab_pad = (ntab + 15) & ~(size_t)15;
    const size_t n_et = (size_t)p->n_cols * p->et_stride;
    int32_t* Et = (int32_t*)malloc(n_et * sizeof(int32_t));
    if (!Et || hipMalloc(&p->d_E, (ntab_pad + n_et) * sizeof(int32_t)) != hipSuccess) {
        free(Et);
        free(E);
        free(Stab);
        delete p;
        return HOUGH_E_NOMEM;
    }
    for (int c = 0; c < p->n_cols; ++c)
        for (int L = 0; L < p->et_stride; ++L)
            Et[(size_t)c * p->et_stride + L] = L < p->n_layers ? E[(size_t)L * p->n_cols + c] : INT32_MIN;
    p->d_Et = p->d_E + ntab_pad;
    if (hipMalloc(&p->d_zero, (size_t)g.n_phi * 4) != hipSuccess ||
        hipMemset(p->d_zero, 0, (size_t)g.n_phi * 4) != hipSuccess) {
        if (p->d_zero) (void)hipFree(p->d_zero);
        (void)hipFree(p->d_E);
        free(E);
        free(Stab);
        delete p;
        return HOUGH_E_NOMEM;
    }
    if (Stab && hipMalloc(&p->d_S, ntab * sizeof(int32_t)) != hipSuccess) {
        (void)hipFree(p->d_zero);
        (void)hipFree(p->d_E);
        free(E);
        free(Stab);
        delete p;
        return HOUGH_E_NOMEM;
    }
    hipError_t ce = hipMemcpy(p->d_E, E, ntab * sizeof(int32_t), hipMemcpyHostToDevice);
    if (ce == hipSuccess)
        ce = hipMemcpy(p->d_E + ntab_pad, Et, n_et * sizeof(int32_t), hipMemcpyHostToDevice);
    if (ce == hipSuccess && Stab) ce = hipMemcpy(p->d_S, Stab, ntab * sizeof(int32_t), hipMemcpyHostToDevice);
    free(E);
    free(Et);
    free(Stab);
    if (ce != hipSuccess) {
        (void)hipFree(p->d_E);
        (void)hipFree(p->d_zero);
        if (p->d_S) (void)hipFree(p->d_S);
        delete p;
        return HOUGH_E_HIP;
    }
    // dynamic LDS limits set to the whole 160 KiB once (a lower per-plan value would break other plans)
    hipError_t ae = hipFuncSetAttribute((const void*)k_vote<false, false>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_vote<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_vote<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_assign_fill<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_assign_fill<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_prep_bucket, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kLdsBytes - 1024);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_assign_pt<kAssignThreads>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_assign_pt<kAssignThreads / 2>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes / 2);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_prep_fine, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kLdsBytes - 1024);  // static LDS aside
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_zvote, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_peaks_mark<int32_t, false, false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_peaks_mark<int32_t, false, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_peaks_mark<int32_t, true, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_peaks_mark<int16_t, false, false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_peaks_mark<int16_t, false, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_peaks_mark<int16_t, true, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (ae == hipSuccess)
        ae = hipFuncSetAttribute((const void*)k_fit_res, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (ae != hipSuccess) {
        (void)hipFree(p->d_E);
        (void)hipFree(p->d_zero);
        if (p->d_S) (void)hipFree(p->d_S);
        delete p;
        return HOUGH_E_HIP;
    }
    *out = p;
    return HOUGH_OK;
}

void hough_plan_destroy(hough_plan_t* plan) {
    if (!plan) return;
    if (plan->d_E) (void)hipFree(plan->d_E);
    if (plan->d_S) (void)hipFree(plan->d_S);
    if (plan->d_zero) (void)hipFree(plan->d_zero);
    delete plan;
}

int hough_plan_set_tuning(hough_plan_t* p, const hough_tuning_t* t) {
    if (!p || !t) return HOUGH_E_INVAL;
    if (t->vote_threads != 256 && t->vote_threads != 512 && t->vote_threads != 1024) return HOUGH_E_INVAL;
    if (t->vote_grid < 0 || t->peak_planes < 1 || t->peak_planes > kMaxPeakPlanes) return HOUGH_E_INVAL;
    if (t->vote_cols != 0 && (t->vote_cols < 4 || t->vote_cols > 64 || (t->vote_cols & (t->vote_cols - 1))))
        return HOUGH_E_INVAL;
    if (t->assign_blocks < 0 || t->assign_blocks > 4096) return HOUGH_E_INVAL;
    if (t->prep_rows != 0 && (t->prep_rows < 16 || t->prep_rows > 256 || (t->prep_rows & (t->prep_rows - 1))))
        return HOUGH_E_INVAL;
    p->tuning = *t;
    return HOUGH_OK;
}

int hough_plan_set_vote_events(hough_plan_t* p, hipEvent_t start, hipEvent_t stop) {
    if (!p) return HOUGH_E_INVAL;
    p->vote_start = start;
    p->vote_stop = stop;
    return HOUGH_OK;
}

int hough_plan_set_assign_events(hough_plan_t* p, hipEvent_t start, hipEvent_t stop) {
    if (!p) return HOUGH_E_INVAL;
    p->assign_start = start;
    p->assign_stop = stop;
    return HOUGH_OK;
}

int hough_plan_get_tuning(const hough_plan_t* p, hough_tuning_t* t) {
    if (!p || !t) return HOUGH_E_INVAL;
    *t = p->tuning;
    return HOUGH_OK;
}

size_t hough_acc_bytes(const hough_plan_t* p) { return p ? (size_t)p->n_bins * (p->g.acc_bits / 8) : 0; }

size_t hough_event_ws_bytes(const hough_plan_t* p, int32_t max_peaks) {
    return p ? ws_layout(p, max_peaks).total : 0;
}

int32_t hough_angle_bits(const hough_plan_t* p) { return p ? p->M : -1; }

int hough_plan_table(const hough_plan_t* p, int32_t* out) {
    if (!p || !out) return HOUGH_E_INVAL;
    const size_t n = (size_t)p->n_layers * p->n_cols;
    return hipMemcpy(out, p->d_E, n * sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess ? HOUGH_OK
                                                                                             : HOUGH_E_HIP;
}

int hough_plan_arclen_table(const hough_plan_t* p, int32_t* out) {
    if (!p || !out) return HOUGH_E_INVAL;
    if (!p->zvote) return HOUGH_E_UNSUPPORTED;
    const size_t n = (size_t)p->n_layers * p->n_cols;
    return hipMemcpy(out, p->d_S, n * sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess ? HOUGH_OK
                                                                                             : HOUGH_E_HIP;
}

int hough_prep(const hough_plan_t* p, const hough_hits_t* hits, uint32_t* phi_out, void* ws, size_t ws_bytes,
               hough_status_t* st, hipStream_t stream) {
    int rc = check_hits(p, hits);
    if (rc) return rc;
    if (!ws || !st) return HOUGH_E_INVAL;
    const WsLayout L = ws_layout(p, 0);
    if (ws_bytes < L.total) return HOUGH_E_SMALL_WS;
    launch_prep(p, single_event(p, hits->n), 1, hits->n, hits->x, hits->y, hits->layer, phi_out,
                static_cast<char*>(ws), ws_off(L), st, stream);
    return launch_status();
}

int hough_vote_prepared(const hough_plan_t* p, void* acc, void* ws, size_t ws_bytes, hough_status_t* st,
                        hipStream_t stream) {
    if (!p || !acc || !ws || !st) return HOUGH_E_INVAL;
    const WsLayout L = ws_layout(p, 0);
    if (ws_bytes < L.total) return HOUGH_E_SMALL_WS;
    launch_vote(p, single_event(p, 0), 1, static_cast<char*>(ws), ws_off(L), acc, 0, nullptr, nullptr,
                p->n_cols / kVoteCols, st, stream);
    return launch_status();
}

int hough_vote(const hough_plan_t* p, const hough_hits_t* hits, void* acc, void* ws, size_t ws_bytes,
               hough_status_t* st, hipStream_t stream) {
    if (!acc) return HOUGH_E_INVAL;
    int rc = hough_prep(p, hits, nullptr, ws, ws_bytes, st, stream);
    if (rc) return rc;
    return hough_vote_prepared(p, acc, ws, ws_bytes, st, stream);
}

int hough_peaks(const hough_plan_t* p, const void* acc, int32_t threshold, hough_peak_t* peaks, int32_t cap,
                void* ws, size_t ws_bytes, hough_status_t* st, hipStream_t stream) {
    if (!p || !acc || !peaks || !ws || !st || cap < 1 || threshold < 1) return HOUGH_E_INVAL;
    const WsLayout L = ws_layout(p, cap);
    if (ws_bytes < L.total) return HOUGH_E_SMALL_WS;
    launch_peaks(p, single_event(p, 0), 1, acc, 0, threshold, peaks, cap, static_cast<char*>(ws), ws_off(L), st,
                 stream);
    return launch_status();
}

int hough_assign(const hough_plan_t* p, const hough_peak_t* peaks, int32_t cap_peaks, int32_t* offsets,
                 int32_t* hit_idx, int32_t cap_pairs, void* ws, size_t ws_bytes, hough_status_t* st,
                 hipStream_t stream) {
    if (!p || !peaks || !offsets || !hit_idx || !ws || !st || cap_peaks < 1 || cap_pairs < 1) return HOUGH_E_INVAL;
    const WsLayout L = ws_layout(p, cap_peaks);
    if (ws_bytes < L.total) return HOUGH_E_SMALL_WS;
    launch_assign(p, single_event(p, 0), 1, peaks, cap_peaks, cap_peaks, offsets, hit_idx, cap_pairs,
                  static_cast<char*>(ws), ws_off(L), st, stream);
    return launch_status();
}

int hough_zvote(const hough_plan_t* p, const hough_hits_t* hits, const hough_peak_t* peaks, int32_t cap_peaks,
                const int32_t* offsets, const int32_t* hit_idx, int32_t cap_pairs, const hough_status_t* st,
                int32_t* out, hipStream_t stream) {
    if (!p || !hits || !peaks || !offsets || !hit_idx || !st || !out || cap_peaks < 1 || cap_pairs < 1)
        return HOUGH_E_INVAL;
    if (!p->zvote) return HOUGH_E_UNSUPPORTED;
    if (hits->n < 0 || hits->n > p->g.max_hits_per_event) return HOUGH_E_INVAL;
    if (hits->n > 0 && (!hits->z || !hits->layer)) return HOUGH_E_INVAL;
    launch_zvote(p, single_event(p, hits->n), 1, hits->z, hits->layer, peaks, cap_peaks, offsets, hit_idx, cap_pairs,
                 st, out, stream);
    return launch_status();
}

int hough_fit(const hough_plan_t* p, const hough_hits_t* hits, const int32_t* offsets, const int32_t* hit_idx,
              int32_t cap_peaks, int32_t cap_pairs, const hough_status_t* st, double* out, hipStream_t stream) {
    if (!p || !hits || !offsets || !hit_idx || !st || !out || cap_peaks < 1 || cap_pairs < 1) return HOUGH_E_INVAL;
    if (hits->n < 0 || hits->n > p->g.max_hits_per_event) return HOUGH_E_INVAL;
    if (hits->n > 0 && (!hits->x || !hits->y)) return HOUGH_E_INVAL;
    launch_fit(single_event(p, hits->n), 1, p->n_cu, hits->x, hits->y, offsets, hit_idx, cap_peaks, cap_pairs, st, out,
               stream);
    return launch_status();
}

// ---------------------------------------------------------------------- batches
size_t hough_batch_ws_bytes(const hough_plan_t* p, int32_t n_events, int32_t cap_peaks) {
    if (!p || n_events < 1) return 0;
    return batch_header_bytes(n_events) + (size_t)n_events * ws_layout(p, cap_peaks).total;
}

}  // extern "C"

namespace {

// The batched chain on the workspace `ws_base` of `ws_bytes` bytes (the caller's, or the scratch array).
int run_batch_on(const hough_plan_t* p, const hough_batch_t* b, void* ws_base, size_t ws_bytes,
                 hipStream_t stream) {
    if (b->n_events < 1 || b->cap_peaks < 1 || b->cap_pairs < 1 || b->threshold < 1) return HOUGH_E_INVAL;
    if (!b->hit_offsets || !b->x || !b->y || !b->layer || !b->acc || !b->peaks || !b->offsets || !b->hit_idx ||
        !ws_base || !b->status)
        return HOUGH_E_INVAL;
    if (b->zvote && (!p->zvote || !b->z)) return p->zvote ? HOUGH_E_INVAL : HOUGH_E_UNSUPPORTED;
    const WsLayout L = ws_layout(p, b->cap_peaks);
    const size_t hdr = batch_header_bytes(b->n_events);
    if (ws_bytes < hdr + (size_t)b->n_events * L.total) return HOUGH_E_SMALL_WS;
    char* ws = static_cast<char*>(ws_base);
    int32_t* queue = reinterpret_cast<int32_t*>(ws);
    int32_t* order = reinterpret_cast<int32_t*>(ws + 256);
    char* ev_ws = ws + hdr;
    const Events ev{b->hit_offsets, 0, p->g.max_hits_per_event, L.total};
    const WsOff O = ws_off(L);
    const int max_n = p->g.max_hits_per_event;  // per-event grids cover the plan's limit; extra blocks exit
    hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(1024), 0, stream, b->hit_offsets, b->n_events, queue, order);
    launch_prep(p, ev, b->n_events, max_n, b->x, b->y, b->layer, nullptr, ev_ws, O, b->status, stream);
    int grid = p->tuning.vote_grid;
    if (!p->pt) {
        if (grid <= 0) grid = 256;
        const int items = b->n_events * (p->n_cols / kVoteCols);
        if (grid > items) grid = items;
    }
    launch_vote(p, ev, b->n_events, ev_ws, O, b->acc, hough_acc_bytes(p), order, queue, grid, b->status, stream);
    launch_peaks(p, ev, b->n_events, b->acc, hough_acc_bytes(p), b->threshold, b->peaks, b->cap_peaks, ev_ws, O,
                 b->status, stream);
    launch_assign(p, ev, b->n_events, b->peaks, b->cap_peaks, b->cap_peaks, b->offsets, b->hit_idx, b->cap_pairs,
                  ev_ws, O, b->status, stream, order);
    if (b->zvote)
        launch_zvote(p, ev, b->n_events, b->z, b->layer, b->peaks, b->cap_peaks, b->offsets, b->hit_idx,
                     b->cap_pairs, b->status, b->zvote, stream);
    return launch_status();
}

}  // namespace

extern "C" {

int hough_run_batch(const hough_plan_t* p, const hough_batch_t* b, hipStream_t stream) {
    if (!p || !b) return HOUGH_E_INVAL;
    return run_batch_on(p, b, b->ws, b->ws_bytes, stream);
}

// The workspace of hough_run_batch_noalloc: a file-scope device array, one copy per GPU.  Host code
// never uses its name as an address: the device address of each GPU's copy is looked up once per
// device (noalloc_scratch_init, called by hough_plan_create with the plan's device current) and kept.
int hough_run_batch_noalloc(const hough_plan_t* p, const hough_batch_t* b, hipStream_t stream) {
    if (!p || !b) return HOUGH_E_INVAL;
    if (b->ws || b->ws_bytes) return HOUGH_E_INVAL;
    if (b->n_events < 1 || b->cap_peaks < 1) return HOUGH_E_INVAL;
    if (hough_batch_ws_bytes(p, b->n_events, b->cap_peaks) > (size_t)HOUGH_NOALLOC_SCRATCH_BYTES)
        return HOUGH_E_SMALL_WS;
    void* scratch_ptr = noalloc_scratch_get(p->device);
    if (!scratch_ptr) return HOUGH_E_HIP;
    return run_batch_on(p, b, scratch_ptr, (size_t)HOUGH_NOALLOC_SCRATCH_BYTES, stream);
}

struct hough_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

int hough_batch_graph_create(const hough_plan_t* p, const hough_batch_t* b, hipStream_t stream,
                             hough_graph_t** out) {
    if (!p || !b || !out || !stream) return HOUGH_E_INVAL;
    *out = nullptr;
    hough_graph* g = new (std::nothrow) hough_graph();
    if (!g) return HOUGH_E_NOMEM;
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        delete g;
        return HOUGH_E_HIP;
    }
    const int rc = hough_run_batch(p, b, stream);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(stream, &graph);
    if (rc != HOUGH_OK || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        return rc != HOUGH_OK ? rc : HOUGH_E_HIP;
    }
    if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return HOUGH_E_HIP;
    }
    g->graph = graph;
    *out = g;
    return HOUGH_OK;
}

int hough_graph_launch(hough_graph_t* g, hipStream_t stream) {
    if (!g) return HOUGH_E_INVAL;
    return hipGraphLaunch(g->exec, stream) == hipSuccess ? HOUGH_OK : HOUGH_E_HIP;
}

void hough_graph_destroy(hough_graph_t* g) {
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}


int hough_fit_batch(const hough_plan_t* p, const hough_batch_t* b, double* out, hipStream_t stream) {
    if (!p || !b || !out) return HOUGH_E_INVAL;
    if (b->n_events < 1 || b->n_events > 65535 || b->cap_peaks < 1 || b->cap_pairs < 1) return HOUGH_E_INVAL;
    if (!b->hit_offsets || !b->x || !b->y || !b->offsets || !b->hit_idx || !b->status) return HOUGH_E_INVAL;
    const Events ev{b->hit_offsets, 0, p->g.max_hits_per_event, 0};
    launch_fit(ev, b->n_events, p->n_cu, b->x, b->y, b->offsets, b->hit_idx, b->cap_peaks, b->cap_pairs, b->status,
               out, stream);
    return launch_status();
}

// ---------------------------------------------------------------------- per-hit radius
int hough_vote_cr(const hough_plan_t* p, const hough_hits_t* hits, int32_t* acc, hough_status_t* st,
                  hipStream_t stream) {
    int rc = check_hits(p, hits);
    if (rc) return rc;
    if (!acc || !st) return HOUGH_E_INVAL;
    if (p->g.acc_bits != 32) return HOUGH_E_UNSUPPORTED;
    CrGrid g{};
    g.n_layers = p->n_layers;
    g.n_qpt = p->g.n_qpt;
    g.n_cols = p->n_cols;
    g.n_phi = p->g.n_phi;
    g.M = p->M;
    g.F = p->F;
    g.qpt_min = p->g.qpt_min;
    g.qstep = (p->g.qpt_max - p->g.qpt_min) / (double)p->g.n_qpt;
    g.d0_min = p->g.d0_min;
    g.dstep = (p->g.d0_max - p->g.d0_min) / (double)p->g.n_d0;
    g.kappa = 0.299792458e-2 * p->B;
    const int64_t n_bins = p->n_bins;
    const unsigned iblocks = (unsigned)((n_bins / 4 + 255) / 256 + 1);
    hipLaunchKernelGGL(k_cr_init, dim3(iblocks), dim3(256), 0, stream, acc, n_bins, hits->n, st);
    const int chunks = (p->n_cols + kCrCols - 1) / kCrCols;
    const int64_t threads = (int64_t)hits->n * chunks;
    if (threads > 0) {
        const unsigned blocks = (unsigned)((threads + kCrThreads - 1) / kCrThreads);
        hipLaunchKernelGGL(k_vote_cr, dim3(blocks), dim3(kCrThreads), 0, stream, hits->x, hits->y, hits->layer,
                           hits->n, g, p->cordic, acc, st);
    }
    return launch_status();
}

int hough_refine(const hough_plan_t* p, const hough_peak_t* peaks, int32_t cap_peaks, const int32_t* offsets,
                 const int32_t* hit_idx, int32_t cap_pairs, const void* ws, size_t ws_bytes, const hough_status_t* st,
                 int32_t window, int32_t* out_hits, int32_t* out_layers, hipStream_t stream) {
    if (!p || !peaks || !offsets || !hit_idx || !ws || !st || !out_hits || !out_layers) return HOUGH_E_INVAL;
    if (cap_peaks < 1 || cap_pairs < 1 || window < 1 || window > (1 << p->F)) return HOUGH_E_INVAL;
    if (p->n_layers > 32 || p->F > 8) return HOUGH_E_UNSUPPORTED;
    const WsLayout L = ws_layout(p, cap_peaks);
    if (ws_bytes < L.total) return HOUGH_E_SMALL_WS;
    hipLaunchKernelGGL(k_refine, dim3((unsigned)((cap_peaks + kRefineThreads - 1) / kRefineThreads)),
                       dim3(kRefineThreads), 0, stream, peaks, cap_peaks, offsets, hit_idx, cap_pairs,
                       static_cast<const char*>(ws), ws_off(L), st, p->d_E, p->n_layers, p->n_cols, p->g.n_qpt, p->M,
                       p->F, window, out_hits, out_layers);
    return launch_status();
}

size_t hough_assign_cr_ws_bytes(const hough_plan_t* p, int32_t cap_peaks, int32_t cap_pairs) {
    if (!p || cap_peaks < 1 || cap_pairs < 1) return 0;
    return align_up(4 * (size_t)p->n_bins, 256) + align_up(4 * (size_t)cap_peaks, 256) +
           8 * ((size_t)cap_pairs + (size_t)p->g.max_hits_per_event);
}

int hough_assign_cr(const hough_plan_t* p, const hough_hits_t* hits, const hough_peak_t* peaks, int32_t cap_peaks,
                    int32_t* offsets, int32_t* hit_idx, int32_t cap_pairs, void* ws, size_t ws_bytes, void* ws_cr,
                    size_t ws_cr_bytes, hough_status_t* st, hipStream_t stream) {
    int rc = check_hits(p, hits);
    if (rc) return rc;
    if (!peaks || !offsets || !hit_idx || !ws || !ws_cr || !st || cap_peaks < 1 || cap_pairs < 1)
        return HOUGH_E_INVAL;
    if (p->g.acc_bits != 32) return HOUGH_E_UNSUPPORTED;
    const WsLayout L = ws_layout(p, cap_peaks);
    if (ws_bytes < L.total || ws_cr_bytes < hough_assign_cr_ws_bytes(p, cap_peaks, cap_pairs)) return HOUGH_E_SMALL_WS;
    const WsOff O = ws_off(L);
    char* w = static_cast<char*>(ws_cr);
    int32_t* map = reinterpret_cast<int32_t*>(w);
    int32_t* fill = reinterpret_cast<int32_t*>(w + align_up(4 * (size_t)p->n_bins, 256));
    uint64_t* keys = reinterpret_cast<uint64_t*>(w + align_up(4 * (size_t)p->n_bins, 256) +
                                                 align_up(4 * (size_t)cap_peaks, 256));
    CrGrid g{};
    g.n_layers = p->n_layers;
    g.n_qpt = p->g.n_qpt;
    g.n_cols = p->n_cols;
    g.n_phi = p->g.n_phi;
    g.M = p->M;
    g.F = p->F;
    g.qpt_min = p->g.qpt_min;
    g.qstep = (p->g.qpt_max - p->g.qpt_min) / (double)p->g.n_qpt;
    g.d0_min = p->g.d0_min;
    g.dstep = (p->g.d0_max - p->g.d0_min) / (double)p->g.n_d0;
    g.kappa = 0.299792458e-2 * p->B;
    const int64_t n_init = p->n_bins > cap_peaks ? p->n_bins : cap_peaks;
    hipLaunchKernelGGL(k_cra_init, dim3((unsigned)((n_init + 255) / 256)), dim3(256), 0, stream, map, p->n_bins, fill,
                       cap_peaks);
    hipLaunchKernelGGL(k_cra_map, dim3((unsigned)((cap_peaks + 255) / 256)), dim3(256), 0, stream, peaks, cap_peaks,
                       static_cast<const char*>(ws), O, p->g.n_qpt, p->g.n_phi, map);
    const int chunks = (p->n_cols + kCrCols - 1) / kCrCols;
    const int64_t threads = (int64_t)hits->n * chunks;
    if (threads > 0)
        hipLaunchKernelGGL(k_cra_vote, dim3((unsigned)((threads + kCrThreads - 1) / kCrThreads)), dim3(kCrThreads), 0,
                           stream, hits->x, hits->y, hits->layer, hits->n, g, p->cordic, map,
                           at<const int64_t>(static_cast<char*>(ws), O.peak_voff), fill, keys, cap_pairs);
    hipLaunchKernelGGL(k_cra_sort, dim3((unsigned)((cap_peaks + 255) / 256)), dim3(256), 0, stream, peaks, cap_peaks,
                       static_cast<const char*>(ws), O, keys, offsets, hit_idx, cap_pairs, st);
    return launch_status();
}

// ---------------------------------------------------------------------- second transform
int hough_vertex_plan_create(const hough_plan_t* p, const hough_vertex_grid_t* vgrid, hough_vertex_plan_t** out) {
    if (!p || !vgrid || !out) return HOUGH_E_INVAL;
    *out = nullptr;
    const hough_vertex_grid_t& v = *vgrid;
    if (v.min_votes < 1 || !std::isfinite(v.r_min) || !std::isfinite(v.r_max) || !(v.r_min >= 0.0) ||
        !(v.r_max > v.r_min))
        return HOUGH_E_INVAL;
    if (v.r_max > 32768.0) return HOUGH_E_UNSUPPORTED;
    if (v.n_vr < 64 || v.n_vr % 64 || v.n_vr > 4096) return HOUGH_E_UNSUPPORTED;
    const int lv = ilog2_exact(v.n_vphi);
    if (lv < 4 || v.n_vphi > 1024 || lv > p->M) return HOUGH_E_UNSUPPORTED;
    if ((int64_t)p->g.n_d0 * p->g.n_qpt * v.n_vr > ((int64_t)1 << 31)) return HOUGH_E_UNSUPPORTED;

    hough_vertex_plan* vp = new (std::nothrow) hough_vertex_plan();
    if (!vp) return HOUGH_E_NOMEM;
    vp->first = p;
    vp->vg = v;
    vp->slabs = v.n_vr / 64;
    // workgroups resident per CU: LDS of one slab, at most 32 waves
    int per_cu = (int)((size_t)kLdsBytes / ((size_t)v.n_vphi * 128));
    const int by_waves = 32 / (kVvoteThreads / 64);
    per_cu = per_cu < by_waves ? per_cu : by_waves;
    per_cu = per_cu > 1 ? per_cu : 1;
    vp->groups = (p->n_cu * per_cu + vp->slabs - 1) / vp->slabs;

    // the vertex space's own grid, for its peak finder (threshold and tie rule of the first stage)
    const double r1 = 1.0;
    hough_geometry_t geo{1, &r1, nullptr, 0.0};
    hough_grid_t gg{};
    gg.n_phi = v.n_vphi;
    gg.n_qpt = v.n_vr;
    gg.n_d0 = 1;
    gg.frac_bits = 7;
    gg.acc_bits = 32;
    gg.max_hits_per_event = 1;
    int rc = hough_plan_create(&geo, &gg, &vp->grid);
    if (rc) {
        delete vp;
        return rc;
    }
    vp->grid->tuning = p->tuning;
    vp->grid->stage = false;  // vertex-space bins count candidates, which may exceed 16 bits

    // sample table at the row radii, in IEEE double in the operation order of the first table
    const hough_grid_t& g = p->g;
    const size_t ntab = (size_t)g.n_d0 * g.n_qpt * v.n_vr;
    int32_t* T = (int32_t*)malloc(ntab * sizeof(int32_t));
    if (!T) {
        hough_plan_destroy(vp->grid);
        delete vp;
        return HOUGH_E_NOMEM;
    }
    const double kappa = 0.299792458e-2 * p->B;
    const double K = ldexp(1.0, p->M - 1) / M_PI;
    for (int l = 0; l < g.n_d0; ++l) {
        const double d = g.d0_min + ((double)l + 0.5) * ((g.d0_max - g.d0_min) / (double)g.n_d0);
        for (int k = 0; k < g.n_qpt; ++k) {
            const double q = g.qpt_min + ((double)k + 0.5) * ((g.qpt_max - g.qpt_min) / (double)g.n_qpt);
            const double c = -kappa * q;
            for (int j = 0; j < v.n_vr; ++j) {
                const double r = v.r_min + ((double)j + 0.5) * ((v.r_max - v.r_min) / (double)v.n_vr);
                const double num = c * (r * r + d * d) + 2.0 * d;
                const double den = 2.0 * r * (1.0 + c * d);
                int32_t e = INT32_MIN;
                if (den > 0.0) {
                    const double A = num / den;
                    if (fabs(A) <= 1.0) e = (int32_t)llrint(asin(A) * K);
                }
                T[((size_t)l * g.n_qpt + k) * v.n_vr + j] = e;
            }
        }
    }
    hipError_t e = hipMalloc(&vp->d_T, ntab * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpy(vp->d_T, T, ntab * sizeof(int32_t), hipMemcpyHostToDevice);
    free(T);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_vvote, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) {
        if (vp->d_T) (void)hipFree(vp->d_T);
        hough_plan_destroy(vp->grid);
        delete vp;
        return e == hipErrorOutOfMemory ? HOUGH_E_NOMEM : HOUGH_E_HIP;
    }
    *out = vp;
    return HOUGH_OK;
}

void hough_vertex_plan_destroy(hough_vertex_plan_t* vp) {
    if (!vp) return;
    if (vp->d_T) (void)hipFree(vp->d_T);
    hough_plan_destroy(vp->grid);
    delete vp;
}

int hough_vertex_set_groups(hough_vertex_plan_t* vp, int32_t groups) {
    if (!vp || groups < 1 || groups > 65536) return HOUGH_E_INVAL;
    vp->groups = groups;
    return HOUGH_OK;
}

int32_t hough_vertex_get_groups(const hough_vertex_plan_t* vp) { return vp ? vp->groups : -1; }

size_t hough_vertex_vote_ws_bytes(const hough_vertex_plan_t* vp, int32_t cap_peaks) {
    if (!vp || cap_peaks < 1) return 0;
    return vertex_partial_bytes(vp, cap_peaks);
}

size_t hough_vertex_peaks_ws_bytes(const hough_vertex_plan_t* vp, int32_t cap_vpeaks) {
    if (!vp || cap_vpeaks < 1) return 0;
    return ws_layout(vp->grid, cap_vpeaks).total;
}

int hough_vertex_table(const hough_vertex_plan_t* vp, int32_t* out) {
    if (!vp || !out) return HOUGH_E_INVAL;
    const size_t n = (size_t)vp->first->g.n_d0 * vp->first->g.n_qpt * vp->vg.n_vr;
    return hipMemcpy(out, vp->d_T, n * sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess ? HOUGH_OK
                                                                                              : HOUGH_E_HIP;
}

int hough_vertex_vote(const hough_vertex_plan_t* vp, const hough_peak_t* peaks, int32_t cap_peaks,
                      const hough_status_t* st, int32_t* acc_v, void* ws, size_t ws_bytes, hough_status_t* st_v,
                      hipStream_t stream) {
    if (!vp || !peaks || !st || !acc_v || !ws || !st_v || cap_peaks < 1) return HOUGH_E_INVAL;
    if (ws_bytes < vertex_partial_bytes(vp, cap_peaks)) return HOUGH_E_SMALL_WS;
    launch_vertex_vote(vertex_vgrid(vp, cap_peaks), vp->slabs, 1, peaks, cap_peaks, st, vp->d_T,
                       static_cast<uint32_t*>(ws), acc_v, st_v, stream);
    return launch_status();
}

size_t hough_vertex_batch_vote_ws_bytes(const hough_vertex_plan_t* vp, int32_t n_events, int32_t cap_peaks) {
    if (!vp || n_events < 1 || cap_peaks < 1) return 0;
    return vertex_partial_bytes(vp, cap_peaks, n_events);
}

size_t hough_vertex_batch_peaks_ws_bytes(const hough_vertex_plan_t* vp, int32_t n_events, int32_t cap_vpeaks) {
    if (!vp || n_events < 1 || cap_vpeaks < 1) return 0;
    return (size_t)n_events * ws_layout(vp->grid, cap_vpeaks).total;
}

int hough_vertex_vote_batch(const hough_vertex_plan_t* vp, int32_t n_events, const hough_peak_t* peaks,
                            int32_t cap_peaks, const hough_status_t* st, int32_t* acc_v, void* ws, size_t ws_bytes,
                            hough_status_t* st_v, hipStream_t stream) {
    if (!vp || !peaks || !st || !acc_v || !ws || !st_v || cap_peaks < 1 || n_events < 1 || n_events > 65535)
        return HOUGH_E_INVAL;
    if (ws_bytes < vertex_partial_bytes(vp, cap_peaks, n_events)) return HOUGH_E_SMALL_WS;
    launch_vertex_vote(vertex_vgrid(vp, cap_peaks, n_events), vp->slabs, n_events, peaks, cap_peaks, st, vp->d_T,
                       static_cast<uint32_t*>(ws), acc_v, st_v, stream);
    return launch_status();
}

int hough_vertex_peaks_batch(const hough_vertex_plan_t* vp, int32_t n_events, const int32_t* acc_v,
                             int32_t threshold, hough_peak_t* vpeaks, int32_t cap, void* ws, size_t ws_bytes,
                             hough_status_t* st_v, hipStream_t stream) {
    if (!vp || !acc_v || !vpeaks || !ws || !st_v || cap < 1 || threshold < 1 || n_events < 1 || n_events > 65535)
        return HOUGH_E_INVAL;
    const WsLayout L = ws_layout(vp->grid, cap);
    if (ws_bytes < (size_t)n_events * L.total) return HOUGH_E_SMALL_WS;
    const Events ev{nullptr, 0, 1, L.total};
    launch_peaks(vp->grid, ev, n_events, acc_v, (size_t)vp->vg.n_vr * vp->vg.n_vphi * 4, threshold, vpeaks, cap,
                 static_cast<char*>(ws), ws_off(L), st_v, stream);
    return launch_status();
}

int hough_vertex_peaks(const hough_vertex_plan_t* vp, const int32_t* acc_v, int32_t threshold, hough_peak_t* vpeaks,
                       int32_t cap, void* ws, size_t ws_bytes, hough_status_t* st_v, hipStream_t stream) {
    if (!vp) return HOUGH_E_INVAL;
    return hough_peaks(vp->grid, acc_v, threshold, vpeaks, cap, ws, ws_bytes, st_v, stream);
}

}  // extern "C"
