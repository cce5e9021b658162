// hough.hip -- gfx950 kernels and C ABI of the Hough-transform track finder.
//
// The operations (prep, vote, peaks, assign) and their exact integer
// definitions are documented in include/hough.h.  This file is the MI355X
// implementation:
//   prep    per-hit Q16.16 + integer CORDIC azimuth, then a counting sort of
//           the valid hits by (layer, azimuth cell) so that the vote reads
//           each layer's hits as one contiguous run and the assignment can
//           answer "which hits of layer L lie in this phi0 window" by cells;
//   vote    one workgroup per slab of 64 (l, k) columns holds the whole phi0
//           range of its columns in LDS as [bin][column] (one 256-byte row per
//           bin), loops over all hits of the event layer by layer and adds
//           each vote with a conflict-free ds_add_u32: one lane per column,
//           one hit per instruction, 2 VALU ops + 1 LDS atomic per vote; the
//           slab is then written once to HBM (no global atomics, slabs are
//           disjoint, integer sums are order independent);
//   peaks   one thread per 8-bin strip of a column walks an l range keeping
//           a 3-plane window in registers (separable 3-wide maxima), writes
//           one flag byte per strip and per-group counts; a scan and a write
//           pass compact the candidates in increasing linear index;
//   assign  the CSR offsets are the prefix sums of the candidates' vote
//           counts; each candidate gathers its hits from the cells its phi0
//           window covers, layer by layer, and sorts them by hit index.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>

#include "hough.h"

namespace {

constexpr int kMaxLayers = 32;
constexpr int kCordicSteps = 30;
constexpr int kVoteThreads = 1024;
constexpr int kVoteCols = 64;       // columns per vote slab (one per lane)
constexpr int kStrip = 8;           // phi0 bins per peak-finder thread
constexpr int kPeakPlanes = 8;      // d0 planes per peak-finder thread
constexpr int kScanThreads = 1024;
constexpr int kAssignBlock = 256;

struct CordicTable {
    int32_t t[kCordicSteps];
};

struct LayerTable {
    int32_t valid_cols[kMaxLayers];  // number of (l, k) columns whose sample is valid, per layer
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
    int32_t* d_E;    // [n_layers][n_d0][n_qpt], INT32_MIN = invalid
};

namespace {

// ------------------------------------------------------------------ layout
struct WsLayout {
    size_t phi32, lay, cell_count, cell_start, cell_cursor, sorted_phi, sorted_h;
    size_t flags, grp_count, grp_off, blk_sum, blk_off, misc, total;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int peak_group_lanes(const hough_plan* p) {
    int strips = p->g.n_phi / kStrip;
    return strips < 64 ? strips : 64;
}

int64_t peak_groups(const hough_plan* p) {
    return p->n_bins / ((int64_t)kStrip * peak_group_lanes(p));
}

WsLayout ws_layout(const hough_plan* p, int32_t max_peaks) {
    WsLayout L{};
    size_t o = 0;
    const size_t maxh = (size_t)p->g.max_hits_per_event;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.phi32 = take(4 * maxh);
    L.lay = take(maxh);
    L.cell_count = take(4 * ((size_t)p->n_cells + 1));
    L.cell_start = take(4 * ((size_t)p->n_cells + 1));
    L.cell_cursor = take(4 * ((size_t)p->n_cells + 1));
    L.sorted_phi = take(4 * maxh);
    L.sorted_h = take(4 * maxh);
    L.flags = take((size_t)(p->n_bins / kStrip));
    L.grp_count = take(4 * (size_t)(peak_groups(p) + 1));
    L.grp_off = take(4 * (size_t)(peak_groups(p) + 1));
    size_t nblk = (size_t)(max_peaks > 0 ? max_peaks : 1) / kAssignBlock + 2;
    L.blk_sum = take(8 * nblk);
    L.blk_off = take(8 * nblk);
    L.misc = take(256);
    L.total = o;
    return L;
}

template <typename T>
T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

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

__device__ __forceinline__ int32_t wave_sum(int32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// exclusive scan of n int32 counts by one workgroup of kScanThreads threads
__device__ int64_t block_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int64_t* sums) {
    __shared__ int64_t part[kScanThreads];
    const int tid = threadIdx.x;
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t lo = per * tid, hi = lo + per < n ? lo + per : n;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += in[i];
    part[tid] = s;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        int64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - s;
    for (int64_t i = lo; i < hi; ++i) {
        int32_t c = in[i];
        if (out) out[i] = (int32_t)run;
        if (sums) sums[i] = run;
        run += c;
    }
    int64_t total = part[kScanThreads - 1];
    __syncthreads();
    return total;
}

// ------------------------------------------------------------------ prep kernels
__global__ void k_prep_init(int32_t* cell_count, int n_cells, hough_status_t* st, int32_t n_hits) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (; i <= n_cells; i += gridDim.x * blockDim.x) cell_count[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_hits = n_hits;
        st->n_bad_hits = 0;
        st->n_votes = 0;
        st->n_peaks = 0;
        st->flags = 0;
        st->n_pairs = 0;
    }
}

__global__ __launch_bounds__(256) void k_prep_hits(const float* __restrict__ hx, const float* __restrict__ hy,
                                                   const uint8_t* __restrict__ hl, int32_t n, int n_layers,
                                                   int cell_bits, CordicTable T, uint32_t* __restrict__ phi32,
                                                   uint8_t* __restrict__ lay, uint32_t* __restrict__ phi_out,
                                                   int32_t* __restrict__ cell_count, hough_status_t* st) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = false;
    uint32_t phi = 0;
    uint8_t L = 0xFF;
    if (h < n) {
        const float x = hx[h], y = hy[h];
        L = hl[h];
        ok = (int)L < n_layers && isfinite(x) && isfinite(y) && fabsf(x) < 32768.0f && fabsf(y) < 32768.0f;
        if (ok) {
            // x * 2^16 is exact in float; round half to even
            const int32_t X = __float2int_rn(x * 65536.0f);
            const int32_t Y = __float2int_rn(y * 65536.0f);
            ok = !(X == 0 && Y == 0);
            if (ok) phi = cordic_azimuth(X, Y, T);
        }
        phi32[h] = phi;
        lay[h] = ok ? L : (uint8_t)0xFF;
        if (phi_out) phi_out[h] = phi;
        if (ok) atomicAdd(&cell_count[((int)L << cell_bits) | (int)(phi >> (32 - cell_bits))], 1);
    }
    const uint64_t bad = __ballot(h < n && !ok);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(&st->n_bad_hits, (int32_t)__popcll(bad));
}

__global__ __launch_bounds__(kScanThreads) void k_prep_scan(const int32_t* __restrict__ cell_count,
                                                            int32_t* __restrict__ cell_start,
                                                            int32_t* __restrict__ cell_cursor, int n_cells,
                                                            int n_layers, int cell_bits, LayerTable LT,
                                                            hough_status_t* st) {
    int64_t total = block_exclusive_scan(cell_count, cell_start, n_cells, nullptr);
    for (int i = threadIdx.x; i < n_cells; i += blockDim.x) cell_cursor[i] = cell_start[i];
    if (threadIdx.x == 0) cell_start[n_cells] = (int32_t)total;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t votes = 0;
        for (int L = 0; L < n_layers; ++L) {
            const int lo = cell_start[L << cell_bits];
            const int hi = (L + 1 == n_layers) ? (int32_t)total : cell_start[(L + 1) << cell_bits];
            votes += (int64_t)(hi - lo) * LT.valid_cols[L];
        }
        st->n_votes = votes;
    }
}

__global__ __launch_bounds__(256) void k_prep_scatter(const uint32_t* __restrict__ phi32,
                                                      const uint8_t* __restrict__ lay, int32_t n, int cell_bits,
                                                      int M, int32_t* __restrict__ cell_cursor,
                                                      uint32_t* __restrict__ sorted_phi,
                                                      int32_t* __restrict__ sorted_h) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n) return;
    const uint8_t L = lay[h];
    if (L == 0xFF) return;
    const uint32_t phi = phi32[h];
    const int pos = atomicAdd(&cell_cursor[((int)L << cell_bits) | (int)(phi >> (32 - cell_bits))], 1);
    sorted_phi[pos] = phi >> (32 - M);
    sorted_h[pos] = h;
}

// ------------------------------------------------------------------ vote
__device__ __forceinline__ void lds_vote(uint32_t phi, uint32_t e, uint32_t mask, uint32_t lanebits,
                                         uint32_t data) {
    const uint32_t t = phi - e;
    uint32_t a;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(a) : "v"(t), "s"(mask), "v"(lanebits));
    asm volatile("ds_add_u32 %0, %1" ::"v"(a), "v"(data) : "memory");
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

// ACC16 = false: slab dword (b * 64 + c), one int32 counter per (bin, column), F = 8.
// ACC16 = true : slab dword (b * 32 + c % 32), 16-bit halves for columns c and c + 32, F = 7.
template <bool ACC16>
__global__ __launch_bounds__(kVoteThreads) void k_vote(const int32_t* __restrict__ E,
                                                       const int32_t* __restrict__ cell_start,
                                                       const uint32_t* __restrict__ sorted_phi, int n_layers,
                                                       int cell_bits, int n_cols, int n_phi, int F,
                                                       void* __restrict__ acc_out, hough_status_t* st) {
    extern __shared__ uint32_t slab[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_waves = kVoteThreads / 64;
    const int col = blockIdx.x * kVoteCols + lane;
    const int slab_dwords = ACC16 ? n_phi * 32 : n_phi * 64;

    // The vote addresses LDS by byte offset from 0: the slab must be the only LDS allocation.
    const uint32_t lds_base = (uint32_t)(uintptr_t)(lds_u32*)slab;
    if (lds_base != 0) {
        if (tid == 0 && blockIdx.x == 0) atomicOr(&st->flags, 0x40000000);
        return;
    }

    uint4* s4 = reinterpret_cast<uint4*>(slab);
    for (int i = tid; i < slab_dwords / 4; i += kVoteThreads) s4[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();

    const uint32_t mask = (uint32_t)(n_phi - 1) << F;
    const uint32_t lanebits = ACC16 ? (uint32_t)(lane & 31) << 2 : (uint32_t)lane << 2;
    const uint32_t data = ACC16 ? (lane >= 32 ? 0x10000u : 1u) : 1u;

    // The hits of each layer are cut into chunks of 64; chunk g (counted over all layers) goes to
    // wave g % n_waves.  A wave loads a chunk with one coalesced load (one hit per lane) and then
    // broadcasts hit j with v_readlane: the hit values travel in VGPRs, so waiting for them never
    // waits for the LDS atomics (scalar loads would share the LDS wait counter).
    int chunk_base = 0;
    for (int L = 0; L < n_layers; ++L) {
        const int lo = cell_start[L << cell_bits];
        const int hi = cell_start[(L + 1) << cell_bits];
        const int n_chunks = (hi - lo + 63) >> 6;
        const int first = (wave - chunk_base % n_waves + n_waves) % n_waves;
        chunk_base += n_chunks;
        if (first >= n_chunks) continue;
        const int32_t e = E[(size_t)L * n_cols + col];
        const bool valid = e != INT32_MIN;
        const uint32_t ue = (uint32_t)e;
        int c = first;
        int h = lo + (c << 6);
        uint32_t cur = h + lane < hi ? sorted_phi[h + lane] : 0u;
        for (; c < n_chunks; c += n_waves) {
            h = lo + (c << 6);
            const int hn = h + (n_waves << 6);
            const uint32_t nxt = hn + lane < hi ? sorted_phi[hn + lane] : 0u;  // prefetch the next chunk
            const int cnt = min(64, hi - h);
            if (valid) {
                if (cnt == 64) {
#pragma unroll
                    for (int j = 0; j < 64; ++j)
                        lds_vote((uint32_t)__builtin_amdgcn_readlane((int)cur, j), ue, mask, lanebits, data);
                } else {
                    for (int j = 0; j < cnt; ++j)
                        lds_vote((uint32_t)__builtin_amdgcn_readlane((int)cur, j), ue, mask, lanebits, data);
                }
            }
            cur = nxt;
        }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __syncthreads();

    // store the slab: acc[col][b], b fastest
    const int col0 = blockIdx.x * kVoteCols;
    if (!ACC16) {
        int32_t* acc = static_cast<int32_t*>(acc_out);
        const int quads = n_phi / 4;
        for (int i = tid; i < quads * kVoteCols; i += kVoteThreads) {
            const int c = i & 63, q = i >> 6;
            uint4 v;
            v.x = slab[(4 * q + 0) * 64 + c];
            v.y = slab[(4 * q + 1) * 64 + c];
            v.z = slab[(4 * q + 2) * 64 + c];
            v.w = slab[(4 * q + 3) * 64 + c];
            *reinterpret_cast<uint4*>(acc + (size_t)(col0 + c) * n_phi + 4 * q) = v;
        }
    } else {
        int16_t* acc = static_cast<int16_t*>(acc_out);
        const int octs = n_phi / 8;
        for (int i = tid; i < octs * kVoteCols; i += kVoteThreads) {
            const int c = i & 63, q = i >> 6;
            const int sh = c >= 32 ? 16 : 0;
            uint32_t w[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) w[j] = (slab[(8 * q + j) * 32 + (c & 31)] >> sh) & 0xFFFFu;
            uint4 v;
            v.x = w[0] | (w[1] << 16);
            v.y = w[2] | (w[3] << 16);
            v.z = w[4] | (w[5] << 16);
            v.w = w[6] | (w[7] << 16);
            *reinterpret_cast<uint4*>(acc + (size_t)(col0 + c) * n_phi + 8 * q) = v;
        }
    }
}

// ------------------------------------------------------------------ peaks
template <typename T>
__device__ __forceinline__ void load_strip(const T* __restrict__ acc, int l, int k, int s, int n_d0, int n_qpt,
                                           int n_phi, int32_t v[kStrip + 2]) {
    if (l < 0 || l >= n_d0 || k < 0 || k >= n_qpt) {
#pragma unroll
        for (int i = 0; i < kStrip + 2; ++i) v[i] = INT32_MIN;
        return;
    }
    const T* row = acc + ((size_t)l * n_qpt + k) * n_phi;
    const int b0 = s * kStrip;
    if (sizeof(T) == 4) {
        const uint4 a = *reinterpret_cast<const uint4*>(row + b0);
        const uint4 c = *reinterpret_cast<const uint4*>(row + b0 + 4);
        v[1] = (int32_t)a.x; v[2] = (int32_t)a.y; v[3] = (int32_t)a.z; v[4] = (int32_t)a.w;
        v[5] = (int32_t)c.x; v[6] = (int32_t)c.y; v[7] = (int32_t)c.z; v[8] = (int32_t)c.w;
    } else {
        const uint4 a = *reinterpret_cast<const uint4*>(row + b0);
        v[1] = (int16_t)(a.x & 0xFFFF); v[2] = (int16_t)(a.x >> 16);
        v[3] = (int16_t)(a.y & 0xFFFF); v[4] = (int16_t)(a.y >> 16);
        v[5] = (int16_t)(a.z & 0xFFFF); v[6] = (int16_t)(a.z >> 16);
        v[7] = (int16_t)(a.w & 0xFFFF); v[8] = (int16_t)(a.w >> 16);
    }
    v[0] = (int32_t)row[(b0 - 1) & (n_phi - 1)];
    v[kStrip + 1] = (int32_t)row[(b0 + kStrip) & (n_phi - 1)];
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

template <typename T>
__device__ __forceinline__ void load_plane(const T* __restrict__ acc, int l, int k, int s, int n_d0, int n_qpt,
                                           int n_phi, PlaneWin& w) {
    int32_t a[kStrip + 2], c[kStrip + 2], m0[kStrip];
    load_strip(acc, l, k - 1, s, n_d0, n_qpt, n_phi, a);
    load_strip(acc, l, k, s, n_d0, n_qpt, n_phi, w.mid);
    load_strip(acc, l, k + 1, s, n_d0, n_qpt, n_phi, c);
    max3(a, w.lo);
    max3(w.mid, m0);
    max3(c, w.hi);
#pragma unroll
    for (int i = 0; i < kStrip; ++i) w.all[i] = max(max(w.lo[i], m0[i]), w.hi[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_peaks_mark(const T* __restrict__ acc, int32_t thr, int n_d0, int n_qpt,
                                                    int n_phi, int group_lanes, uint8_t* __restrict__ flags,
                                                    int32_t* __restrict__ grp_count) {
    const int strips = n_phi / kStrip;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = (int)(t % strips);
    const int k = (int)((t / strips) % n_qpt);
    const int lr = (int)(t / ((int64_t)strips * n_qpt));
    const int l0 = lr * kPeakPlanes;
    if (l0 >= n_d0) return;  // whole groups exit together (groups never straddle planes)
    const int l1 = min(n_d0, l0 + kPeakPlanes);
    PlaneWin prev, cur, next;
    load_plane(acc, l0 - 1, k, s, n_d0, n_qpt, n_phi, prev);
    load_plane(acc, l0, k, s, n_d0, n_qpt, n_phi, cur);
    for (int l = l0; l < l1; ++l) {
        load_plane(acc, l + 1, k, s, n_d0, n_qpt, n_phi, next);
        uint32_t bits = 0;
#pragma unroll
        for (int i = 0; i < kStrip; ++i) {
            const int32_t v = cur.mid[i + 1];
            // neighbours that precede (l-1 plane, column k-1 of this plane, bin b-1) must be < v,
            // neighbours that follow must be <= v
            const int32_t P = max(max(prev.all[i], cur.lo[i]), cur.mid[i]);
            const int32_t Q = max(max(next.all[i], cur.hi[i]), cur.mid[i + 2]);
            if (v >= thr && v > P && v >= Q) bits |= 1u << i;
        }
        const int64_t strip_id = ((int64_t)l * n_qpt + k) * strips + s;
        flags[strip_id] = (uint8_t)bits;
        // per-group counts: a group is `group_lanes` consecutive strips of one column
        int32_t cnt = __popc(bits);
        for (int o = group_lanes >> 1; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if ((threadIdx.x & (group_lanes - 1)) == 0) grp_count[strip_id / group_lanes] = cnt;
        prev = cur;
        cur = next;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_peaks_scan(const int32_t* __restrict__ grp_count,
                                                             int32_t* __restrict__ grp_off, int64_t n_groups,
                                                             int32_t cap, hough_status_t* st) {
    int64_t total = block_exclusive_scan(grp_count, grp_off, n_groups, nullptr);
    if (threadIdx.x == 0) {
        grp_off[n_groups] = (int32_t)min(total, (int64_t)INT32_MAX);
        st->n_peaks = (int32_t)min(total, (int64_t)INT32_MAX);
        if (total > cap) atomicOr(&st->flags, HOUGH_F_PEAK_OVERFLOW);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_peaks_write(const T* __restrict__ acc, const uint8_t* __restrict__ flags,
                                                     const int32_t* __restrict__ grp_off, int n_qpt, int n_phi,
                                                     int group_lanes, int64_t n_strips, hough_peak_t* peaks,
                                                     int32_t cap) {
    const int strips = n_phi / kStrip;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t bits = t < n_strips ? flags[t] : 0u;
    // exclusive prefix of the popcounts within the group
    const int gl = threadIdx.x & (group_lanes - 1);
    int32_t inc = __popc(bits);
    for (int o = 1; o < group_lanes; o <<= 1) {
        const int32_t v = __shfl_up(inc, o, group_lanes);
        if (gl >= o) inc += v;
    }
    if (t >= n_strips || bits == 0) return;
    int32_t pos = grp_off[t / group_lanes] + inc - __popc(bits);
    const int s = (int)(t % strips);
    const int64_t row = t / strips;
    const int k = (int)(row % n_qpt);
    const int l = (int)(row / n_qpt);
    const T* r = acc + row * n_phi;
    for (int i = 0; i < kStrip; ++i) {
        if (!(bits & (1u << i))) continue;
        if (pos < cap) {
            const int b = s * kStrip + i;
            hough_peak_t pk;
            pk.l = l;
            pk.k = k;
            pk.b = b;
            pk.votes = (int32_t)r[b];
            peaks[pos] = pk;
        }
        ++pos;
    }
}

// ------------------------------------------------------------------ assign
__global__ __launch_bounds__(kAssignBlock) void k_assign_blocksum(const hough_peak_t* __restrict__ peaks,
                                                                  int32_t cap_peaks, const hough_status_t* st,
                                                                  int64_t* __restrict__ blk_sum) {
    const int n = min(st->n_peaks, cap_peaks);
    const int i = blockIdx.x * kAssignBlock + threadIdx.x;
    if ((int)blockIdx.x * kAssignBlock >= n) return;
    int32_t v = i < n ? peaks[i].votes : 0;
    __shared__ int32_t red[kAssignBlock / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int w = 0; w < kAssignBlock / 64; ++w) s += red[w];
        blk_sum[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_assign_topscan(const int64_t* __restrict__ blk_sum,
                                                                 int64_t* __restrict__ blk_off, int32_t cap_peaks,
                                                                 int32_t* offsets, int32_t cap_pairs,
                                                                 hough_status_t* st) {
    const int n = min(st->n_peaks, cap_peaks);
    const int nblk = (n + kAssignBlock - 1) / kAssignBlock;
    __shared__ int64_t part[kScanThreads];
    const int tid = threadIdx.x;
    const int per = (nblk + kScanThreads - 1) / kScanThreads;
    const int lo = per * tid, hi = min(nblk, lo + per);
    int64_t s = 0;
    for (int i = lo; i < hi; ++i) s += blk_sum[i];
    part[tid] = s;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        int64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - s;
    for (int i = lo; i < hi; ++i) {
        blk_off[i] = run;
        run += blk_sum[i];
    }
    if (tid == 0) {
        const int64_t total = part[kScanThreads - 1];
        st->n_pairs = total;
        offsets[n] = (int32_t)min(total, (int64_t)INT32_MAX);
        if (total > cap_pairs) atomicOr(&st->flags, HOUGH_F_PAIR_OVERFLOW);
    }
}

__global__ __launch_bounds__(kAssignBlock) void k_assign_fill(
    const hough_peak_t* __restrict__ peaks, int32_t cap_peaks, const hough_status_t* st,
    const int64_t* __restrict__ blk_off, const int32_t* __restrict__ E, const int32_t* __restrict__ cell_start,
    const uint32_t* __restrict__ sorted_phi, const int32_t* __restrict__ sorted_h, int n_layers, int cell_bits,
    int n_cols, int n_qpt, int M, int F, int32_t* __restrict__ offsets, int32_t* __restrict__ hit_idx,
    int32_t cap_pairs) {
    const int n = min(st->n_peaks, cap_peaks);
    if ((int)blockIdx.x * kAssignBlock >= n) return;
    const int i = blockIdx.x * kAssignBlock + threadIdx.x;
    const int32_t votes = i < n ? peaks[i].votes : 0;
    // block-local exclusive scan of the vote counts
    __shared__ int32_t sc[kAssignBlock];
    sc[threadIdx.x] = votes;
    __syncthreads();
    for (int d = 1; d < kAssignBlock; d <<= 1) {
        int32_t v = threadIdx.x >= d ? sc[threadIdx.x - d] : 0;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    if (i >= n) return;
    const int64_t off = blk_off[blockIdx.x] + sc[threadIdx.x] - votes;
    offsets[i] = (int32_t)min(off, (int64_t)INT32_MAX);
    if (off >= cap_pairs || votes == 0) return;
    const int64_t room = (int64_t)cap_pairs - off;
    const int limit = (int)min((int64_t)votes, room);
    int32_t* out = hit_idx + off;

    const hough_peak_t pk = peaks[i];
    const uint32_t maskM = (M >= 32) ? 0xFFFFFFFFu : ((1u << M) - 1u);
    const uint32_t W = 1u << F;
    const int cshift = M - cell_bits;
    const uint32_t n_cell = 1u << cell_bits;
    int found = 0;
    for (int L = 0; L < n_layers; ++L) {
        const int32_t e = E[(size_t)L * n_cols + (size_t)pk.l * n_qpt + pk.k];
        if (e == INT32_MIN) continue;
        // hits of layer L with PhiM in [lo, lo + W) (mod 2^M) fall into bin b
        const uint32_t lo = ((uint32_t)e + ((uint32_t)pk.b << F)) & maskM;
        const uint32_t c0 = lo >> cshift;
        const uint32_t c1 = ((lo + W - 1) & maskM) >> cshift;
        const uint32_t ncells = ((c1 - c0) & (n_cell - 1)) + 1;
        for (uint32_t j = 0; j < ncells; ++j) {
            const int cell = (L << cell_bits) | (int)((c0 + j) & (n_cell - 1));
            const int a = cell_start[cell], z = cell_start[cell + 1];
            for (int q = a; q < z; ++q) {
                if (((sorted_phi[q] - lo) & maskM) >= W) continue;
                const int32_t h = sorted_h[q];
                // keep the `limit` smallest hit indices, ascending (insertion)
                if (found < limit) {
                    int p = found++;
                    while (p > 0 && out[p - 1] > h) {
                        out[p] = out[p - 1];
                        --p;
                    }
                    out[p] = h;
                } else if (out[limit - 1] > h) {
                    int p = limit - 1;
                    while (p > 0 && out[p - 1] > h) {
                        out[p] = out[p - 1];
                        --p;
                    }
                    out[p] = h;
                }
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

}  // namespace

// ====================================================================== C ABI
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
    if (g.n_qpt % kVoteCols) return HOUGH_E_UNSUPPORTED;
    if (g.acc_bits == 32) {
        if (g.frac_bits != 8) return HOUGH_E_UNSUPPORTED;
    } else if (g.acc_bits == 16) {
        if (g.frac_bits != 7 || g.max_hits_per_event > 32767) return HOUGH_E_UNSUPPORTED;
    } else {
        return HOUGH_E_UNSUPPORTED;
    }
    // the slab of one vote workgroup must fit the 160 KiB of LDS
    if ((size_t)g.n_phi * 256 > 160 * 1024 && g.acc_bits == 32) return HOUGH_E_UNSUPPORTED;
    if ((size_t)g.n_phi * 128 > 160 * 1024 && g.acc_bits == 16) return HOUGH_E_UNSUPPORTED;
    if (!(g.qpt_max >= g.qpt_min) || !(g.d0_max >= g.d0_min)) return HOUGH_E_INVAL;
    if ((int64_t)g.n_d0 * g.n_qpt * g.n_phi > ((int64_t)1 << 31)) return HOUGH_E_UNSUPPORTED;

    hough_plan* p = new (std::nothrow) hough_plan();
    if (!p) return HOUGH_E_NOMEM;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return HOUGH_E_HIP;
    }
    p->n_layers = geom->n_layers;
    for (int L = 0; L < p->n_layers; ++L) {
        p->r[L] = geom->r_cm[L];
        p->halflen[L] = geom->halflen_cm ? geom->halflen_cm[L] : 0.0;
    }
    p->B = geom->B_tesla;
    p->g = g;
    p->log2_phi = lp;
    p->F = g.frac_bits;
    p->M = lp + g.frac_bits;
    p->cell_bits = p->M < 12 ? p->M : 12;
    p->n_cols = g.n_d0 * g.n_qpt;
    p->n_cells = p->n_layers << p->cell_bits;
    p->n_bins = (int64_t)p->n_cols * g.n_phi;
    for (int i = 0; i < kCordicSteps; ++i)
        p->cordic.t[i] = (int32_t)llrint(atan(ldexp(1.0, -i)) * (2147483648.0 / M_PI));

    // sample table E[L][l][k] in IEEE double (no contraction: built with -ffp-contract=off)
    const size_t ntab = (size_t)p->n_layers * p->n_cols;
    int32_t* E = (int32_t*)malloc(ntab * sizeof(int32_t));
    if (!E) {
        delete p;
        return HOUGH_E_NOMEM;
    }
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
                int32_t v = INT32_MIN;
                if (den > 0.0) {
                    const double A = num / den;
                    if (fabs(A) <= 1.0) {
                        v = (int32_t)llrint(asin(A) * K);
                        ++nvalid;
                    }
                }
                E[((size_t)L * g.n_d0 + l) * g.n_qpt + k] = v;
            }
        }
        p->layers.valid_cols[L] = nvalid;
    }
    if (hipMalloc(&p->d_E, ntab * sizeof(int32_t)) != hipSuccess) {
        free(E);
        delete p;
        return HOUGH_E_NOMEM;
    }
    const hipError_t ce = hipMemcpy(p->d_E, E, ntab * sizeof(int32_t), hipMemcpyHostToDevice);
    free(E);
    if (ce != hipSuccess) {
        (void)hipFree(p->d_E);
        delete p;
        return HOUGH_E_HIP;
    }
    const int vote_lds = g.acc_bits == 32 ? g.n_phi * 256 : g.n_phi * 128;
    hipError_t ae = g.acc_bits == 32
                        ? hipFuncSetAttribute((const void*)k_vote<false>, hipFuncAttributeMaxDynamicSharedMemorySize, vote_lds)
                        : hipFuncSetAttribute((const void*)k_vote<true>, hipFuncAttributeMaxDynamicSharedMemorySize, vote_lds);
    if (ae != hipSuccess) {
        (void)hipFree(p->d_E);
        delete p;
        return HOUGH_E_HIP;
    }
    *out = p;
    return HOUGH_OK;
}

void hough_plan_destroy(hough_plan_t* plan) {
    if (!plan) return;
    if (plan->d_E) (void)hipFree(plan->d_E);
    delete plan;
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

static int check_hits(const hough_plan_t* p, const hough_hits_t* hits) {
    if (!p || !hits) return HOUGH_E_INVAL;
    if (hits->n < 0 || hits->n > p->g.max_hits_per_event) return HOUGH_E_INVAL;
    if (hits->n > 0 && (!hits->x || !hits->y || !hits->layer)) return HOUGH_E_INVAL;
    return HOUGH_OK;
}

int hough_prep(const hough_plan_t* p, const hough_hits_t* hits, uint32_t* phi_out, void* ws, size_t ws_bytes,
               hough_status_t* st, hipStream_t stream) {
    int rc = check_hits(p, hits);
    if (rc) return rc;
    if (!ws || !st) return HOUGH_E_INVAL;
    const WsLayout L = ws_layout(p, 0);
    if (ws_bytes < L.total) return HOUGH_E_SMALL_WS;
    const int n = hits->n;
    hipLaunchKernelGGL(k_prep_init, dim3(((p->n_cells + 1) + 1023) / 1024), dim3(1024), 0, stream,
                       at<int32_t>(ws, L.cell_count), p->n_cells, st, n);
    if (n > 0)
        hipLaunchKernelGGL(k_prep_hits, dim3((n + 255) / 256), dim3(256), 0, stream, hits->x, hits->y,
                           hits->layer, n, p->n_layers, p->cell_bits, p->cordic, at<uint32_t>(ws, L.phi32),
                           at<uint8_t>(ws, L.lay), phi_out, at<int32_t>(ws, L.cell_count), st);
    hipLaunchKernelGGL(k_prep_scan, dim3(1), dim3(kScanThreads), 0, stream, at<int32_t>(ws, L.cell_count),
                       at<int32_t>(ws, L.cell_start), at<int32_t>(ws, L.cell_cursor), p->n_cells, p->n_layers,
                       p->cell_bits, p->layers, st);
    if (n > 0)
        hipLaunchKernelGGL(k_prep_scatter, dim3((n + 255) / 256), dim3(256), 0, stream, at<uint32_t>(ws, L.phi32),
                           at<uint8_t>(ws, L.lay), n, p->cell_bits, p->M, at<int32_t>(ws, L.cell_cursor),
                           at<uint32_t>(ws, L.sorted_phi), at<int32_t>(ws, L.sorted_h));
    return launch_status();
}

int hough_vote(const hough_plan_t* p, const hough_hits_t* hits, void* acc, void* ws, size_t ws_bytes,
               hough_status_t* st, hipStream_t stream) {
    if (!acc) return HOUGH_E_INVAL;
    int rc = hough_prep(p, hits, nullptr, ws, ws_bytes, st, stream);
    if (rc) return rc;
    const WsLayout L = ws_layout(p, 0);
    const int n_slabs = p->n_cols / kVoteCols;
    if (p->g.acc_bits == 32)
        hipLaunchKernelGGL(k_vote<false>, dim3(n_slabs), dim3(kVoteThreads), p->g.n_phi * 256, stream, p->d_E,
                           at<int32_t>(ws, L.cell_start), at<uint32_t>(ws, L.sorted_phi), p->n_layers,
                           p->cell_bits, p->n_cols, p->g.n_phi, p->F, acc, st);
    else
        hipLaunchKernelGGL(k_vote<true>, dim3(n_slabs), dim3(kVoteThreads), p->g.n_phi * 128, stream, p->d_E,
                           at<int32_t>(ws, L.cell_start), at<uint32_t>(ws, L.sorted_phi), p->n_layers,
                           p->cell_bits, p->n_cols, p->g.n_phi, p->F, acc, st);
    return launch_status();
}

int hough_peaks(const hough_plan_t* p, const void* acc, int32_t threshold, hough_peak_t* peaks, int32_t cap,
                void* ws, size_t ws_bytes, hough_status_t* st, hipStream_t stream) {
    if (!p || !acc || !peaks || !ws || !st || cap < 1 || threshold < 1) return HOUGH_E_INVAL;
    const WsLayout L = ws_layout(p, 0);
    if (ws_bytes < L.total) return HOUGH_E_SMALL_WS;
    const int strips = p->g.n_phi / kStrip;
    const int gl = peak_group_lanes(p);
    const int lranges = (p->g.n_d0 + kPeakPlanes - 1) / kPeakPlanes;
    const int64_t mark_threads = (int64_t)strips * p->g.n_qpt * lranges;
    const int64_t n_strips = p->n_bins / kStrip;
    const int64_t groups = peak_groups(p);
    if (p->g.acc_bits == 32)
        hipLaunchKernelGGL(k_peaks_mark<int32_t>, dim3((unsigned)((mark_threads + 255) / 256)), dim3(256), 0,
                           stream, static_cast<const int32_t*>(acc), threshold, p->g.n_d0, p->g.n_qpt,
                           p->g.n_phi, gl, at<uint8_t>(ws, L.flags), at<int32_t>(ws, L.grp_count));
    else
        hipLaunchKernelGGL(k_peaks_mark<int16_t>, dim3((unsigned)((mark_threads + 255) / 256)), dim3(256), 0,
                           stream, static_cast<const int16_t*>(acc), threshold, p->g.n_d0, p->g.n_qpt,
                           p->g.n_phi, gl, at<uint8_t>(ws, L.flags), at<int32_t>(ws, L.grp_count));
    hipLaunchKernelGGL(k_peaks_scan, dim3(1), dim3(kScanThreads), 0, stream, at<int32_t>(ws, L.grp_count),
                       at<int32_t>(ws, L.grp_off), groups, cap, st);
    if (p->g.acc_bits == 32)
        hipLaunchKernelGGL(k_peaks_write<int32_t>, dim3((unsigned)((n_strips + 255) / 256)), dim3(256), 0, stream,
                           static_cast<const int32_t*>(acc), at<uint8_t>(ws, L.flags), at<int32_t>(ws, L.grp_off),
                           p->g.n_qpt, p->g.n_phi, gl, n_strips, peaks, cap);
    else
        hipLaunchKernelGGL(k_peaks_write<int16_t>, dim3((unsigned)((n_strips + 255) / 256)), dim3(256), 0, stream,
                           static_cast<const int16_t*>(acc), at<uint8_t>(ws, L.flags), at<int32_t>(ws, L.grp_off),
                           p->g.n_qpt, p->g.n_phi, gl, n_strips, peaks, cap);
    return launch_status();
}

int hough_assign(const hough_plan_t* p, const hough_peak_t* peaks, int32_t cap_peaks, int32_t* offsets,
                 int32_t* hit_idx, int32_t cap_pairs, void* ws, size_t ws_bytes, hough_status_t* st,
                 hipStream_t stream) {
    if (!p || !peaks || !offsets || !hit_idx || !ws || !st || cap_peaks < 1 || cap_pairs < 1) return HOUGH_E_INVAL;
    const WsLayout L = ws_layout(p, cap_peaks);
    if (ws_bytes < L.total) return HOUGH_E_SMALL_WS;
    const unsigned nblk = (unsigned)((cap_peaks + kAssignBlock - 1) / kAssignBlock);
    hipLaunchKernelGGL(k_assign_blocksum, dim3(nblk), dim3(kAssignBlock), 0, stream, peaks, cap_peaks, st,
                       at<int64_t>(ws, L.blk_sum));
    hipLaunchKernelGGL(k_assign_topscan, dim3(1), dim3(kScanThreads), 0, stream, at<int64_t>(ws, L.blk_sum),
                       at<int64_t>(ws, L.blk_off), cap_peaks, offsets, cap_pairs, st);
    hipLaunchKernelGGL(k_assign_fill, dim3(nblk), dim3(kAssignBlock), 0, stream, peaks, cap_peaks, st,
                       at<int64_t>(ws, L.blk_off), p->d_E, at<int32_t>(ws, L.cell_start),
                       at<uint32_t>(ws, L.sorted_phi), at<int32_t>(ws, L.sorted_h), p->n_layers, p->cell_bits,
                       p->n_cols, p->g.n_qpt, p->M, p->F, offsets, hit_idx, cap_pairs);
    return launch_status();
}

}  // extern "C"
