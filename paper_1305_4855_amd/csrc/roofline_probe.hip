// roofline_probe.hip -- micro-benchmarks that measure the ceilings the Hough kernels are compared
// with on one gfx950 device: the rate of conflict-free LDS atomic adds (ds_add_u32 without return,
// the operation of the slab votes), plain LDS reads and writes of the same width as controls, wide
// LDS reads (LDS bandwidth), and an HBM streaming copy.
//
// Every kernel runs a fixed, bounded number of iterations on its own buffers; nothing waits on
// another workgroup.  The host entry points time `reps` back-to-back launches between two HIP
// events and return the average launch time in microseconds together with the number of
// operations (lane-operations for the LDS kernels, bytes for the copy) of one launch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "roofline_probe.h"

namespace {

constexpr int kThreads = 1024;  // 16 waves per workgroup
constexpr int kUnroll = 16;     // independent LDS instructions per loop iteration

// LDS atomic add, no return: lane i of a wave adds to dword (wave * 64 + i) of the workgroup's
// array, so the 64 lanes of an instruction touch 64 consecutive dwords (every bank once per 32
// lanes) and the instructions of a wave carry no dependency on one another.
__global__ __launch_bounds__(kThreads) void k_lds_atomic(int iters, uint32_t* __restrict__ out) {
    __shared__ uint32_t s[kThreads * 2];
    const int t = threadIdx.x;
    s[t] = 0u;
    s[t + kThreads] = 0u;
    __syncthreads();
    uint32_t* p = &s[t];
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) __hip_atomic_fetch_add(p + (u & 1) * kThreads, 1u, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    if (s[t] != (uint32_t)(iters * (kUnroll / 2))) out[blockIdx.x * kThreads + t] = s[t];  // never, keeps the adds
}

// LDS atomic add with return (ds_add_rtn_u32), addresses as for k_lds_atomic; the returned words
// are folded into one value so that every return is used.
__global__ __launch_bounds__(kThreads) void k_lds_atomic_rtn(int iters, uint32_t* __restrict__ out) {
    __shared__ uint32_t s[kThreads * 2];
    const int t = threadIdx.x;
    s[t] = 0u;
    s[t + kThreads] = 0u;
    __syncthreads();
    uint32_t* p = &s[t];
    uint32_t acc = 0u;
    for (int i = 0; i < iters; ++i) {
        uint32_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            v[u] = __hip_atomic_fetch_add(p + (u & 1) * kThreads, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc ^= v[u];
    }
    __syncthreads();
    if (s[t] != (uint32_t)(iters * (kUnroll / 2)) || acc == 0x9e3779b9u) out[blockIdx.x * kThreads + t] = s[t] | 1u;
}

// The counting step of a vote into a histogram whose words are restored right away: an atomic add
// with return of 2^16 followed by an atomic subtract of 2^16 from the same word (one lane-vote =
// two LDS atomics).  Every word ends where it started.
__global__ __launch_bounds__(kThreads) void k_lds_vote_pair(int iters, uint32_t* __restrict__ out) {
    __shared__ uint32_t s[kThreads * 2];
    const int t = threadIdx.x;
    s[t] = 0u;
    s[t + kThreads] = 0u;
    __syncthreads();
    uint32_t* p = &s[t];
    uint32_t best = 0u;
    for (int i = 0; i < iters; ++i) {
        uint32_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            v[u] = __hip_atomic_fetch_add(p + (u & 1) * kThreads, 0x10000u, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_sub(p + (u & 1) * kThreads, 0x10000u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) best = max(best, v[u]);
    }
    __syncthreads();
    if (s[t] != 0u || best != 0u) out[blockIdx.x * kThreads + t] = s[t] | best | 1u;
}

// LDS read of one dword per lane: 16 loads per iteration at immediate offsets of one base address
// (64 consecutive dwords per load, so conflict-free), the base passed through an empty asm each
// iteration so that the loads cannot be hoisted out of the loop; one XOR per loaded value keeps the
// loads alive (one VALU per LDS instruction, below the LDS rate).  The loads are kStride dwords
// apart, more than a paired load (ds_read2) can span and not a multiple of 64 dwords, so each
// stays a single ds_read_b32.
constexpr int kWords = 4096;   // dwords of the 32-bit probe arrays (16 KiB)
constexpr int kStride = 257;   // dwords between the loads of one iteration
static_assert((kUnroll - 1) * kStride + 64 <= kWords, "probe array too small");

__global__ __launch_bounds__(kThreads) void k_lds_read32(int iters, uint32_t* __restrict__ out) {
    __shared__ uint32_t s[kWords];
    const int t = threadIdx.x;
    for (int i = t; i < kWords; i += kThreads) s[i] = (uint32_t)(3 * i + 1);
    __syncthreads();
    uint32_t acc = 0u;
    int base = t & 63;
    for (int i = 0; i < iters; ++i) {
        asm volatile("" : "+v"(base));
        uint32_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = s[base + u * kStride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc ^= v[u];
    }
    if (acc == 0x9e3779b9u) out[blockIdx.x * kThreads + t] = acc;
}

// LDS write of one dword per lane (addresses as for the read).
__global__ __launch_bounds__(kThreads) void k_lds_write32(int iters, uint32_t* __restrict__ out) {
    __shared__ uint32_t s[kWords];
    const int t = threadIdx.x;
    int base = t & 63;
    uint32_t val = (uint32_t)t;
    for (int i = 0; i < iters; ++i) {
        asm volatile("" : "+v"(base), "+v"(val));
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) s[base + u * kStride] = val;
    }
    __syncthreads();
    if (s[t] == 0x9e3779b9u) out[blockIdx.x * kThreads + t] = s[t];
}

// LDS read of 16 bytes per lane (ds_read_b128): the LDS read bandwidth in bytes per clock.
__global__ __launch_bounds__(kThreads) void k_lds_read128(int iters, uint32_t* __restrict__ out) {
    __shared__ uint4 s[kThreads * 2];
    const int t = threadIdx.x;
    s[t] = make_uint4(t, t + 1, t + 2, t + 3);
    s[t + kThreads] = make_uint4(3 * t, t, 7, t ^ 5);
    __syncthreads();
    uint32_t acc = 0u;
    int base = t & 63;
    for (int i = 0; i < iters; ++i) {
        asm volatile("" : "+v"(base));
        uint4 v[kUnroll / 2];
#pragma unroll
        for (int u = 0; u < kUnroll / 2; ++u) v[u] = s[base + u * 64];  // 1 KiB per wave per load
#pragma unroll
        for (int u = 0; u < kUnroll / 2; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    if (acc == 0x9e3779b9u) out[blockIdx.x * kThreads + t] = acc;
}

// HBM streaming copy, 16 bytes per lane per step, grid-stride.
__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

// HBM streaming write (fill), 16 bytes per lane per step.
__global__ __launch_bounds__(256) void k_fill(uint4* __restrict__ dst, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = make_uint4((uint32_t)i, 0u, 0u, 0u);
}

template <typename Launch>
int timed(int reps, float* us, Launch launch) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1;
    }
    launch();  // warm-up
    (void)hipEventRecord(a, nullptr);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(b, nullptr);
    int rc = hipEventSynchronize(b) == hipSuccess ? 0 : -1;
    float ms = 0.0f;
    if (rc == 0 && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = -1;
    *us = ms * 1000.0f / (float)reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (hipGetLastError() != hipSuccess) rc = -1;
    return rc;
}

}  // namespace

extern "C" {

// kind: 0 = LDS atomic add (no return), 1 = LDS read 32-bit, 2 = LDS write 32-bit, 3 = LDS read
// 128-bit, 4 = LDS atomic add with return, 5 = vote pair (add with return + subtract; one lane-op
// counts the pair).  blocks workgroups of 1024 threads, iters loop iterations of 16 instructions (8 for
// kind 3) per wave.  out: device scratch of blocks * 1024 dwords (written only in impossible cases).
// *lane_ops = lane-operations of one launch; *us = average launch time.  Returns 0 or -1.
int probe_lds(int kind, int blocks, int iters, int reps, uint32_t* out, double* lane_ops, float* us) {
    if (blocks < 1 || iters < 1 || reps < 1 || !out || !lane_ops || !us) return -1;
    const double per_iter = kind == 3 ? kUnroll / 2 : kUnroll;
    *lane_ops = (double)blocks * kThreads * iters * per_iter;
    switch (kind) {
        case 0: return timed(reps, us, [&] { hipLaunchKernelGGL(k_lds_atomic, dim3(blocks), dim3(kThreads), 0, nullptr, iters, out); });
        case 1: return timed(reps, us, [&] { hipLaunchKernelGGL(k_lds_read32, dim3(blocks), dim3(kThreads), 0, nullptr, iters, out); });
        case 2: return timed(reps, us, [&] { hipLaunchKernelGGL(k_lds_write32, dim3(blocks), dim3(kThreads), 0, nullptr, iters, out); });
        case 3: return timed(reps, us, [&] { hipLaunchKernelGGL(k_lds_read128, dim3(blocks), dim3(kThreads), 0, nullptr, iters, out); });
        case 4: return timed(reps, us, [&] { hipLaunchKernelGGL(k_lds_atomic_rtn, dim3(blocks), dim3(kThreads), 0, nullptr, iters, out); });
        case 5: return timed(reps, us, [&] { hipLaunchKernelGGL(k_lds_vote_pair, dim3(blocks), dim3(kThreads), 0, nullptr, iters, out); });
        default: return -1;
    }
}

// kind: 0 = copy (bytes read + bytes written counted), 1 = fill (bytes written).  src and dst are
// device buffers of `bytes` bytes (a multiple of 16); blocks workgroups of 256 threads.
int probe_hbm(int kind, const void* src, void* dst, size_t bytes, int blocks, int reps, double* moved, float* us) {
    if (!dst || bytes % 16 || blocks < 1 || reps < 1 || !moved || !us || (kind == 0 && !src)) return -1;
    const size_t n16 = bytes / 16;
    if (kind == 0) {
        *moved = 2.0 * (double)bytes;
        return timed(reps, us, [&] {
            hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, nullptr, static_cast<const uint4*>(src),
                               static_cast<uint4*>(dst), n16);
        });
    }
    if (kind == 1) {
        *moved = (double)bytes;
        return timed(reps, us, [&] {
            hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, nullptr, static_cast<uint4*>(dst), n16);
        });
    }
    return -1;
}

}  // extern "C"
