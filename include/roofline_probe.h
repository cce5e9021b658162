/* roofline_probe.h -- micro-benchmarks of libroofline_probe.so: the device ceilings the Hough
 * kernels' roofline fractions are taken against (measurement code, not part of the track-finding
 * path).
 *
 * Every call launches its kernel `reps` times back to back on the default stream after one
 * warm-up launch, times them between two HIP events, and returns the average launch time in
 * microseconds (*us) with the amount of work of one launch.  Kernels run a fixed number of
 * iterations on their own buffers; none waits on another workgroup.  Return value: 0, or -1 for an
 * invalid argument (checked before any HIP call) or a HIP error.
 */
#ifndef ROOFLINE_PROBE_H
#define ROOFLINE_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* LDS rate.  kind: 0 = atomic add without return (ds_add_u32), 1 = 32-bit read, 2 = 32-bit write,
 * 3 = 128-bit read, 4 = atomic add with return (ds_add_rtn_u32), 5 = vote pair: an atomic add with
 * return followed by an atomic subtract of the same word (counted as one lane-operation).  `blocks` workgroups of 1024 threads, each wave issuing `iters` iterations of
 * 16 independent conflict-free instructions (8 for kind 3: 64 consecutive words per instruction).
 * out: (dev) caller-owned, blocks * 1024 words, zero on entry; a kernel writes to it only if its own
 * self-check fails, so a non-zero word after the call means a wrong result.
 * *lane_ops: lane-operations of one launch. */
int probe_lds(int kind, int blocks, int iters, int reps, uint32_t* out, double* lane_ops, float* us);

/* HBM streaming rate.  kind: 0 = copy src -> dst (*moved = 2 * bytes: read + written), 1 = fill dst
 * (*moved = bytes).  src, dst: (dev) caller-owned buffers of `bytes` bytes, a multiple of 16 (src
 * may be NULL for the fill).  `blocks` workgroups of 256 threads, 16 bytes per lane per step. */
int probe_hbm(int kind, const void* src, void* dst, size_t bytes, int blocks, int reps, double* moved, float* us);

#ifdef __cplusplus
}
#endif

#endif
