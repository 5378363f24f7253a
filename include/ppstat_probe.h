/*
 * ppstat_probe.h -- peak-rate microbenchmarks of libppstat_probe.so, the
 * measured ceilings beside MI355X's published ones that the benchmark sets
 * its roofline fractions against.  Not part of the encrypted-statistics
 * library (include/ppstat.h).
 *
 * Every call enqueues one kernel on `stream` (a hipStream_t, NULL for the
 * default stream) and returns 0, -1 for a malformed argument (nothing is
 * launched) or -6 when the launch failed.  Buffers are device memory owned
 * by the caller; the caller times the launch (HIP events on the stream).
 */
#ifndef PPSTAT_PROBE_H
#define PPSTAT_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[0..bytes) = src[0..bytes): 16-byte vector loads and stores over a
 * grid-stride loop (8192 workgroups of 256); bytes a multiple of 16; the
 * buffers must not overlap.  Moves 2 * bytes through HBM. */
int ppst_probe_copy(const void* src, void* dst, size_t bytes, void* stream);
/* `threads` work-items (a multiple of 256), each running eight independent
 * chains of `iters` FP64 fused multiply-adds; out[threads] receives one
 * double per work-item.  8 * threads * iters FMAs. */
int ppst_probe_fma_f64(double* out, size_t threads, int iters, void* stream);
/* the same with 32 x 32 -> 64-bit multiply-adds into 64-bit accumulators
 * (v_mad_u64_u32); out[threads] receives one word per work-item */
int ppst_probe_mad_u64_u32(uint64_t* out, size_t threads, int iters, void* stream);

#ifdef __cplusplus
}
#endif

#endif
