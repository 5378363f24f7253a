// probe.hip -- peak-rate microbenchmarks the roofline figures are set
// against: a streaming copy (HBM read + write), a fused multiply-add chain in
// FP64 (the NTT's exact modular product runs on it for primes below 2^50)
// and a v_mad_u64_u32 chain (the 32 x 32 + 64-bit integer multiply-add of the
// base conversions).  Built into libppstat_probe.so, separate from the
// library proper.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ppstat_probe.h"

namespace {

typedef uint64_t u64;

__global__ void __launch_bounds__(256) k_copy(const ulonglong2* __restrict__ src,
                                              ulonglong2* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

// eight independent chains per thread keep the pipeline full; the result is
// stored so that no chain is dead code
__global__ void __launch_bounds__(256) k_fma_f64(double* out, int iters, double a, double b) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = (double)(t + k) * 1e-9;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = __fma_rn(x[k], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[t] = s;
}

__global__ void __launch_bounds__(256) k_mad_u64_u32(u64* out, int iters, uint32_t m) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  u64 acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = t * 8 + k;
  // each step multiplies the accumulator's low word: a dependent chain the
  // compiler cannot hoist
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = (u64)(uint32_t)acc[k] * m + acc[k];
  }
  u64 s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s ^= acc[k];
  out[t] = s;
}

int status(hipError_t e) { return e == hipSuccess ? 0 : -6; }

}  // namespace

extern "C" {

int ppst_probe_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst || bytes % 16) return -1;
  const size_t n = bytes / 16;
  hipLaunchKernelGGL(k_copy, dim3(256 * 32), dim3(256), 0, (hipStream_t)stream,
                     (const ulonglong2*)src, (ulonglong2*)dst, n);
  return status(hipGetLastError());
}

int ppst_probe_fma_f64(double* out, size_t threads, int iters, void* stream) {
  if (!out || threads == 0 || threads % 256 || iters <= 0) return -1;
  hipLaunchKernelGGL(k_fma_f64, dim3((unsigned)(threads / 256)), dim3(256), 0,
                     (hipStream_t)stream, out, iters, 0.999999, 1e-7);
  return status(hipGetLastError());
}

int ppst_probe_mad_u64_u32(uint64_t* out, size_t threads, int iters, void* stream) {
  if (!out || threads == 0 || threads % 256 || iters <= 0) return -1;
  hipLaunchKernelGGL(k_mad_u64_u32, dim3((unsigned)(threads / 256)), dim3(256), 0,
                     (hipStream_t)stream, (u64*)out, iters, 2246822519u);
  return status(hipGetLastError());
}

}  // extern "C"
