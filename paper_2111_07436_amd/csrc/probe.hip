// Measurement probes: the device's achievable HBM copy bandwidth (STREAM copy) and FP64
// FMA rate, measured with the same launch machinery as the solver, so rooflines can be
// quoted against both the published peaks and what this device sustains.
#include <hip/hip_runtime.h>

#include "runtime.hpp"

namespace {

// dst[i] = src[i], 16-byte accesses: each workgroup copies kCopyUnroll * 256 consecutive
// 16-byte elements, every thread issuing its kCopyUnroll loads before its stores.
constexpr int kCopyUnroll = 4;
typedef double dvec2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void copy_kernel(const dvec2* __restrict__ src,
                                                   dvec2* __restrict__ dst, size_t n2) {
  const size_t base = (size_t)blockIdx.x * 256 * kCopyUnroll + threadIdx.x;
  dvec2 v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const size_t i = base + (size_t)u * 256;
    if (i < n2) v[u] = __builtin_nontemporal_load(&src[i]);
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const size_t i = base + (size_t)u * 256;
    if (i < n2) __builtin_nontemporal_store(v[u], &dst[i]);
  }
}

// kChains independent FMA chains per lane, `iters` rounds; the sums go to sink so nothing
// is dead code.
constexpr int kChains = 16;
__global__ __launch_bounds__(256) void fma_kernel(double* sink, int iters, double b, double c) {
  double a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (double)(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = fma(a[k], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

using namespace camp;

extern "C" {

int camp_probe_copy(const double* d_src, double* d_dst, size_t n, int reps, void* stream,
                    double* gb_per_s) {
  if (!d_src || !d_dst || !gb_per_s || n < 2 || (n & 1) || reps < 1) {
    set_error("camp_probe_copy: bad argument");
    return CAMP_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  const size_t n2 = n / 2;
  const size_t per_block = 256 * kCopyUnroll;
  if ((n2 + per_block - 1) / per_block > 0x7FFFFFFF) {
    set_error("camp_probe_copy: buffer too large");
    return CAMP_EINVAL;
  }
  const unsigned grid = (unsigned)((n2 + per_block - 1) / per_block);
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, s, (const dvec2*)d_src, (dvec2*)d_dst, n2);
  hipEventRecord(a, s);
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, s, (const dvec2*)d_src, (dvec2*)d_dst, n2);
  hipEventRecord(b, s);
  e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(e, "copy probe");
  *gb_per_s = 2.0 * 8.0 * (double)n * reps / (ms * 1e-3) / 1e9;
  return CAMP_OK;
}

int camp_probe_fma(double* d_sink, int blocks, int iters, void* stream, double* tflop_per_s) {
  if (!d_sink || !tflop_per_s || blocks < 1 || iters < 1) {
    set_error("camp_probe_fma: bad argument");
    return CAMP_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  hipLaunchKernelGGL(fma_kernel, dim3(blocks), dim3(256), 0, s, d_sink, 16, 1.0000001, 1e-9);
  hipEventRecord(a, s);
  hipLaunchKernelGGL(fma_kernel, dim3(blocks), dim3(256), 0, s, d_sink, iters, 1.0000001, 1e-9);
  hipEventRecord(b, s);
  e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(e, "fma probe");
  *tflop_per_s = 2.0 * kChains * (double)iters * blocks * 256 / (ms * 1e-3) / 1e12;
  return CAMP_OK;
}

}  // extern "C"
