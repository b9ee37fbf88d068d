// Deterministic reductions: wave64 shuffles, then a fixed-order sum of the
// waves of a workgroup; workgroup partials are summed by one workgroup in a
// fixed pattern.  Results are bitwise reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

namespace sts {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum two values over a workgroup of NT threads (NT a multiple of 64); the
// totals are written by thread 0 to out_a / out_b.
template <int NT>
__device__ __forceinline__ void wg_sum2(double a, double b, int tid, double *out_a,
                                        double *out_b) {
  __shared__ double sa[NT / 64], sb[NT / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  if ((tid & 63) == 0) {
    sa[tid >> 6] = a;
    sb[tid >> 6] = b;
  }
  __syncthreads();
  if (tid == 0) {
    double x = 0.0, y = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      x += sa[w];
      y += sb[w];
    }
    *out_a = x;
    if (out_b) *out_b = y;
  }
}

// Sum part[0..n) (and part[stride..stride+n) when two) with one workgroup of
// 256 threads, in a fixed order.
__device__ __forceinline__ void block_sum_parts(const double *part, int n, long long stride,
                                                double *s0, double *s1) {
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int t = tid; t < n; t += 256) {
    a += part[t];
    if (s1) b += part[stride + t];
  }
  __shared__ double ra[256], rb[256];
  ra[tid] = a;
  rb[tid] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      ra[tid] += ra[tid + h];
      rb[tid] += rb[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    *s0 = ra[0];
    if (s1) *s1 = rb[0];
  }
}

}  // namespace sts
