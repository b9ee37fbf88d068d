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
// 256 threads, in a fixed order: each thread issues its (up to) 8 loads of a
// 2048-entry round at once, then wave shuffles and the four wave totals in
// a fixed order.  (One round of independent loads instead of a chain of
// dependent ones; these sums sit between every two PCG sweeps, in a finalize
// kernel or at the start of the next sweep.)  tid is
// the thread's linear index in a workgroup of 256 (x fastest).
__device__ __forceinline__ void block_sum_parts(const double *part, int n, long long stride,
                                                double *s0, double *s1,
                                                int tid = threadIdx.x) {
  double a = 0.0, b = 0.0;
  for (int t0 = 0; t0 < n; t0 += 8 * 256) {
    double va[8], vb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int t = t0 + tid + 256 * q;
      va[q] = t < n ? part[t] : 0.0;
      vb[q] = (s1 && t < n) ? part[stride + t] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      a += va[q];
      b += vb[q];
    }
  }
  a = wave_sum(a);
  b = wave_sum(b);
  __shared__ double ra[4], rb[4];
  if ((tid & 63) == 0) {
    ra[tid >> 6] = a;
    rb[tid >> 6] = b;
  }
  __syncthreads();
  if (tid == 0) {
    *s0 = (ra[0] + ra[1]) + (ra[2] + ra[3]);
    if (s1) *s1 = (rb[0] + rb[1]) + (rb[2] + rb[3]);
  }
}

// alpha = (r.z) / (p.Ap) of a PCG iteration (Sec. 2.2, Fig. pcg), evaluated
// at the start of the x / r update sweep instead of in a kernel of its own:
// p.Ap from pass A's partials pa[0..npa).  Every workgroup sums the same
// partials in the same order, so all get the same alpha, and p.Ap <= 0 or a
// non-finite sum (breakdown) stops them all (returns 0).  The `writer`
// workgroup records p.Ap, alpha (or done / breakdown) and (r.z)_old = r.z for
// the next beta; r.z itself is not written in the same launch.  256 threads,
// linear index tid.
template <class Scalars>
__device__ __forceinline__ int pcg_alpha(const double *pa, int npa, Scalars *sc, bool writer,
                                         int tid, double *alpha) {
  __shared__ double s_py;
  block_sum_parts(pa, npa, 0, &s_py, nullptr, tid);
  __syncthreads();
  const double py = s_py, rz = sc->rr;
  const bool bad = !(py > 0.0) || !isfinite(py);
  if (writer && tid == 0) {
    sc->py = py;
    sc->rr_old = rz;
    if (bad) {
      sc->done = 1;
      sc->status = -4;
    } else {
      sc->alpha = rz / py;
    }
  }
  *alpha = rz / py;
  return !bad;
}

// End of a PCG iteration (Sec. 2.2, Fig. pcg), evaluated at the start
// of the next sweep instead of in a kernel of its own: r.z and r.r from the
// partials of the iteration's x / r update (part[0..n), part[stride..+n)),
// then the stopping test ||r||^2 <= tol2 (converged), a non-finite sum
// (breakdown) or iters >= maxit, else beta = (r.z) / (r.z)_old.  Every
// workgroup of the launch sums the same partials in the same order, so all
// take the same decision; only the `writer` workgroup records the scalars
// (r.z, ||r||^2, iteration count, beta, done / status).  Fields read here
// (rr_old, tol2, maxit) are not written in the same launch.  Returns 1 when
// the iteration is the last.  256 threads, linear index tid.
template <class Scalars>
__device__ __forceinline__ int pcg_decide(const double *part, int n, long long stride, int iters,
                                          Scalars *sc, bool writer, int tid, double *beta) {
  __shared__ double s_z, s_r;
  block_sum_parts(part, n, stride, &s_z, &s_r, tid);
  __syncthreads();
  const double rz = s_z, rr = s_r;
  int done = 0, status = 0;
  if (!isfinite(rr) || !isfinite(rz)) {
    done = 1;
    status = -4;
  } else if (!(rr > sc->tol2)) {
    done = 1;
    status = 1;
  } else if (iters >= sc->maxit) {
    done = 1;
  }
  *beta = rz / sc->rr_old;
  if (writer && tid == 0) {
    sc->rr = rz;
    sc->rnorm2 = rr;
    sc->iters = iters;
    if (done) {
      sc->done = 1;
      if (status) sc->status = status;
    } else {
      sc->beta = *beta;
    }
  }
  return done;
}

}  // namespace sts
