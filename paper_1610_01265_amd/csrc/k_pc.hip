// The factored preconditioner M^-1 = G G^T of the backward-Euler PCG, with G
// lower triangular in the cells' lexicographic order (r slowest, phi
// fastest): row c holds the cell and its -1 neighbours c - e_a that lie in
// the grid without wrapping across the periodic phi seam.  Entries are BF16
// arrays g[q][cell] (a preconditioner's entries need no more: any G with a
// positive diagonal gives an SPD M^-1, and the PCG iterates stay FP64):
// g[0] = G[c, c], g[1 + a] = G[c, c - e_a] (ignored where that neighbour does
// not exist); vectors and arithmetic are FP64.
//
//   (G^T x)_c = g0_c x_c + sum_a g_(1+a)(c + e_a) x_(c + e_a)
//   (G x)_c   = g0_c x_c + sum_a g_(1+a)(c) x_(c - e_a)
//
// A learned factor comes from the network outputs o (4 per cell) and the
// diagonal of A = V - dt S:  G[c, c] = d exp(o0), G[c, c - e_a] = d o_(1+a),
// d = A_cc^-1/2, so M^-1 is symmetric positive definite for any outputs and
// point Jacobi at o = 0.  The training objective per probe vector z is
// L = ||G^T A G z - z||^2 / N; with w = G z, y = A w, r = G^T y - z,
// q = G r, s = A q:  dL/dG[c, m] = 2 (y_c r_m + s_c z_m) / N.
//
// The kernels march the grid in 64 (phi) x 4 (theta) tiles of one r-plane,
// workgroups striding over the tiles; neighbour values are plain loads
// (the previous and next planes of the tile are in the caches).
#include "cnn_internal.h"
#include "k_common.h"
#include "k_reduce.h"

namespace sts {

namespace {

constexpr int TX = 64, TY = 4, NT = TX * TY;

struct PcDims {
  int n0, n1, n2;
  long long n12, n;
  int ntx, nty;
  long long items;
  int rev;  // debug: reversed workgroup order
};

PcDims dims_of(const sts_ctx *c) {
  PcDims d;
  d.n0 = c->n0;
  d.n1 = c->n1;
  d.n2 = c->n2;
  d.n12 = (long long)c->n1 * c->n2;
  d.n = c->ncell;
  d.ntx = (c->n2 + TX - 1) / TX;
  d.nty = (c->n1 + TY - 1) / TY;
  d.items = (long long)d.ntx * d.nty * c->n0;
  d.rev = (c->debug & STS_DEBUG_WG_REVERSE) ? 1 : 0;
  return d;
}

// Visit every cell once: workgroups stride over (tile, plane) items.
template <class F>
__device__ __forceinline__ void for_cells(const PcDims &d, F &&f) {
  for (long long it = wg_index(d.rev); it < d.items; it += gridDim.x) {
    const int bx = (int)(it % d.ntx);
    const long long r = it / d.ntx;
    const int by = (int)(r % d.nty);
    const int i = (int)(r / d.nty);
    const int k = bx * TX + threadIdx.x, j = by * TY + threadIdx.y;
    if (k < d.n2 && j < d.n1) f(i, j, k, (long long)i * d.n12 + (long long)j * d.n2 + k);
  }
}

// t = G^T x (- sub)
__global__ void __launch_bounds__(NT)
    k_pc_gt(PcDims d, const __bf16 *__restrict__ g, const double *__restrict__ x,
            const double *__restrict__ sub, double *__restrict__ t, const PcgScalars *sc) {
  if (sc && sc->done) return;
  const __bf16 *g1 = g + d.n, *g2 = g + 2 * d.n, *g3 = g + 3 * d.n;
  for_cells(d, [&](int i, int j, int k, long long c) {
    double v = (double)(float)g[c] * x[c];
    if (i + 1 < d.n0) v += (double)(float)g1[c + d.n12] * x[c + d.n12];
    if (j + 1 < d.n1) v += (double)(float)g2[c + d.n2] * x[c + d.n2];
    if (k + 1 < d.n2) v += (double)(float)g3[c + 1] * x[c + 1];
    t[c] = sub ? v - sub[c] : v;
  });
}

// z = G t
__global__ void __launch_bounds__(NT)
    k_pc_g(PcDims d, const __bf16 *__restrict__ g, const double *__restrict__ t,
           double *__restrict__ z, const PcgScalars *sc) {
  if (sc && sc->done) return;
  const __bf16 *g1 = g + d.n, *g2 = g + 2 * d.n, *g3 = g + 3 * d.n;
  for_cells(d, [&](int i, int j, int k, long long c) {
    double v = (double)(float)g[c] * t[c];
    if (i > 0) v += (double)(float)g1[c] * t[c - d.n12];
    if (j > 0) v += (double)(float)g2[c] * t[c - d.n2];
    if (k > 0) v += (double)(float)g3[c] * t[c - 1];
    z[c] = v;
  });
}

// 1 / sqrt(A_cc), A_cc = V - dt S_cc
__device__ __forceinline__ double inv_sqrt_diag(const Grid &gr, const double *sdiag, double dt,
                                                int i, int j, int k, long long c) {
  return 1.0 / sqrt(vol(gr, i, j, k) - dt * sdiag[c]);
}

// Factor from the network outputs o4[cell][4] (null: o = 0, point Jacobi).
// A non-finite entry sets *bad.
__global__ void __launch_bounds__(NT)
    k_pc_build(PcDims d, Grid gr, const double *__restrict__ sdiag, double dt,
               const float *__restrict__ o4, __bf16 *__restrict__ g, int *bad) {
  for_cells(d, [&](int i, int j, int k, long long c) {
    const double dd = inv_sqrt_diag(gr, sdiag, dt, i, j, k, c);
    double o[4] = {0.0, 0.0, 0.0, 0.0};
    if (o4) {
      const float4 v = *reinterpret_cast<const float4 *>(o4 + 4 * c);
      o[0] = v.x;
      o[1] = v.y;
      o[2] = v.z;
      o[3] = v.w;
    }
    // rounded to BF16 through FP32 (ties to even at each step)
    const __bf16 e0 = (__bf16)(float)(dd * exp(o[0]));
    const __bf16 e1 = (__bf16)(i > 0 ? (float)(dd * o[1]) : 0.0f);
    const __bf16 e2 = (__bf16)(j > 0 ? (float)(dd * o[2]) : 0.0f);
    const __bf16 e3 = (__bf16)(k > 0 ? (float)(dd * o[3]) : 0.0f);
    const float f0 = (float)e0;
    if (!(isfinite(f0) && f0 > 0.0f && isfinite((float)e1) && isfinite((float)e2) &&
          isfinite((float)e3)))
      atomicOr(bad, 1);
    g[c] = e0;
    g[c + d.n] = e1;
    g[c + 2 * d.n] = e2;
    g[c + 3 * d.n] = e3;
  });
}

// A caller's FP32 factor rounded to the BF16 store; after rounding the
// diagonal must be finite and positive, the other entries finite.
__global__ void __launch_bounds__(NT)
    k_pc_check(PcDims d, const float *__restrict__ g32, __bf16 *__restrict__ g, int *bad) {
  for_cells(d, [&](int i, int j, int k, long long c) {
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const __bf16 e = (__bf16)g32[c + q * d.n];
      const float f = (float)e;
      ok = ok && isfinite(f) && (q > 0 || f > 0.0f);
      g[c + q * d.n] = e;
    }
    if (!ok) atomicOr(bad, 1);
  });
}

// Network input of the factor network, bf16 [cells][16]: channel 0 =
// log(A_cc / V_c) * lscale, channel 1 = (T - tsh) * tsc, the rest 0.
__global__ void __launch_bounds__(NT)
    k_pc_pack(PcDims d, Grid gr, const double *__restrict__ sdiag, double dt, double lscale,
              const double *__restrict__ T, double tsh, double tsc, __bf16 *__restrict__ x) {
  for_cells(d, [&](int i, int j, int k, long long c) {
    const double V = vol(gr, i, j, k);
    const float f0 = (float)(log((V - dt * sdiag[c]) / V) * lscale);
    const float f1 = (float)((T[c] - tsh) * tsc);
    __bf16 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = (__bf16)0.0f;
    v[0] = (__bf16)f0;
    v[1] = (__bf16)f1;
    uint4 lo, hi;
    __builtin_memcpy(&lo, v, 16);
    __builtin_memcpy(&hi, v + 8, 16);
    uint4 *dst = reinterpret_cast<uint4 *>(x + 16 * c);
    dst[0] = lo;
    dst[1] = hi;
  });
}

// Gradient of the objective: dg[q][cell] = dL/dG entries (FP64, may be
// null); dout (bf16 [cells][16], may be null) = dL/do through the entry maps
// (dg0 G_cc, dg_(1+a) d), channels 4..15 zero; partial sums of r.r.
__global__ void __launch_bounds__(NT)
    k_pc_grad(PcDims d, Grid gr, const double *__restrict__ sdiag, double dt,
              const __bf16 *__restrict__ g, const double *__restrict__ y,
              const double *__restrict__ r, const double *__restrict__ s,
              const double *__restrict__ z, double *__restrict__ dg, __bf16 *__restrict__ dout,
              double *part) {
  const double two_n = 2.0 / (double)d.n;
  double rr = 0.0;
  for_cells(d, [&](int i, int j, int k, long long c) {
    const double yc = y[c], sc_ = s[c], rc = r[c];
    rr += rc * rc;
    double e[4];
    e[0] = two_n * (yc * rc + sc_ * z[c]);
    e[1] = i > 0 ? two_n * (yc * r[c - d.n12] + sc_ * z[c - d.n12]) : 0.0;
    e[2] = j > 0 ? two_n * (yc * r[c - d.n2] + sc_ * z[c - d.n2]) : 0.0;
    e[3] = k > 0 ? two_n * (yc * r[c - 1] + sc_ * z[c - 1]) : 0.0;
    if (dg) {
#pragma unroll
      for (int q = 0; q < 4; ++q) dg[c + q * d.n] = e[q];
    }
    if (dout) {
      const double dd = inv_sqrt_diag(gr, sdiag, dt, i, j, k, c);
      __bf16 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = (__bf16)0.0f;
      v[0] = (__bf16)(float)(e[0] * (double)(float)g[c]);
      v[1] = (__bf16)(float)(e[1] * dd);
      v[2] = (__bf16)(float)(e[2] * dd);
      v[3] = (__bf16)(float)(e[3] * dd);
      uint4 lo, hi;
      __builtin_memcpy(&lo, v, 16);
      __builtin_memcpy(&hi, v + 8, 16);
      uint4 *dst = reinterpret_cast<uint4 *>(dout + 16 * c);
      dst[0] = lo;
      dst[1] = hi;
    }
  });
  wg_sum2<NT>(rr, 0.0, threadIdx.y * TX + threadIdx.x, part + wg_index(d.rev), nullptr);
}

// The x / r update of a factor-PCG iteration fused with t = G^T r_new:
// x += alpha p, r_out = r_in - alpha y, t = G^T r_out.  A cell's t needs
// r_new of its +e_a neighbours, formed here from r_in and y exactly as their
// owners form it (the same operations: the same bits), so r_in and r_out
// are different arrays.  Partial sums: t.t (= r.z for z = G t, which
// k_pc_g forms next) and r.r.  FUSE: alpha from pass A's partials pa[0..npa)
// in every workgroup (pcg_alpha), workgroup 0 recording it.
template <bool FUSE>
__global__ void __launch_bounds__(NT)
    k_pc_xr_gt(PcDims d, const __bf16 *__restrict__ g, double *__restrict__ x,
               const double *__restrict__ p, const double *__restrict__ rin,
               double *__restrict__ rout, const double *__restrict__ y, double *__restrict__ t,
               double *part, long long cap, PcgScalars *sc, const double *pa, int npa) {
  if (sc->done) return;
  const int tid = threadIdx.y * TX + threadIdx.x;
  double alpha;
  if (FUSE) {
    if (!pcg_alpha(pa, npa, sc, blockIdx.x == 0, tid, &alpha)) return;
  } else {
    alpha = sc->alpha;
  }
  const __bf16 *g1 = g + d.n, *g2 = g + 2 * d.n, *g3 = g + 3 * d.n;
  double tt = 0.0, rr = 0.0;
  for_cells(d, [&](int i, int j, int k, long long c) {
    const double rn = rin[c] - alpha * y[c];
    x[c] = x[c] + alpha * p[c];
    rout[c] = rn;
    double v = (double)(float)g[c] * rn;
    if (i + 1 < d.n0) v += (double)(float)g1[c + d.n12] * (rin[c + d.n12] - alpha * y[c + d.n12]);
    if (j + 1 < d.n1) v += (double)(float)g2[c + d.n2] * (rin[c + d.n2] - alpha * y[c + d.n2]);
    if (k + 1 < d.n2) v += (double)(float)g3[c + 1] * (rin[c + 1] - alpha * y[c + 1]);
    t[c] = v;
    tt += v * v;
    rr += rn * rn;
  });
  const int w = wg_index(d.rev);
  wg_sum2<NT>(tt, rr, tid, part + w, part + cap + w);
}

int grid_items(const PcDims &d) { return (int)(d.items < 2048 ? d.items : 2048); }

}  // namespace

int pc_parts(const sts_ctx *c) { return grid_items(dims_of(c)); }

void launch_pc_gt(const sts_ctx *c, const void *g, const double *x, const double *sub,
                  double *t, const PcgScalars *sc) {
  STS_PROF(c, "launch_pc_gt");
  const PcDims d = dims_of(c);
  hipLaunchKernelGGL(k_pc_gt, dim3(grid_items(d)), dim3(TX, TY), 0, c->stream, d,
                     (const __bf16 *)g, x, sub, t, sc);
}

void launch_pc_g(const sts_ctx *c, const void *g, const double *t, double *z,
                 const PcgScalars *sc) {
  STS_PROF(c, "launch_pc_g");
  const PcDims d = dims_of(c);
  hipLaunchKernelGGL(k_pc_g, dim3(grid_items(d)), dim3(TX, TY), 0, c->stream, d,
                     (const __bf16 *)g, t, z, sc);
}

void launch_pc_build(const sts_ctx *c, double dt, const float *o4, void *g, int *bad) {
  STS_PROF(c, "launch_pc_build");
  const PcDims d = dims_of(c);
  hipLaunchKernelGGL(k_pc_build, dim3(grid_items(d)), dim3(TX, TY), 0, c->stream, d, c->grid(),
                     (const double *)c->d_sdiag, dt, o4, (__bf16 *)g, bad);
}

void launch_pc_check(const sts_ctx *c, const float *g32, void *g, int *bad) {
  STS_PROF(c, "launch_pc_check");
  const PcDims d = dims_of(c);
  hipLaunchKernelGGL(k_pc_check, dim3(grid_items(d)), dim3(TX, TY), 0, c->stream, d, g32,
                     (__bf16 *)g, bad);
}

void launch_pc_pack(const sts_ctx *c, double dt, double lscale, const double *T, double tsh,
                    double tsc, void *x) {
  STS_PROF(c, "launch_pc_pack");
  const PcDims d = dims_of(c);
  hipLaunchKernelGGL(k_pc_pack, dim3(grid_items(d)), dim3(TX, TY), 0, c->stream, d, c->grid(),
                     (const double *)c->d_sdiag, dt, lscale, T, tsh, tsc, (__bf16 *)x);
}

void launch_pc_grad(const sts_ctx *c, double dt, const void *g, const double *y,
                    const double *r, const double *s, const double *z, double *dg, void *dout,
                    double *part) {
  STS_PROF(c, "launch_pc_grad");
  const PcDims d = dims_of(c);
  hipLaunchKernelGGL(k_pc_grad, dim3(grid_items(d)), dim3(TX, TY), 0, c->stream, d, c->grid(),
                     (const double *)c->d_sdiag, dt, (const __bf16 *)g, y, r, s, z, dg,
                     (__bf16 *)dout, part);
}

void launch_pc_xr_gt(const sts_ctx *c, const void *g, double *x, const double *p,
                     const double *rin, double *rout, const double *y, double *t, double *part,
                     PcgScalars *sc, const double *pa, int npa) {
  STS_PROF(c, "launch_pc_xr_gt");
  const PcDims d = dims_of(c);
  if (pa)
    hipLaunchKernelGGL(k_pc_xr_gt<true>, dim3(grid_items(d)), dim3(TX, TY), 0, c->stream, d,
                       (const __bf16 *)g, x, p, rin, rout, y, t, part, (long long)c->red_cap, sc,
                       pa, npa);
  else
    hipLaunchKernelGGL(k_pc_xr_gt<false>, dim3(grid_items(d)), dim3(TX, TY), 0, c->stream, d,
                       (const __bf16 *)g, x, p, rin, rout, y, t, part, (long long)c->red_cap, sc,
                       (const double *)nullptr, 0);
}


}  // namespace sts
