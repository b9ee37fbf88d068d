// Backward Euler + preconditioned conjugate gradients (Sec. 2, Fig. "pcg").
//
// The system is A x = b with A = V - dt S (symmetric positive definite) and
// b = V u^n + dt g.  Per iteration two fused sweeps replace the figure's
// separate matvec, axpys and preconditioner application:
//   pass A: p = z + beta p_old (z recomputed at every stencil point, so p
//           needs no separate sweep), y = A p, partial sums of p . y;
//   alpha = r.z / p.y                     (one workgroup, on the device)
//   pass B: x += alpha p, r -= alpha y, z = P^-1 r, partial sums r.z, r.r;
//   beta = r.z / r_old.z_old and the convergence test ||r|| <= rtol ||b||
//                                         (one workgroup, on the device).
// alpha and beta never leave the device.  Once the device flag `done` is set
// every later kernel returns at once, so the host may enqueue iterations in
// batches and the result is the iterate at convergence.
#include "k_common.h"
#include "k_reduce.h"

namespace sts {

namespace {

constexpr int TX = 64, TY = 4, NT = TX * TY;

__device__ __forceinline__ double g_term(const Grid &g, const Coef &C, int i, int j, int k) {
  double t = 0.0;
  const int b = j * g.n2 + k;
  if (g.dir_lo && i == 0) t += C.wb_lo[b] * C.ub_lo[b];
  if (g.dir_hi && i == g.n0 - 1) t += C.wb_hi[b] * C.ub_hi[b];
  return t;
}

template <int OP>
__global__ void __launch_bounds__(NT)
    k_be_rhs(Grid g, Coef C, const double *__restrict__ un, double dt,
             const double *__restrict__ sdiag, double *__restrict__ b,
             double *__restrict__ invd) {
  const int k = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int i = blockIdx.z;
  if (k < g.n2 && j < g.n1) {
    const int c = lin(g, i, j, k);
    const double V = vol(g, i, j, k);
    b[c] = V * un[c] + dt * g_term(g, C, i, j, k);
    invd[c] = 1.0 / (V - dt * sdiag[c]);
  }
}

// p = z (z = invd r for Jacobi, or the given z); partial sums r . z.
// zout (may be null) receives the Jacobi z.
__global__ void __launch_bounds__(NT)
    k_init_p(long long n, const double *__restrict__ r, const double *__restrict__ invd,
             const double *__restrict__ zilu, double *__restrict__ p, double *part,
             double *__restrict__ zout, int rev) {
  double rz = 0.0;
  const long long stride = (long long)gridDim.x * NT;
  const int w = wg_index(rev);
  for (long long c = (long long)w * NT + threadIdx.x; c < n; c += stride) {
    const double z = zilu ? zilu[c] : r[c] * invd[c];
    if (zout) zout[c] = z;
    p[c] = z;
    rz += r[c] * z;
  }
  wg_sum2<NT>(rz, 0.0, threadIdx.x, part + w, nullptr);
}

__global__ void k_fin_init(const double *pb, int nb, const double *prr, int nrr,
                           const double *prz, int nrz, PcgScalars *sc, double rtol, int maxit) {
  __shared__ double s_b, s_r, s_z;
  block_sum_parts(pb, nb, 0, &s_b, nullptr);
  __syncthreads();
  block_sum_parts(prr, nrr, 0, &s_r, nullptr);
  __syncthreads();
  block_sum_parts(prz, nrz, 0, &s_z, nullptr);
  __syncthreads();
  if (threadIdx.x == 0) {
    sc->bnorm2 = s_b;
    sc->rnorm2 = s_r;
    sc->rr = s_z;
    sc->rr_old = s_z;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->py = 0.0;
    sc->tol2 = rtol * rtol * s_b;
    sc->iters = 0;
    sc->maxit = maxit;
    sc->status = 0;
    sc->done = 0;
    if (!(s_r > sc->tol2)) {  // already converged (or b = 0)
      sc->done = 1;
      sc->status = 1;
    } else if (!isfinite(s_r) || !isfinite(s_z)) {
      sc->done = 1;
      sc->status = -4;
    } else if (maxit <= 0) {
      sc->done = 1;
    }
  }
}

__global__ void k_fin_alpha(const double *part, int n, PcgScalars *sc) {
  if (sc->done) return;
  __shared__ double s;
  block_sum_parts(part, n, 0, &s, nullptr);
  __syncthreads();
  if (threadIdx.x == 0) {
    sc->py = s;
    if (!(s > 0.0) || !isfinite(s)) {
      sc->done = 1;
      sc->status = -4;
    } else {
      sc->alpha = sc->rr / s;
    }
  }
}

// Grid-stride over the cells with a bounded number of workgroups, so the
// partial sums stay few.  FUSE: alpha is formed here from pass A's partials
// pa[0..npa) by every workgroup (pcg_alpha), workgroup 0 recording it.
template <bool FUSE>
__global__ void __launch_bounds__(NT)
    k_pass_b_jac(long long n, double *__restrict__ x, const double *__restrict__ p,
                 double *__restrict__ r, const double *__restrict__ y,
                 const double *__restrict__ invd, double *__restrict__ zout, double *part,
                 long long cap, PcgScalars *sc, const double *pa, int npa, int rev) {
  if (sc->done) return;
  double alpha;
  if (FUSE) {
    if (!pcg_alpha(pa, npa, sc, blockIdx.x == 0, (int)threadIdx.x, &alpha)) return;
  } else {
    alpha = sc->alpha;
  }
  double rz = 0.0, rr = 0.0;
  const long long stride = (long long)gridDim.x * NT;
  const int w = wg_index(rev);
  for (long long c = (long long)w * NT + threadIdx.x; c < n; c += stride) {
    x[c] = x[c] + alpha * p[c];
    const double rn = r[c] - alpha * y[c];
    r[c] = rn;
    const double zn = rn * invd[c];
    // the stored z lets the next pass A read two arrays per halo plane
    // (z, p) instead of three (r, 1/A_ii, p)
    if (zout) zout[c] = zn;
    rz += rn * zn;
    rr += rn * rn;
  }
  wg_sum2<NT>(rz, rr, threadIdx.x, part + w, part + cap + w);
}

__global__ void k_fin_beta(const double *part, int n, long long cap, PcgScalars *sc) {
  if (sc->done) return;
  __shared__ double s_z, s_r;
  block_sum_parts(part, n, cap, &s_z, &s_r);
  __syncthreads();
  if (threadIdx.x == 0) {
    sc->rr_old = sc->rr;
    sc->rr = s_z;
    sc->rnorm2 = s_r;
    sc->iters += 1;
    if (!isfinite(s_r) || !isfinite(s_z)) {
      sc->done = 1;
      sc->status = -4;
    } else if (!(s_r > sc->tol2)) {
      sc->done = 1;
      sc->status = 1;
    } else if (sc->iters >= sc->maxit) {
      sc->done = 1;
    } else {
      sc->beta = s_z / sc->rr_old;
    }
  }
}

// The end-of-iteration test of the last fused Jacobi-PCG iteration, which
// has no following sweep to evaluate it.
__global__ void k_fin_check(const double *part, int n, long long cap, int iters, PcgScalars *sc) {
  if (sc->done) return;
  double beta;
  pcg_decide(part, n, cap, iters, sc, true, (int)threadIdx.x, &beta);
}

// FP32 form inner solve: r = (float) r64, 1/A_ii in FP32, e = 0, p = z;
// partial sums r.z (region 0) and r.r (region 1).
__global__ void __launch_bounds__(NT)
    k_f32_init(long long n, const double *__restrict__ r64, const double *__restrict__ invd64,
               float *__restrict__ r, float *__restrict__ invd, float *__restrict__ e,
               float *__restrict__ z, double *part, long long cap) {
  double rz = 0.0, rr = 0.0;
  const long long stride = (long long)gridDim.x * NT;
  for (long long c = (long long)blockIdx.x * NT + threadIdx.x; c < n; c += stride) {
    const float rv = (float)r64[c], iv = (float)invd64[c];
    r[c] = rv;
    invd[c] = iv;
    e[c] = 0.0f;
    const float zv = rv * iv;
    z[c] = zv;
    rz += (double)rv * (double)zv;
    rr += (double)rv * (double)rv;
  }
  wg_sum2<NT>(rz, rr, threadIdx.x, part + blockIdx.x, part + cap + blockIdx.x);
}

// FUSE: alpha from pass A's partials pa[0..npa) in every workgroup (pcg_alpha).
template <bool FUSE>
__global__ void __launch_bounds__(NT)
    k_f32_pass_b(long long n, float *__restrict__ e, const float *__restrict__ p,
                 float *__restrict__ r, const float *__restrict__ y,
                 const float *__restrict__ invd, float *__restrict__ z, double *part,
                 long long cap, PcgScalars *sc, const double *pa, int npa) {
  if (sc->done) return;
  double a64;
  if (FUSE) {
    if (!pcg_alpha(pa, npa, sc, blockIdx.x == 0, (int)threadIdx.x, &a64)) return;
  } else {
    a64 = sc->alpha;
  }
  const float alpha = (float)a64;
  double rz = 0.0, rr = 0.0;
  const long long stride = (long long)gridDim.x * NT;
  for (long long c = (long long)blockIdx.x * NT + threadIdx.x; c < n; c += stride) {
    e[c] = e[c] + alpha * p[c];
    const float rn = r[c] - alpha * y[c];
    r[c] = rn;
    const float zn = rn * invd[c];
    z[c] = zn;
    rz += (double)rn * (double)zn;
    rr += (double)rn * (double)rn;
  }
  wg_sum2<NT>(rz, rr, threadIdx.x, part + blockIdx.x, part + cap + blockIdx.x);
}

__global__ void __launch_bounds__(NT) k_f32_add(long long n, double *__restrict__ x,
                                                const float *__restrict__ e) {
  const long long stride = (long long)gridDim.x * NT;
  for (long long c = (long long)blockIdx.x * NT + threadIdx.x; c < n; c += stride)
    x[c] = x[c] + (double)e[c];
}

__global__ void k_fill_f32(float *p, long long n, float v) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_sum2(const double *part, int n, long long cap, double *out) {
  __shared__ double a, b;
  block_sum_parts(part, n, cap, &a, &b);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

int rev_of(const sts_ctx *c) { return (c->debug & STS_DEBUG_WG_REVERSE) ? 1 : 0; }

dim3 grid3(const sts_ctx *c) {
  return dim3((c->n2 + TX - 1) / TX, (c->n1 + TY - 1) / TY, c->n0);
}

long long cap_of(const sts_ctx *c) { return c->red_cap; }

}  // namespace

int pcg_parts(const sts_ctx *c) {
  const long long n3 = stencil_parts(c);
  const long long n1 = (c->ncell + NT - 1) / NT;
  return (int)(n3 > n1 ? n3 : n1);
}

void launch_be_rhs(const sts_ctx *c, const double *u_n, double dt, double *b, double *invd,
                   double *part) {
  STS_PROF(c, "launch_be_rhs");
  if (c->op == OP_SPITZER)
    hipLaunchKernelGGL(k_be_rhs<OP_SPITZER>, grid3(c), dim3(TX, TY), 0, c->stream, c->grid(),
                       c->coef(), u_n, dt, c->d_sdiag, b, invd);
  else
    hipLaunchKernelGGL(k_be_rhs<OP_ISOTROPIC>, grid3(c), dim3(TX, TY), 0, c->stream,
                       c->grid(), c->coef(), u_n, dt, c->d_sdiag, b, invd);
}

void launch_init_p(const sts_ctx *c, const double *r, const double *invd, const double *zilu,
                   double *p, double *part, double *zout) {
  STS_PROF(c, "launch_init_p");
  const long long n = c->ncell;
  hipLaunchKernelGGL(k_init_p, dim3(pass_b_parts(c)), dim3(NT), 0, c->stream, n,
                     r, invd, zilu, p, part, zout, rev_of(c));
}

void launch_finalize_init_n(const sts_ctx *c, const double *pb, int nb, const double *prr,
                            int nrr, const double *prz, int nrz, PcgScalars *sc, double rtol,
                            int maxit) {
  STS_PROF(c, "launch_finalize_init_n");
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(256), 0, c->stream, pb, nb, prr, nrr, prz, nrz, sc,
                     rtol, maxit);
}

void launch_finalize_init3(const sts_ctx *c, const double *pb, const double *prr,
                           const double *prz, PcgScalars *sc, double rtol, int maxit) {
  STS_PROF(c, "launch_finalize_init3");
  const int n3 = stencil_parts(c);
  const int n1 = pass_b_parts(c);
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(256), 0, c->stream, pb, n3, prr, n3, prz, n1, sc,
                     rtol, maxit);
}

void launch_init_p_n(const sts_ctx *c, long long n, const double *r, const double *invd,
                     double *p, double *part, int nparts) {
  STS_PROF(c, "launch_init_p_n");
  hipLaunchKernelGGL(k_init_p, dim3(nparts), dim3(NT), 0, c->stream, n, r, invd,
                     (const double *)nullptr, p, part, (double *)nullptr, rev_of(c));
}

void launch_pass_b_jacobi_n(const sts_ctx *c, long long n, double *x, const double *p, double *r,
                            const double *y, const double *invd, double *part, int nparts,
                            const PcgScalars *sc, const double *pa, int npa) {
  STS_PROF(c, "launch_pass_b_jacobi_n");
  PcgScalars *s = const_cast<PcgScalars *>(sc);
  if (pa)
    hipLaunchKernelGGL(k_pass_b_jac<true>, dim3(nparts), dim3(NT), 0, c->stream, n, x, p, r, y,
                       invd, (double *)nullptr, part, cap_of(c), s, pa, npa, rev_of(c));
  else
    hipLaunchKernelGGL(k_pass_b_jac<false>, dim3(nparts), dim3(NT), 0, c->stream, n, x, p, r, y,
                       invd, (double *)nullptr, part, cap_of(c), s, (const double *)nullptr, 0,
                       rev_of(c));
}

void launch_finalize_alpha(const sts_ctx *c, const double *part, int, PcgScalars *sc) {
  STS_PROF(c, "launch_finalize_alpha");
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(256), 0, c->stream, part, stencil_parts(c), sc);
}

void launch_pass_b_jacobi_fused(const sts_ctx *c, double *x, const double *p, double *r,
                                const double *y, const double *invd, double *z, double *part,
                                PcgScalars *sc, const double *pa, int npa) {
  STS_PROF(c, "launch_pass_b_jacobi_fused");
  hipLaunchKernelGGL(k_pass_b_jac<true>, dim3(pass_b_parts(c)), dim3(NT), 0, c->stream, c->ncell,
                     x, p, r, y, invd, z, part, cap_of(c), sc, pa, npa, rev_of(c));
}

void launch_pass_b_jacobi(const sts_ctx *c, double *x, const double *p, double *r,
                          const double *y, const double *invd, double *z, double *part,
                          PcgScalars *sc) {
  STS_PROF(c, "launch_pass_b_jacobi");
  hipLaunchKernelGGL(k_pass_b_jac<false>, dim3(pass_b_parts(c)), dim3(NT), 0, c->stream,
                     c->ncell, x, p, r, y, invd, z, part, cap_of(c), sc, (const double *)nullptr,
                     0, rev_of(c));
}

void launch_finalize_check(const sts_ctx *c, const double *part, int nparts, int iters,
                           PcgScalars *sc) {
  STS_PROF(c, "launch_finalize_check");
  hipLaunchKernelGGL(k_fin_check, dim3(1), dim3(256), 0, c->stream, part, nparts, cap_of(c), iters,
                     sc);
}

void launch_finalize_beta(const sts_ctx *c, const double *part, int nparts, PcgScalars *sc) {
  STS_PROF(c, "launch_finalize_beta");
  hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(256), 0, c->stream, part, nparts, cap_of(c), sc);
}

int pass_b_parts(const sts_ctx *c) {
  const long long n = (c->ncell + NT - 1) / NT;
  return (int)(n < 2048 ? n : 2048);
}

void launch_sum2(const sts_ctx *c, const double *part, int nparts, double *out2) {
  STS_PROF(c, "launch_sum2");
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, c->stream, part, nparts, cap_of(c), out2);
}


}  // namespace sts

namespace sts {

void f32_inner_init(const sts_ctx *c, const double *r64, const double *invd64, float *r,
                    float *invd, float *e, float *z, double *part) {
  STS_PROF(c, "f32_inner_init");
  hipLaunchKernelGGL(k_f32_init, dim3(pass_b_parts(c)), dim3(NT), 0, c->stream, c->ncell, r64,
                     invd64, r, invd, e, z, part, (long long)c->red_cap);
}

void f32_pass_b(const sts_ctx *c, float *e, const float *p, float *r, const float *y,
                const float *invd, float *z, double *part, const PcgScalars *sc,
                const double *pa, int npa) {
  STS_PROF(c, "f32_pass_b");
  PcgScalars *s = const_cast<PcgScalars *>(sc);
  if (pa)
    hipLaunchKernelGGL(k_f32_pass_b<true>, dim3(pass_b_parts(c)), dim3(NT), 0, c->stream,
                       c->ncell, e, p, r, y, invd, z, part, (long long)c->red_cap, s, pa, npa);
  else
    hipLaunchKernelGGL(k_f32_pass_b<false>, dim3(pass_b_parts(c)), dim3(NT), 0, c->stream,
                       c->ncell, e, p, r, y, invd, z, part, (long long)c->red_cap, s,
                       (const double *)nullptr, 0);
}

void f32_add_to(const sts_ctx *c, double *x, const float *e) {
  STS_PROF(c, "f32_add_to");
  hipLaunchKernelGGL(k_f32_add, dim3(pass_b_parts(c)), dim3(NT), 0, c->stream, c->ncell, x, e);
}

void launch_fill_f32(const sts_ctx *c, float *p, long long n, float v) {
  STS_PROF(c, "launch_fill_f32");
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, p,
                     n, v);
}

}  // namespace sts
