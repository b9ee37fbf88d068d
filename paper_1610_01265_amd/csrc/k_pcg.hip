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

__device__ __forceinline__ int wg_id3() {
  return (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

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
             double *__restrict__ invd, double *part) {
  const int k = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int i = blockIdx.z;
  const int tid = threadIdx.y * TX + threadIdx.x;
  double bb = 0.0;
  if (k < g.n2 && j < g.n1) {
    const int c = lin(g, i, j, k);
    const double V = vol(g, i, j, k);
    const double v = V * un[c] + dt * g_term(g, C, i, j, k);
    b[c] = v;
    invd[c] = 1.0 / (V - dt * sdiag[c]);
    bb = v * v;
  }
  wg_sum2<NT>(bb, 0.0, tid, part + wg_id3(), nullptr);
}

// r = b - A x; partial sums of r . r.  WRITE = false: norms only.
template <int OP, bool WRITE>
__global__ void __launch_bounds__(NT)
    k_resid(Grid g, Coef C, const double *__restrict__ b, const double *__restrict__ x, double dt,
            double *__restrict__ r, double *part, long long cap) {
  const int k = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int i = blockIdx.z;
  const int tid = threadIdx.y * TX + threadIdx.x;
  double rr = 0.0, bb = 0.0;
  if (k < g.n2 && j < g.n1) {
    const int c = lin(g, i, j, k);
    const ArrayField f{x};
    const double su = (OP == OP_SPITZER) ? s19<false>(g, C, f, i, j, k)
                                         : s7<false>(g, C, f, i, j, k);
    const double ax = vol(g, i, j, k) * x[c] - dt * su;
    const double rv = b[c] - ax;
    if (WRITE) r[c] = rv;
    rr = rv * rv;
    bb = b[c] * b[c];
  }
  const int w = wg_id3();
  wg_sum2<NT>(rr, bb, tid, part + w, part + cap + w);
}

// p = z (z = invd r for Jacobi, or the given z); partial sums r . z
__global__ void __launch_bounds__(NT)
    k_init_p(long long n, const double *__restrict__ r, const double *__restrict__ invd,
             const double *__restrict__ zilu, double *__restrict__ p, double *part) {
  const long long c = (long long)blockIdx.x * NT + threadIdx.x;
  double rz = 0.0;
  if (c < n) {
    const double z = zilu ? zilu[c] : invd[c] * r[c];
    p[c] = z;
    rz = r[c] * z;
  }
  wg_sum2<NT>(rz, 0.0, threadIdx.x, part + blockIdx.x, nullptr);
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

// z at a stencil point: Jacobi (r / A_ii) or a stored block-ILU0 result.
template <int PC>
struct PField {
  const double *__restrict__ r;
  const double *__restrict__ invd;
  const double *__restrict__ zilu;
  const double *__restrict__ pold;
  double beta;
  __device__ __forceinline__ double operator()(int idx) const {
    const double z = (PC == STS_PC_JACOBI) ? r[idx] * invd[idx] : zilu[idx];
    return pold ? z + beta * pold[idx] : z;
  }
};

template <int OP, int PC>
__global__ void __launch_bounds__(NT)
    k_pass_a(Grid g, Coef C, double dt, const double *__restrict__ r,
             const double *__restrict__ invd, const double *__restrict__ zilu,
             const double *__restrict__ pold, double *__restrict__ pnew,
             double *__restrict__ y, double *part, const PcgScalars *sc, int first) {
  if (sc->done) return;
  const int k = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int i = blockIdx.z;
  const int tid = threadIdx.y * TX + threadIdx.x;
  double py = 0.0;
  if (k < g.n2 && j < g.n1) {
    const PField<PC> f{r, invd, zilu, first ? nullptr : pold, first ? 0.0 : sc->beta};
    const int c = lin(g, i, j, k);
    const double pc = f(c);
    const double su = (OP == OP_SPITZER) ? s19<false>(g, C, f, i, j, k)
                                         : s7<false>(g, C, f, i, j, k);
    const double yc = vol(g, i, j, k) * pc - dt * su;
    pnew[c] = pc;
    y[c] = yc;
    py = pc * yc;
  }
  wg_sum2<NT>(py, 0.0, tid, part + wg_id3(), nullptr);
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

__global__ void __launch_bounds__(NT)
    k_pass_b_jac(long long n, double *__restrict__ x, const double *__restrict__ p,
                 double *__restrict__ r, const double *__restrict__ y,
                 const double *__restrict__ invd, double *part, long long cap,
                 const PcgScalars *sc) {
  if (sc->done) return;
  const double alpha = sc->alpha;
  const long long c = (long long)blockIdx.x * NT + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (c < n) {
    x[c] = x[c] + alpha * p[c];
    const double rn = r[c] - alpha * y[c];
    r[c] = rn;
    const double z = rn * invd[c];
    rz = rn * z;
    rr = rn * rn;
  }
  wg_sum2<NT>(rz, rr, threadIdx.x, part + blockIdx.x, part + cap + blockIdx.x);
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

__global__ void k_sum2(const double *part, int n, long long cap, double *out) {
  __shared__ double a, b;
  block_sum_parts(part, n, cap, &a, &b);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

dim3 grid3(const sts_ctx *c) {
  return dim3((c->n2 + TX - 1) / TX, (c->n1 + TY - 1) / TY, c->n0);
}

long long cap_of(const sts_ctx *c) { return c->red_cap; }

}  // namespace

int pcg_parts(const sts_ctx *c) {
  const dim3 g = grid3(c);
  const long long n3 = (long long)g.x * g.y * g.z;
  const long long n1 = (c->ncell + NT - 1) / NT;
  return (int)(n3 > n1 ? n3 : n1);
}

void launch_be_rhs(const sts_ctx *c, const double *u_n, double dt, double *b, double *invd,
                   double *part) {
  if (c->op == OP_SPITZER)
    hipLaunchKernelGGL(k_be_rhs<OP_SPITZER>, grid3(c), dim3(TX, TY), 0, c->stream, c->grid(),
                       c->coef(), u_n, dt, c->d_sdiag, b, invd, part);
  else
    hipLaunchKernelGGL(k_be_rhs<OP_ISOTROPIC>, grid3(c), dim3(TX, TY), 0, c->stream,
                       c->grid(), c->coef(), u_n, dt, c->d_sdiag, b, invd, part);
}

// r = b - A x (part region 0: r.r), then p = z (part region 2: r.z) and the
// initial scalars (b.b from region 1 of the rhs launch).
void launch_residual_init(const sts_ctx *c, const double *b, const double *x, double dt,
                          const double *invd, const double *zilu, double *r, double *p,
                          double *part) {
  const long long cap = cap_of(c);
  if (c->op == OP_SPITZER)
    hipLaunchKernelGGL((k_resid<OP_SPITZER, true>), grid3(c), dim3(TX, TY), 0, c->stream,
                       c->grid(), c->coef(), b, x, dt, r, part, cap);
  else
    hipLaunchKernelGGL((k_resid<OP_ISOTROPIC, true>), grid3(c), dim3(TX, TY), 0, c->stream,
                       c->grid(), c->coef(), b, x, dt, r, part, cap);
  (void)invd;
  (void)zilu;
  (void)p;
}

void launch_init_p(const sts_ctx *c, const double *r, const double *invd, const double *zilu,
                   double *p, double *part) {
  const long long n = c->ncell;
  hipLaunchKernelGGL(k_init_p, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, c->stream, n,
                     r, invd, zilu, p, part);
}

void launch_finalize_init3(const sts_ctx *c, const double *pb, const double *prr,
                           const double *prz, PcgScalars *sc, double rtol, int maxit) {
  const dim3 g = grid3(c);
  const int n3 = (int)(g.x * g.y * g.z);
  const int n1 = (int)((c->ncell + NT - 1) / NT);
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(256), 0, c->stream, pb, n3, prr, n3, prz, n1, sc,
                     rtol, maxit);
}

void launch_pass_a(const sts_ctx *c, double dt, const double *r, const double *invd,
                   const double *zilu, const double *pold, double *pnew, double *y, double *part,
                   const PcgScalars *sc, int first) {
  const dim3 g = grid3(c), b(TX, TY);
  if (c->op == OP_SPITZER) {
    if (zilu)
      hipLaunchKernelGGL((k_pass_a<OP_SPITZER, STS_PC_BLOCK_ILU0>), g, b, 0, c->stream,
                         c->grid(), c->coef(), dt, r, invd, zilu, pold, pnew, y, part, sc, first);
    else
      hipLaunchKernelGGL((k_pass_a<OP_SPITZER, STS_PC_JACOBI>), g, b, 0, c->stream, c->grid(),
                         c->coef(), dt, r, invd, zilu, pold, pnew, y, part, sc, first);
  } else {
    if (zilu)
      hipLaunchKernelGGL((k_pass_a<OP_ISOTROPIC, STS_PC_BLOCK_ILU0>), g, b, 0, c->stream,
                         c->grid(), c->coef(), dt, r, invd, zilu, pold, pnew, y, part, sc, first);
    else
      hipLaunchKernelGGL((k_pass_a<OP_ISOTROPIC, STS_PC_JACOBI>), g, b, 0, c->stream,
                         c->grid(), c->coef(), dt, r, invd, zilu, pold, pnew, y, part, sc, first);
  }
}

void launch_finalize_alpha(const sts_ctx *c, const double *part, int, PcgScalars *sc) {
  const dim3 g = grid3(c);
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(256), 0, c->stream, part,
                     (int)(g.x * g.y * g.z), sc);
}

void launch_pass_b_jacobi(const sts_ctx *c, double *x, const double *p, double *r,
                          const double *y, const double *invd, double *part,
                          const PcgScalars *sc) {
  const long long n = c->ncell;
  hipLaunchKernelGGL(k_pass_b_jac, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, c->stream,
                     n, x, p, r, y, invd, part, cap_of(c), sc);
}

void launch_finalize_beta(const sts_ctx *c, const double *part, int nparts, PcgScalars *sc) {
  hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(256), 0, c->stream, part, nparts, cap_of(c), sc);
}

int pass_b_parts(const sts_ctx *c) { return (int)((c->ncell + NT - 1) / NT); }

void launch_true_residual(const sts_ctx *c, const double *b, const double *x, double dt,
                          double *part) {
  const long long cap = cap_of(c);
  if (c->op == OP_SPITZER)
    hipLaunchKernelGGL((k_resid<OP_SPITZER, false>), grid3(c), dim3(TX, TY), 0, c->stream,
                       c->grid(), c->coef(), b, x, dt, (double *)nullptr, part, cap);
  else
    hipLaunchKernelGGL((k_resid<OP_ISOTROPIC, false>), grid3(c), dim3(TX, TY), 0, c->stream,
                       c->grid(), c->coef(), b, x, dt, (double *)nullptr, part, cap);
}

void launch_sum2(const sts_ctx *c, const double *part, int nparts, double *out2) {
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, c->stream, part, nparts, cap_of(c), out2);
}

int stencil_parts(const sts_ctx *c) {
  const dim3 g = grid3(c);
  return (int)(g.x * g.y * g.z);
}

}  // namespace sts
