// The operator application, as a 2.5D march over r-planes, fused with the
// consumer of F(u): the RKL2 stage recurrence, or the PCG matvec.
//
// A workgroup owns a TJ x TK (theta, phi) tile and walks a chunk of CI
// consecutive r-planes.  The stencil input (u_{k-1} for RKL2, p = z + beta p
// for PCG) is staged once per cell into a 4-plane LDS ring (tile + one halo
// cell on each side); the next-but-one plane is fetched from HBM while the
// current plane is computed, so one barrier per plane suffices.  The 6 face /
// edge coefficient arrays are read with unconditional loads (indices clamped
// inside the grid, terms of absent faces / edges masked), so the compiler can
// issue them together.  Geometry factors are products of per-axis tables:
// the r-factors are uniform over a plane (scalar loads), the theta / phi
// factors are loaded once per thread.
//
// RKL2 (Sec. 3, Fig. "rkl2"): stage k >= 2 writes
//   u_k = mu_k u_{k-1} + nu_k u_{k-2} + (1 - mu_k - nu_k) u_0
//         + mu~_k dt F(u_{k-1}) + gamma~_k dt F(u_0)
// in the same pass; u_{k-2}, u_0 and F(u_0) are read at the cell only, so u_k
// may overwrite u_{k-2} or u_0 in place.
#include "k_common.h"
#include "k_reduce.h"

namespace sts {

namespace {

#ifndef STS_MARCH_TJ
#define STS_MARCH_TJ 4
#endif
#ifndef STS_MARCH_WG
#define STS_MARCH_WG 2048
#endif
constexpr int TK = 64, TJ = STS_MARCH_TJ, NT = TK * TJ;
constexpr int HK = TK + 2, HJ = TJ + 2, PL = HK * HJ;  // one LDS plane (tile + halo)
constexpr int NLOAD = (PL + NT - 1) / NT;

enum { M_F = 0, M_RK1 = 1, M_RK = 2, M_PA = 3, M_RES = 4, M_RESN = 5 };

// Index along an axis for a position that may lie outside [0, n): periodic
// axes wrap (a tile may be wider than a short axis, so use a full modulo),
// others clamp.
__device__ __forceinline__ int wrapclamp(int x, int n, int per) {
  if (x >= 0 && x < n) return x;
  if (per) {
    const int m = x % n;
    return m < 0 ? m + n : m;
  }
  return x < 0 ? 0 : n - 1;
}

struct LoadU {
  const double *__restrict__ u;
  __device__ __forceinline__ void prepare() {}
  __device__ __forceinline__ double operator()(long long idx) const { return u[idx]; }
};

// p = z + beta p_old with z = r / A_ii (Jacobi) or a stored block-ILU0 z.
template <int PC>
struct LoadP {
  const double *__restrict__ r;
  const double *__restrict__ invd;
  const double *__restrict__ zilu;
  const double *__restrict__ pold;
  const PcgScalars *sc;
  int first;
  double beta;
  __device__ __forceinline__ void prepare() { beta = first ? 0.0 : sc->beta; }
  __device__ __forceinline__ double operator()(long long idx) const {
    const double z = (PC == STS_PC_JACOBI) ? r[idx] * invd[idx] : zilu[idx];
    return first ? z : z + beta * pold[idx];
  }
};

struct Args {
  double *out;         // F, u_k, p (pass A), r (residual)
  double *F0;          // RKL2 F(u_0)
  const double *ukm2;  // RKL2 u_{k-2}
  const double *u0;    // RKL2 u_0
  const double *b;     // residual: right-hand side
  double *y;           // pass A: A p
  double *part;        // per-workgroup partial sums (two regions of cap)
  long long cap;
  double mu, nu, mut_dt, gt_dt, dt;
  const PcgScalars *sc;
};

struct PlaneGeo {
  Nb A;
  double s00m, s00, s10m, s10, s10p, s20m, s20, s20p, v0;
  double a00m, a00;  // isotropic: A00[i-1], A00[i]
  double a10, a20;   // isotropic: A10[i], A20[i]
  int dIm;
};

struct ThreadGeo {
  Nb B, C;
  double t11m, t11, t21m, t21, t21p, t22m, t22, v12;
  double a01, a02, a01m, a11, a11m, a12, a21, a22, a22m;  // isotropic area factors
  int dJm, dKm;
};

// (S u)_c (+ g_c when WITH_G), u read through U(di, dj, dk).
template <int OP, bool WITH_G, class UF>
__device__ __forceinline__ double apply_S(const Grid &g, const Coef &C, const UF &U, int i, int j,
                                          int k, int c, const PlaneGeo &pg,
                                          const ThreadGeo &tg) {
  const double u0 = U(0, 0, 0);
  double acc;
  if (OP == OP_SPITZER) {
    // unconditional coefficient loads (all indices lie inside the grid)
    const int cA = c + pg.dIm, cB = c + tg.dJm, cC = c + tg.dKm;
    const double w0p = C.w0[c], w0m = C.w0[cA], w1p = C.w1[c], w1m = C.w1[cB];
    const double w2p = C.w2[c], w2m = C.w2[cC];
    const double K01[4] = {C.k01[c], C.k01[cA], C.k01[cB], C.k01[cA + tg.dJm]};
    const double K02[4] = {C.k02[c], C.k02[cA], C.k02[cC], C.k02[cA + tg.dKm]};
    const double K12[4] = {C.k12[c], C.k12[cB], C.k12[cC], C.k12[cB + tg.dKm]};
    acc = w0p * (U(1, 0, 0) - u0) + (pg.A.hm ? w0m : 0.0) * (U(-1, 0, 0) - u0);
    acc += w1p * (U(0, 1, 0) - u0) + (tg.B.hm ? w1m : 0.0) * (U(0, -1, 0) - u0);
    acc += w2p * (U(0, 0, 1) - u0) + (tg.C.hm ? w2m : 0.0) * (U(0, 0, -1) - u0);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int r = p + 2 * q;  // index into K**[]: (0,0), (1,0), (0,1), (1,1)
        // plane (0, 1)
        {
          const bool ex = (p ? pg.A.hm : pg.A.hp) && (q ? tg.B.hm : tg.B.hp);
          EdgeGeo e;
          e.ia0 = e.ia1 = p ? pg.s00m : pg.s00;
          const double tj = q ? tg.t11m : tg.t11;
          e.ib0 = (p ? pg.s10m : pg.s10) * tj;
          e.ib1 = (p ? pg.s10 : pg.s10p) * tj;
          acc += edge_term(ex ? K01[r] : 0.0, U(-p, -q, 0), U(1 - p, -q, 0), U(-p, 1 - q, 0),
                           U(1 - p, 1 - q, 0), e, p, q);
        }
        // plane (0, 2)
        {
          const bool ex = (p ? pg.A.hm : pg.A.hp) && (q ? tg.C.hm : tg.C.hp);
          EdgeGeo e;
          e.ia0 = e.ia1 = p ? pg.s00m : pg.s00;
          const double tk = q ? tg.t22m : tg.t22;
          e.ib0 = (p ? pg.s20m : pg.s20) * tg.t21 * tk;
          e.ib1 = (p ? pg.s20 : pg.s20p) * tg.t21 * tk;
          acc += edge_term(ex ? K02[r] : 0.0, U(-p, 0, -q), U(1 - p, 0, -q), U(-p, 0, 1 - q),
                           U(1 - p, 0, 1 - q), e, p, q);
        }
        // plane (1, 2)
        {
          const bool ex = (p ? tg.B.hm : tg.B.hp) && (q ? tg.C.hm : tg.C.hp);
          EdgeGeo e;
          e.ia0 = e.ia1 = pg.s10 * (p ? tg.t11m : tg.t11);
          const double tk = q ? tg.t22m : tg.t22;
          e.ib0 = pg.s20 * (p ? tg.t21m : tg.t21) * tk;
          e.ib1 = pg.s20 * (p ? tg.t21 : tg.t21p) * tk;
          acc += edge_term(ex ? K12[r] : 0.0, U(0, -p, -q), U(0, 1 - p, -q), U(0, -p, 1 - q),
                           U(0, 1 - p, 1 - q), e, p, q);
        }
      }
  } else {
    // nu * (area / distance) on each face, from the separable tables
    const double w0p = pg.a00 * tg.a01 * tg.a02 * pg.s00;
    const double w0m = pg.a00m * tg.a01 * tg.a02 * pg.s00m;
    const double w1p = pg.a10 * tg.a11 * tg.a12 * (pg.s10 * tg.t11);
    const double w1m = pg.a10 * tg.a11m * tg.a12 * (pg.s10 * tg.t11m);
    const double w2p = pg.a20 * tg.a21 * tg.a22 * (pg.s20 * tg.t21 * tg.t22);
    const double w2m = pg.a20 * tg.a21 * tg.a22m * (pg.s20 * tg.t21 * tg.t22m);
    acc = w0p * (U(1, 0, 0) - u0) + (pg.A.hm ? w0m : 0.0) * (U(-1, 0, 0) - u0);
    acc += w1p * (U(0, 1, 0) - u0) + (tg.B.hm ? w1m : 0.0) * (U(0, -1, 0) - u0);
    acc += w2p * (U(0, 0, 1) - u0) + (tg.C.hm ? w2m : 0.0) * (U(0, 0, -1) - u0);
    acc *= C.nu;
  }
  if ((g.dir_lo && i == 0) || (g.dir_hi && i == g.n0 - 1)) {
    const int bi = j * g.n2 + k;
    const bool lo = g.dir_lo && i == 0;
    const double wb = lo ? C.wb_lo[bi] : C.wb_hi[bi];
    const double ub = lo ? C.ub_lo[bi] : C.ub_hi[bi];
    acc += WITH_G ? wb * (ub - u0) : -wb * u0;
    if (g.dir_lo && g.dir_hi && i == 0 && i == g.n0 - 1) {  // single radial cell
      acc += WITH_G ? C.wb_hi[bi] * (C.ub_hi[bi] - u0) : -C.wb_hi[bi] * u0;
    }
  }
  return acc;
}

template <int OP, int MODE, class Loader>
__global__ void __launch_bounds__(NT)
    k_march(Grid g, Coef C, Loader ld, Args a, int CI, int nchunk, long long ncell) {
  if (MODE == M_PA && a.sc->done) return;
  __shared__ double s_u[4][PL];
  ld.prepare();
  const int tk = threadIdx.x, tj = threadIdx.y, tid = tj * TK + tk;
  // XCD-aware order: workgroup w runs on XCD w % 8; each XCD gets a
  // contiguous range of the logical (chunk, row-tile, column-tile) order.
  const int nwg = gridDim.x, w = blockIdx.x;
  const int q8 = nwg >> 3, r8 = nwg & 7, x8 = w & 7, s8 = w >> 3;
  const int L = x8 < r8 ? x8 * (q8 + 1) + s8 : r8 * (q8 + 1) + (x8 - r8) * q8 + s8;
  const int ntk = (g.n2 + TK - 1) / TK, ntj = (g.n1 + TJ - 1) / TJ;
  const int bx = L % ntk, by = (L / ntk) % ntj, bz = L / (ntk * ntj);
  const int k0 = bx * TK, j0 = by * TJ;
  const int comp = bz / nchunk, chunk = bz - comp * nchunk;
  const int i0 = chunk * CI, i1 = min(i0 + CI, g.n0);
  const long long off = (long long)comp * ncell;
  const long long n12 = (long long)g.n1 * g.n2;

  // fixed in-plane source offsets of this thread's halo-tile loads
  int hoff[NLOAD];
#pragma unroll
  for (int q = 0; q < NLOAD; ++q) {
    const int e = min(tid + q * NT, PL - 1);
    const int hj = e / HK, hk = e - hj * HK;
    hoff[q] = wrapclamp(j0 - 1 + hj, g.n1, g.per1) * g.n2 + wrapclamp(k0 - 1 + hk, g.n2, g.per2);
  }
  auto load_plane = [&](int ip, double *v) {
    const long long base = off + (long long)wrapclamp(ip, g.n0, g.per0) * n12;
#pragma unroll
    for (int q = 0; q < NLOAD; ++q) v[q] = ld(base + hoff[q]);
  };
  auto store_plane = [&](int ip, const double *v) {
    double *s = s_u[ip & 3];
#pragma unroll
    for (int q = 0; q < NLOAD; ++q)
      if (tid + q * NT < PL) s[tid + q * NT] = v[q];
  };
  double v[NLOAD];
  load_plane(i0 - 1, v);
  store_plane(i0 - 1, v);
  load_plane(i0, v);
  store_plane(i0, v);
  load_plane(i0 + 1, v);
  store_plane(i0 + 1, v);

  const int j = j0 + tj, k = k0 + tk;
  const bool active = j < g.n1 && k < g.n2;
  const int jc = min(j, g.n1 - 1), kc = min(k, g.n2 - 1);
  ThreadGeo tg;
  tg.B = nbr(jc, g.n1, g.per1);
  tg.C = nbr(kc, g.n2, g.per2);
  tg.t11m = T1(g, T_IL11, tg.B.m);
  tg.t11 = T1(g, T_IL11, jc);
  tg.t21m = T1(g, T_IL21, tg.B.m);
  tg.t21 = T1(g, T_IL21, jc);
  tg.t21p = T1(g, T_IL21, tg.B.p);
  tg.t22m = T2(g, T_IL22, tg.C.m);
  tg.t22 = T2(g, T_IL22, kc);
  tg.v12 = T1(g, T_V1, jc) * T2(g, T_V2, kc);
  tg.dJm = (tg.B.m - jc) * g.n2;
  tg.dKm = tg.C.m - kc;
  if (OP == OP_ISOTROPIC) {
    tg.a01 = T1(g, T_A01, jc);
    tg.a02 = T2(g, T_A02, kc);
    tg.a11 = T1(g, T_A11, jc);
    tg.a11m = T1(g, T_A11, tg.B.m);
    tg.a12 = T2(g, T_A12, kc);
    tg.a21 = T1(g, T_A21, jc);
    tg.a22 = T2(g, T_A22, kc);
    tg.a22m = T2(g, T_A22, tg.C.m);
  }
  double acc_a = 0.0, acc_b = 0.0;
  __syncthreads();

  for (int i = i0; i < i1; ++i) {
    const bool pre = i + 2 <= i1;
    if (pre) load_plane(i + 2, v);
    if (active) {
      PlaneGeo pg;
      pg.A = nbr(i, g.n0, g.per0);
      pg.s00m = T0(g, T_IL00, pg.A.m);
      pg.s00 = T0(g, T_IL00, i);
      pg.s10m = T0(g, T_IL10, pg.A.m);
      pg.s10 = T0(g, T_IL10, i);
      pg.s10p = T0(g, T_IL10, pg.A.p);
      pg.s20m = T0(g, T_IL20, pg.A.m);
      pg.s20 = T0(g, T_IL20, i);
      pg.s20p = T0(g, T_IL20, pg.A.p);
      pg.v0 = T0(g, T_V0, i);
      pg.dIm = (pg.A.m - i) * g.n1 * g.n2;
      if (OP == OP_ISOTROPIC) {
        pg.a00 = T0(g, T_A00, i);
        pg.a00m = T0(g, T_A00, pg.A.m);
        pg.a10 = T0(g, T_A10, i);
        pg.a20 = T0(g, T_A20, i);
      }
      const int base = (tj + 1) * HK + (tk + 1);
      const double *sm = s_u[(i - 1) & 3], *s0 = s_u[i & 3], *sp = s_u[(i + 1) & 3];
      auto U = [&](int di, int dj, int dk) -> double {
        const double *s = di < 0 ? sm : (di > 0 ? sp : s0);
        return s[base + dj * HK + dk];
      };
      const int c = (i * g.n1 + j) * g.n2 + k;
      const long long cc = off + c;
      const bool with_g = MODE == M_F || MODE == M_RK1 || MODE == M_RK;
      const double su = apply_S<OP, with_g>(g, C, U, i, j, k, c, pg, tg);
      const double V = pg.v0 * tg.v12;
      const double uc = s0[base];
      if (MODE == M_F) {
        a.out[cc] = su / V;
      } else if (MODE == M_RK1) {
        const double F = su / V;
        a.F0[cc] = F;
        a.out[cc] = uc + a.mut_dt * F;
      } else if (MODE == M_RK) {
        const double F = su / V;
        a.out[cc] = a.mu * uc + a.nu * a.ukm2[cc] + (1.0 - a.mu - a.nu) * a.u0[cc] +
                    a.mut_dt * F + a.gt_dt * a.F0[cc];
      } else if (MODE == M_PA) {
        const double yv = V * uc - a.dt * su;
        a.out[cc] = uc;
        a.y[cc] = yv;
        acc_a += uc * yv;
      } else {  // residual r = b - A x
        const double bv = a.b[cc];
        const double rv = bv - (V * uc - a.dt * su);
        if (MODE == M_RES) a.out[cc] = rv;
        acc_a += rv * rv;
        acc_b += bv * bv;
      }
    }
    if (pre) store_plane(i + 2, v);
    __syncthreads();
  }
  if (MODE == M_PA || MODE == M_RES || MODE == M_RESN)
    wg_sum2<NT>(acc_a, acc_b, tid, a.part + w, a.part + a.cap + w);
}

int chunk_of(const sts_ctx *c) {
  const long long tiles = (long long)((c->n2 + TK - 1) / TK) * ((c->n1 + TJ - 1) / TJ);
  long long ci = tiles * c->n0 / STS_MARCH_WG;
  if (ci < 1) ci = 1;
  if (ci > 16) ci = 16;
  return (int)ci;
}

dim3 march_grid(const sts_ctx *c, int ncomp, int *CI, int *nchunk) {
  *CI = chunk_of(c);
  *nchunk = (c->n0 + *CI - 1) / *CI;
  return dim3(((c->n2 + TK - 1) / TK) * ((c->n1 + TJ - 1) / TJ) * *nchunk * ncomp);
}

template <int OP, int MODE, class Loader>
void launch(const sts_ctx *c, int ncomp, const Loader &ld, const Args &a) {
  int CI, nchunk;
  const dim3 grid = march_grid(c, ncomp, &CI, &nchunk);
  hipLaunchKernelGGL((k_march<OP, MODE, Loader>), grid, dim3(TK, TJ), 0, c->stream, c->grid(),
                     c->coef(), ld, a, CI, nchunk, c->ncell);
}

#ifndef STS_GATHER19
#define STS_GATHER19 1
#endif

template <int MODE, class Loader>
void launch_op(const sts_ctx *c, int ncomp, const Loader &ld, const Args &a) {
  if (STS_GATHER19 && c->op == OP_SPITZER)
    launch<OP_SPITZER, MODE>(c, ncomp, ld, a);
  else
    launch<OP_ISOTROPIC, MODE>(c, ncomp, ld, a);
}

}  // namespace

// Conduction (19-point) runs the flux-form kernels of k_flux.hip; the
// isotropic 7-point operator runs the gather march below.
int flux_parts(const sts_ctx *c);
void flux_stage(const sts_ctx *c, int mode, int ncomp, const double *ukm1, const double *ukm2,
                const double *u0, double *F0, double *out, double mu, double nu, double mut_dt,
                double gt_dt);
void flux_pass_a(const sts_ctx *c, double dt, const double *r, const double *invd,
                 const double *zilu, const double *pold, double *pnew, double *y, double *part,
                 const PcgScalars *sc, int first);
void flux_residual(const sts_ctx *c, const double *b, const double *x, double dt, double *r,
                   double *part);

int stencil_parts(const sts_ctx *c) {
  if (c->op == OP_SPITZER && !STS_GATHER19) return flux_parts(c);
  int CI, nchunk;
  const dim3 g = march_grid(c, 1, &CI, &nchunk);
  return (int)(g.x * g.y * g.z);
}

void launch_stage(const sts_ctx *c, int mode, int ncomp, const double *ukm1, const double *ukm2,
                  const double *u0, double *F0, double *out, double mu, double nu, double mut_dt,
                  double gt_dt) {
  if (c->op == OP_SPITZER && !STS_GATHER19) {
    flux_stage(c, mode, ncomp, ukm1, ukm2, u0, F0, out, mu, nu, mut_dt, gt_dt);
    return;
  }
  Args a{};
  a.out = out;
  a.F0 = F0;
  a.ukm2 = ukm2;
  a.u0 = u0;
  a.mu = mu;
  a.nu = nu;
  a.mut_dt = mut_dt;
  a.gt_dt = gt_dt;
  const LoadU ld{ukm1};
  if (mode == 0)
    launch_op<M_F>(c, ncomp, ld, a);
  else if (mode == 1)
    launch_op<M_RK1>(c, ncomp, ld, a);
  else
    launch_op<M_RK>(c, ncomp, ld, a);
}

void launch_pass_a(const sts_ctx *c, double dt, const double *r, const double *invd,
                   const double *zilu, const double *pold, double *pnew, double *y, double *part,
                   const PcgScalars *sc, int first) {
  if (c->op == OP_SPITZER && !STS_GATHER19) {
    flux_pass_a(c, dt, r, invd, zilu, pold, pnew, y, part, sc, first);
    return;
  }
  Args a{};
  a.out = pnew;
  a.y = y;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  a.sc = sc;
  if (zilu) {
    const LoadP<STS_PC_BLOCK_ILU0> ld{r, invd, zilu, pold, sc, first, 0.0};
    launch_op<M_PA>(c, 1, ld, a);
  } else {
    const LoadP<STS_PC_JACOBI> ld{r, invd, zilu, pold, sc, first, 0.0};
    launch_op<M_PA>(c, 1, ld, a);
  }
}

void launch_residual_init(const sts_ctx *c, const double *b, const double *x, double dt,
                          const double *, const double *, double *r, double *, double *part) {
  if (c->op == OP_SPITZER && !STS_GATHER19) {
    flux_residual(c, b, x, dt, r, part);
    return;
  }
  Args a{};
  a.out = r;
  a.b = b;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  launch_op<M_RES>(c, 1, LoadU{x}, a);
}

void launch_true_residual(const sts_ctx *c, const double *b, const double *x, double dt,
                          double *part) {
  if (c->op == OP_SPITZER && !STS_GATHER19) {
    flux_residual(c, b, x, dt, nullptr, part);
    return;
  }
  Args a{};
  a.b = b;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  launch_op<M_RESN>(c, 1, LoadU{x}, a);
}

}  // namespace sts
