// The 19-point conduction operator in flux form, as a 2.5D march over
// r-planes, fused with the consumer of F(u) (RKL2 stage, PCG matvec,
// residual).
//
// The operator is S u = -dE/du of the discrete energy (face terms + edge
// cross terms, see k_common.h).  Grouping its terms by face gives
//   (S u)_c = sum_a [ G_a(c) - G_a(c - e_a) ]  (+ Dirichlet face terms)
//   G_a(c)  = w_a(c) (u(c+e_a) - u(c))
//             + il_a(c) sum_{b != a} [ E^{ab}_b(c) + E^{ab}_b(c - e_b) ]
//   E^{ab}_b(e) = K_ab(e)/2 * (mean b-difference quotient at the edge e)
// where il_a(c) = 1 / (centre distance across the +a face of c) and the edge
// e in the (a, b) plane has origin e (cells e, e+e_a, e+e_b, e+e_a+e_b).
// Each cell therefore needs only its own 6 coefficients: it forms the 6 edge
// fluxes E of its own edges and its 3 face fluxes G, and the neighbours'
// values arrive through LDS (same plane) or registers (previous plane).
//
// Workgroup: a core tile of 8 (theta) x 64 (phi) cells plus the 73 cells of
// the low-side halo row / column whose E and G the core needs; 640 threads,
// one position each.  The workgroup marches over a chunk of r-planes,
// starting one plane early to form the previous-plane carries.  The stencil
// input is staged in a 3-plane LDS ring (fetched two planes ahead); the own
// coefficients and epilogue operands are fetched one plane ahead.
#include "k_common.h"
#include "k_reduce.h"

namespace sts {

namespace {

#ifndef STS_FLUX_CJ
#define STS_FLUX_CJ 8
#endif
#ifndef STS_FLUX_PF
#define STS_FLUX_PF 1
#endif
constexpr int CK = 64, CJ = STS_FLUX_CJ;     // core tile
constexpr int NCORE = CK * CJ;
constexpr int NHALO = (CK + 1) + CJ;         // halo row (incl. corner) + halo column
constexpr int NPOS = NCORE + NHALO;
constexpr int NTH = (NPOS + 63) / 64 * 64;   // whole wavefronts
constexpr int UK = CK + 2, UJ = CJ + 2;      // u tile: rows j0-1..j0+8, cols k0-1..k0+64
constexpr int UPL = UK * UJ;
constexpr int ULOAD = (UPL + NTH - 1) / NTH;
constexpr int EK = CK + 1, EJ = CJ + 1;      // E / G grid: rows j0-1..j0+7, cols k0-1..k0+63
constexpr int EPL = EK * EJ;

enum { M_F = 0, M_RK1 = 1, M_RK = 2, M_PA = 3, M_RES = 4, M_RESN = 5 };

__device__ __forceinline__ int wrapclamp(int x, int n, int per) {
  if (x >= 0 && x < n) return x;
  if (per) {
    const int m = x % n;
    return m < 0 ? m + n : m;
  }
  return x < 0 ? 0 : n - 1;
}

__device__ __forceinline__ bool inside(int x, int n, int per) { return per || (x >= 0 && x < n); }

struct LoadU {
  const double *__restrict__ u;
  __device__ __forceinline__ void prepare() {}
  __device__ __forceinline__ double operator()(long long idx) const { return u[idx]; }
};

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
  double *out;
  double *F0;
  const double *ukm2;
  const double *u0;
  const double *b;
  double *y;
  double *part;
  long long cap;
  double mu, nu, mut_dt, gt_dt, dt;
  const PcgScalars *sc;
};

// XCD-aware order: hardware places workgroup w on XCD w % 8; give each XCD a
// contiguous range of the logical tile order (chunk-major), so neighbouring
// tiles share an L2.
__device__ __forceinline__ int logical_wg(int w, int n) {
  const int q = n >> 3, r = n & 7, x = w & 7, s = w >> 3;
  return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

template <int MODE, class Loader>
__global__ void __launch_bounds__(NTH)
    k_flux(Grid g, Coef C, Loader ld, Args a, int CI, int ntk, int ntj, int nchunk,
           long long ncell) {
  if (MODE == M_PA && a.sc->done) return;
  __shared__ double s_u[3][UPL];
  __shared__ double s_e[4][EPL];  // E01_1, E02_2, E12_2, E12_1
  __shared__ double s_g[2][EPL];  // G1, G2
  ld.prepare();
  const int t = threadIdx.x;
  const int nwg = gridDim.x;
  const int L = logical_wg(blockIdx.x, nwg);
  const int tkx = L % ntk, tjy = (L / ntk) % ntj, cz = L / (ntk * ntj);
  const int comp = cz / nchunk, chunk = cz - comp * nchunk;
  const int k0 = tkx * CK, j0 = tjy * CJ;
  const int i0 = chunk * CI, i1 = min(i0 + CI, g.n0);
  const long long off = (long long)comp * ncell;
  const int n12 = g.n1 * g.n2;

  // ---- this thread's position (jj, kk) relative to (j0, k0) ----
  int jj, kk;
  if (t < NCORE) {
    jj = t / CK;
    kk = t - jj * CK;
  } else if (t < NCORE + CK + 1) {
    jj = -1;
    kk = t - NCORE - 1;
  } else {
    jj = t - (NCORE + CK + 1);
    kk = -1;
  }
  const bool posv = t < NPOS;
  const bool core = t < NCORE && (j0 + jj) < g.n1 && (k0 + kk) < g.n2;
  const int jr = j0 + jj, kr = k0 + kk;
  // a position is "real" when it is a cell of the domain (after wrapping)
  const bool real = posv && inside(jr, g.n1, g.per1) && inside(kr, g.n2, g.per2) &&
                    (jr < g.n1 || g.per1) && (kr < g.n2 || g.per2);
  const int jc = wrapclamp(jr, g.n1, g.per1), kc = wrapclamp(kr, g.n2, g.per2);
  const int jp = wrapclamp(jr + 1, g.n1, g.per1);
  const int eidx = (jj + 1) * EK + (kk + 1);
  const int ubase = (jj + 1) * UK + (kk + 1);
  // per-position geometry (theta, phi factors)
  const double t11 = T1(g, T_IL11, jc), t21 = T1(g, T_IL21, jc), t21p = T1(g, T_IL21, jp);
  const double t22 = T2(g, T_IL22, kc), v12 = T1(g, T_V1, jc) * T2(g, T_V2, kc);
  const int cpl = jc * g.n2 + kc;  // in-plane offset of this position

  // ---- u tile loads ----
  int hoff[ULOAD];
#pragma unroll
  for (int q = 0; q < ULOAD; ++q) {
    const int e = min(t + q * NTH, UPL - 1);
    const int hj = e / UK, hk = e - hj * UK;
    hoff[q] = wrapclamp(j0 - 1 + hj, g.n1, g.per1) * g.n2 + wrapclamp(k0 - 1 + hk, g.n2, g.per2);
  }
  auto load_plane = [&](int ip, double *v) {
    const long long base = off + (long long)wrapclamp(ip, g.n0, g.per0) * n12;
#pragma unroll
    for (int q = 0; q < ULOAD; ++q) v[q] = ld(base + hoff[q]);
  };
  auto store_plane = [&](int ip, const double *v) {
    double *s = s_u[(ip + 3) % 3];
#pragma unroll
    for (int q = 0; q < ULOAD; ++q)
      if (t + q * NTH < UPL) s[t + q * NTH] = v[q];
  };
  // ---- own coefficients (one plane ahead) ----
  struct Coefs {
    double w0, w1, w2, k01, k02, k12;
  };
  auto load_coefs = [&](int ip, Coefs &cf) {
    const int c = wrapclamp(ip, g.n0, g.per0) * n12 + cpl;
    cf.w0 = C.w0[c];
    cf.w1 = C.w1[c];
    cf.w2 = C.w2[c];
    cf.k01 = C.k01[c];
    cf.k02 = C.k02[c];
    cf.k12 = C.k12[c];
  };
  struct Epi {
    double a, b, c;
  };
  auto load_epi = [&](int ip, Epi &ep) {
    const long long cc = off + (long long)wrapclamp(ip, g.n0, g.per0) * n12 + cpl;
    if (MODE == M_RK) {
      ep.a = a.ukm2[cc];
      ep.b = a.u0[cc];
      ep.c = a.F0[cc];
    } else if (MODE == M_RES || MODE == M_RESN) {
      ep.a = a.b[cc];
    }
  };

  const int ist = (i0 > 0 || g.per0) ? i0 - 1 : i0;  // warm-up plane for the carries
  double v[ULOAD];
  load_plane(ist, v);
  store_plane(ist, v);
  load_plane(ist + 1, v);
  store_plane(ist + 1, v);
  Coefs cf{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  Epi ep{0.0, 0.0, 0.0};
  if (STS_FLUX_PF) {
    load_coefs(ist, cf);
    if (core && ist >= i0) load_epi(ist, ep);
  }
  double e01_0p = 0.0, e02_0p = 0.0, g0p = 0.0;  // previous-plane carries
  double acc_a = 0.0, acc_b = 0.0;
  __syncthreads();

  for (int i = ist; i < i1; ++i) {
    const bool pre = i + 2 <= i1;
    if (pre) load_plane(i + 2, v);
    Coefs cn = cf;
    Epi en{0.0, 0.0, 0.0};
    if (STS_FLUX_PF && i + 1 < i1) {
      load_coefs(i + 1, cn);
      if (core) load_epi(i + 1, en);
    }
    if (!STS_FLUX_PF) {
      load_coefs(i, cf);
      if (core && i >= i0) load_epi(i, ep);
    }
    const int ic = wrapclamp(i, g.n0, g.per0);
    const int ipn = wrapclamp(i + 1, g.n0, g.per0);
    const bool plane_real = g.per0 || i >= 0;
    // uniform r-factors of this plane
    const double s00 = T0(g, T_IL00, ic), s10 = T0(g, T_IL10, ic), s10p = T0(g, T_IL10, ipn);
    const double s20 = T0(g, T_IL20, ic), s20p = T0(g, T_IL20, ipn);
    const double *su0 = s_u[(i + 3) % 3], *su1 = s_u[(i + 4) % 3];

    // ---- phase 1: edge fluxes of the edges with origin at this position ----
    // (the u values stay in registers: phases 2 and 3 must not read the LDS
    // ring, whose oldest slot other wavefronts refill during phase 1)
    double e01_0 = 0.0, e02_0 = 0.0, e01_1 = 0.0, e02_2 = 0.0, e12_2 = 0.0, e12_1 = 0.0;
    double u000 = 0.0, u010 = 0.0, u001 = 0.0, u100 = 0.0;
    if (real && plane_real) {
      u000 = su0[ubase];
      u010 = su0[ubase + UK];
      u001 = su0[ubase + 1];
      u100 = su1[ubase];
      const double u011 = su0[ubase + UK + 1];
      const double u110 = su1[ubase + UK], u101 = su1[ubase + 1];
      const double il1 = s10 * t11;
      // plane (0, 1): r- and theta-difference quotients at the edge
      const double d0a = 0.5 * s00 * ((u100 - u000) + (u110 - u010));
      const double d1a = 0.5 * ((u010 - u000) * il1 + (u110 - u100) * (s10p * t11));
      // plane (0, 2)
      const double d0b = 0.5 * s00 * ((u100 - u000) + (u101 - u001));
      const double d2b = 0.5 * t21 * t22 * ((u001 - u000) * s20 + (u101 - u100) * s20p);
      // plane (1, 2)
      const double d1c = 0.5 * il1 * ((u010 - u000) + (u011 - u001));
      const double d2c = 0.5 * s20 * t22 * ((u001 - u000) * t21 + (u011 - u010) * t21p);
      const double h01 = 0.5 * cf.k01, h02 = 0.5 * cf.k02, h12 = 0.5 * cf.k12;
      e01_0 = h01 * d0a;
      e01_1 = h01 * d1a;
      e02_0 = h02 * d0b;
      e02_2 = h02 * d2b;
      e12_1 = h12 * d1c;
      e12_2 = h12 * d2c;
    }
    if (posv) {
      s_e[0][eidx] = e01_1;
      s_e[1][eidx] = e02_2;
      s_e[2][eidx] = e12_2;
      s_e[3][eidx] = e12_1;
    }
    if (pre) store_plane(i + 2, v);
    __syncthreads();

    // ---- phase 2: face fluxes ----
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    if (real && plane_real) {
      const double il1 = s10 * t11, il2 = s20 * t21 * t22;
      // neighbours at j-1 / k-1 (zero outside the E grid: only reached by
      // positions whose G is never used)
      const double e01_1m = jj >= 0 ? s_e[0][eidx - EK] : 0.0;
      const double e02_2m = kk >= 0 ? s_e[1][eidx - 1] : 0.0;
      const double e12_2m = kk >= 0 ? s_e[2][eidx - 1] : 0.0;
      const double e12_1m = jj >= 0 ? s_e[3][eidx - EK] : 0.0;
      g0 = cf.w0 * (u100 - u000) + s00 * ((e01_1 + e01_1m) + (e02_2 + e02_2m));
      g1 = cf.w1 * (u010 - u000) + il1 * ((e01_0 + e01_0p) + (e12_2 + e12_2m));
      g2 = cf.w2 * (u001 - u000) + il2 * ((e02_0 + e02_0p) + (e12_1 + e12_1m));
    }
    if (posv) {
      s_g[0][eidx] = g1;
      s_g[1][eidx] = g2;
    }
    __syncthreads();

    // ---- phase 3: divergence and the consumer of F ----
    if (core && i >= i0) {
      const double uc = u000;
      double su = (g0 - g0p) + (g1 - s_g[0][eidx - EK]) + (g2 - s_g[1][eidx - 1]);
      if ((g.dir_lo && i == 0) || (g.dir_hi && i == g.n0 - 1)) {
        const bool with_g = MODE == M_F || MODE == M_RK1 || MODE == M_RK;
        const bool lo = g.dir_lo && i == 0;
        const double wb = lo ? C.wb_lo[cpl] : C.wb_hi[cpl];
        const double ub = lo ? C.ub_lo[cpl] : C.ub_hi[cpl];
        su += with_g ? wb * (ub - uc) : -wb * uc;
        if (g.dir_lo && g.dir_hi && i == 0 && i == g.n0 - 1)
          su += with_g ? C.wb_hi[cpl] * (C.ub_hi[cpl] - uc) : -C.wb_hi[cpl] * uc;
      }
      const double V = T0(g, T_V0, ic) * v12;
      const long long cc = off + (long long)i * n12 + cpl;
      if (MODE == M_F) {
        a.out[cc] = su / V;
      } else if (MODE == M_RK1) {
        const double F = su / V;
        a.F0[cc] = F;
        a.out[cc] = uc + a.mut_dt * F;
      } else if (MODE == M_RK) {
        const double F = su / V;
        a.out[cc] = a.mu * uc + a.nu * ep.a + (1.0 - a.mu - a.nu) * ep.b + a.mut_dt * F +
                    a.gt_dt * ep.c;
      } else if (MODE == M_PA) {
        const double yv = V * uc - a.dt * su;
        a.out[cc] = uc;
        a.y[cc] = yv;
        acc_a += uc * yv;
      } else {
        const double bv = ep.a;
        const double rv = bv - (V * uc - a.dt * su);
        if (MODE == M_RES) a.out[cc] = rv;
        acc_a += rv * rv;
        acc_b += bv * bv;
      }
    }
    e01_0p = e01_0;
    e02_0p = e02_0;
    g0p = g0;
    if (STS_FLUX_PF) {
      cf = cn;
      ep = en;
    }
  }
  if (MODE == M_PA || MODE == M_RES || MODE == M_RESN) {
    // reduce over the 8 core wavefronts only (halo wavefronts hold zeros)
    __shared__ double ra[NTH / 64], rb[NTH / 64];
    const double sa = wave_sum(acc_a), sb = wave_sum(acc_b);
    if ((t & 63) == 0) {
      ra[t >> 6] = sa;
      rb[t >> 6] = sb;
    }
    __syncthreads();
    if (t == 0) {
      double x = 0.0, y = 0.0;
      for (int w = 0; w < NTH / 64; ++w) {
        x += ra[w];
        y += rb[w];
      }
      a.part[blockIdx.x] = x;
      a.part[a.cap + blockIdx.x] = y;
    }
  }
}

struct Plan {
  int CI, ntk, ntj, nchunk, nwg;
};

Plan plan_of(const sts_ctx *c, int ncomp) {
  Plan p;
  p.ntk = (c->n2 + CK - 1) / CK;
  p.ntj = (c->n1 + CJ - 1) / CJ;
  const long long tiles = (long long)p.ntk * p.ntj;
  long long ci = tiles * c->n0 / 1024;  // aim for ~1024 workgroups
  if (ci < 2) ci = 2;
  if (ci > 32) ci = 32;
  if (ci > c->n0) ci = c->n0;
  p.CI = (int)ci;
  p.nchunk = (c->n0 + p.CI - 1) / p.CI;
  p.nwg = p.ntk * p.ntj * p.nchunk * ncomp;
  return p;
}

template <int MODE, class Loader>
void launch(const sts_ctx *c, int ncomp, const Loader &ld, const Args &a) {
  const Plan p = plan_of(c, ncomp);
  hipLaunchKernelGGL((k_flux<MODE, Loader>), dim3(p.nwg), dim3(NTH), 0, c->stream, c->grid(),
                     c->coef(), ld, a, p.CI, p.ntk, p.ntj, p.nchunk, c->ncell);
}

}  // namespace

int flux_parts(const sts_ctx *c) { return plan_of(c, 1).nwg; }

void flux_stage(const sts_ctx *c, int mode, int ncomp, const double *ukm1, const double *ukm2,
                const double *u0, double *F0, double *out, double mu, double nu, double mut_dt,
                double gt_dt) {
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
    launch<M_F>(c, ncomp, ld, a);
  else if (mode == 1)
    launch<M_RK1>(c, ncomp, ld, a);
  else
    launch<M_RK>(c, ncomp, ld, a);
}

void flux_pass_a(const sts_ctx *c, double dt, const double *r, const double *invd,
                 const double *zilu, const double *pold, double *pnew, double *y, double *part,
                 const PcgScalars *sc, int first) {
  Args a{};
  a.out = pnew;
  a.y = y;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  a.sc = sc;
  if (zilu) {
    const LoadP<STS_PC_BLOCK_ILU0> ld{r, invd, zilu, pold, sc, first, 0.0};
    launch<M_PA>(c, 1, ld, a);
  } else {
    const LoadP<STS_PC_JACOBI> ld{r, invd, zilu, pold, sc, first, 0.0};
    launch<M_PA>(c, 1, ld, a);
  }
}

void flux_residual(const sts_ctx *c, const double *b, const double *x, double dt, double *r,
                   double *part) {
  Args a{};
  a.out = r;
  a.b = b;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  if (r)
    launch<M_RES>(c, 1, LoadU{x}, a);
  else
    launch<M_RESN>(c, 1, LoadU{x}, a);
}

}  // namespace sts
