// RKL2 stages of the conduction term with the Spitzer diffusivity taken from
// the stage value itself instead of the step's start (RKL2 only evaluates F,
// so it can apply the nonlinear operator; Sec. 2.4, Sec. 3.1):
//   F(u) = V^-1 (S(kappa(u)) u + g(kappa(u))),  kappa(u) = kappa0 max(u, 0)^{5/2},
//   D = kappa b b^T (Eq. mhd:e1), b fixed over the step,
// with S, g the 19-point energy-form operator: face weights A Dbar_aa / dl
// (Dbar over the face's two cells), edge weights W_e Dbar_ab (W_e, Dbar over
// the edge's four cells).
//
// No coefficient arrays are read or written.  A workgroup marches a chunk of
// r-planes of a TJ x TK tile; per plane p it forms, on the tile plus one halo
// cell, the tensors D(p) from u and b and stores in LDS the in-plane parts
// D11, D22, D12 of plane p and the pair sums P01 = D01(p-1) + D01(p),
// P02 = D02(p-1) + D02(p) (the r-direction halves of the (0,1) / (0,2) edge
// weights of plane p-1).  The row of a cell of plane i then takes every face
// and edge weight it needs from these sums over its 3 x 3 in-plane
// neighbourhood, and the weights that join planes i-1 and i from registers
// (kept from the previous plane).  Tensor planes are triple-buffered and pair
// sums double-buffered, so one barrier per plane separates the tensor stage
// of plane i+1 from the rows of plane i.
// Per cell and stage: u_{k-1}, b (3 arrays), u_{k-2}, u_0, F0 read and u_k
// written, 64 B, against 88 B when the six coefficient arrays are stored.
#include "k_row.h"

#include <algorithm>

namespace sts {

namespace {

#ifndef STS_NL_WG
#define STS_NL_WG 512  // about one round of 2 workgroups per CU
#endif

constexpr int NK = 64, NJ = 4, NNT = NK * NJ;          // tile = threads
constexpr int QK = NK + 2, QJ = NJ + 2, QP = QK * QJ;  // plane + one halo cell
constexpr int NRING = QP - NNT;                        // 140 halo cells
constexpr int RING_PER_WAVE = NRING / 4;               // 35 per wavefront

enum { NL_F = 0, NL_RK1 = 1, NL_RK = 2 };
enum { Q11, Q22, Q12, NQ };  // in-plane tensor parts
enum { P01, P02, NPS };      // r-direction pair sums

struct NlArgs {
  const double *ukm1, *ukm2, *u0;
  const double *b0, *b1, *b2;
  double *F0, *out;
  double kappa0, mu, nu, mut_dt, gt_dt;
};

struct Dten {
  double d00, d01, d02, d11, d22, d12;
};

__device__ __forceinline__ Dten spitzer_tensor(double u, double x, double y, double z,
                                               double kappa0) {
  const double t = u > 0.0 ? u : 0.0;
  const double kap = kappa0 * t * t * sqrt(t);
  Dten d;
  d.d00 = kap * x * x;
  d.d01 = kap * x * y;
  d.d02 = kap * x * z;
  d.d11 = kap * y * y;
  d.d22 = kap * z * z;
  d.d12 = kap * y * z;
  return d;
}

// (hj, hk) of halo cell r of a plane: row hj = 0, row hj = NJ + 1, then the
// columns hk = 0 and hk = NK + 1 of the rows between.
__device__ __forceinline__ void ring_cell(int r, int &hj, int &hk) {
  if (r < QK) {
    hj = 0;
    hk = r;
  } else if (r < 2 * QK) {
    hj = NJ + 1;
    hk = r - QK;
  } else if (r < 2 * QK + NJ) {
    hj = r - 2 * QK + 1;
    hk = 0;
  } else {
    hj = r - 2 * QK - NJ + 1;
    hk = NK + 1;
  }
}

// r-direction geometry of plane i: A00 IL00, A10 IL10, A20 IL20, V0 and
// V0 + V0 of the +1 plane.
struct PlaneFac {
  double p0, p1, p2, v, vs;
};

__device__ __forceinline__ PlaneFac plane_fac(const Grid &g, int i) {
  const Nb A = nbr(i, g.n0, g.per0);
  PlaneFac f;
  f.p0 = T0u(g, T_A00, i) * T0u(g, T_IL00, i);
  f.p1 = T0u(g, T_A10, i) * T0u(g, T_IL10, i);
  f.p2 = T0u(g, T_A20, i) * T0u(g, T_IL20, i);
  f.v = T0u(g, T_V0, i);
  f.vs = f.v + T0u(g, T_V0, A.p);
  return f;
}

// In-plane geometry of the weights a cell's row needs (origins at the cell
// and at its -1 neighbours along theta / phi), as theta factors (uniform over
// a wavefront) and phi factors:
//   w0 = p0 [A01][A02],  w1 = p1 [A11 IL11 (j or j-1)][A12],
//   w2 = p2 [A21 IL21][A22 IL22 (k or k-1)],
//   K01 = vs [V1 + V1+][V2] / 16,  K02 = vs [V1][V2 + V2+] / 16,
//   K12 = v [V1 + V1+][V2 + V2+] / 16  (or with the -1 sums).
struct ThetaGeo {
  double a01, a11, a11m, a21, v1, s1p, s1m;
};
struct PhiGeo {
  double a02, a12, a22, a22m, v2, s2p, s2m;
};

__device__ __forceinline__ ThetaGeo theta_geo(const Grid &g, int j) {
  const Nb B = nbr(j, g.n1, g.per1);
  ThetaGeo o;
  o.a01 = T1u(g, T_A01, j);
  o.a11 = T1u(g, T_A11, j) * T1u(g, T_IL11, j);
  o.a11m = T1u(g, T_A11, B.m) * T1u(g, T_IL11, B.m);
  o.a21 = T1u(g, T_A21, j) * T1u(g, T_IL21, j);
  o.v1 = T1u(g, T_V1, j);
  o.s1p = o.v1 + T1u(g, T_V1, B.p);
  o.s1m = T1u(g, T_V1, B.m) + o.v1;
  return o;
}

__device__ __forceinline__ PhiGeo phi_geo(const Grid &g, int k) {
  const Nb C = nbr(k, g.n2, g.per2);
  PhiGeo o;
  o.a02 = T2(g, T_A02, k);
  o.a12 = T2(g, T_A12, k);
  o.a22 = T2(g, T_A22, k) * T2(g, T_IL22, k);
  o.a22m = T2(g, T_A22, C.m) * T2(g, T_IL22, C.m);
  o.v2 = T2(g, T_V2, k);
  o.s2p = o.v2 + T2(g, T_V2, C.p);
  o.s2m = T2(g, T_V2, C.m) + o.v2;
  return o;
}

template <int MODE>
__global__ void __launch_bounds__(NNT) k_march_nl(Grid g, CoefS<double> C, NlArgs a, int CI) {
  __shared__ double s_u[4][QP];
  __shared__ double s_q[3][NQ][QP];
  __shared__ double s_p[2][NPS][QP];

  // a wavefront is one tile row (blockDim.x = 64): theta-dependent values
  // are uniform across it and live in scalar registers
  const int tk = threadIdx.x, tj = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int tid = tj * NK + tk;
  // XCD-aware order (workgroup w runs on XCD w % 8; each XCD gets a
  // contiguous range of the logical (chunk, row-tile, column-tile) order)
  const int nwg = gridDim.x, w = wg_index(g.wg_rev);
  const int q8 = nwg >> 3, r8 = nwg & 7, x8 = w & 7, s8 = w >> 3;
  const int L = x8 < r8 ? x8 * (q8 + 1) + s8 : r8 * (q8 + 1) + (x8 - r8) * q8 + s8;
  const int ntk = (g.n2 + NK - 1) / NK, ntj = (g.n1 + NJ - 1) / NJ;
  const int bx = L % ntk, by = (L / ntk) % ntj, chunk = L / (ntk * ntj);
  const int k0 = bx * NK, j0 = by * NJ;
  const int i0 = chunk * CI, i1 = min(i0 + CI, g.n0);
  const long long n12 = (long long)g.n1 * g.n2;

  // cells of this thread in every plane: its own, and one halo cell for the
  // first 35 lanes of each wavefront
  const int lane = tid & 63, wv = tid >> 6;
  const bool has_ring = lane < RING_PER_WAVE;
  int rhj, rhk;
  ring_cell(has_ring ? wv * RING_PER_WAVE + lane : 0, rhj, rhk);
  const int e = (tj + 1) * QK + (tk + 1), e_ring = rhj * QK + rhk;
  const int off_own = wrapclamp(j0 + tj, g.n1, g.per1) * g.n2 + wrapclamp(k0 + tk, g.n2, g.per2);
  // lanes without a halo cell load their own cell twice: every lane issues
  // the same loads, so the in-order load counter waits exactly
  const int off_ring = has_ring ? wrapclamp(j0 - 1 + rhj, g.n1, g.per1) * g.n2 +
                                      wrapclamp(k0 - 1 + rhk, g.n2, g.per2)
                                : off_own;

  auto plane_base = [&](int ip) { return (long long)wrapclamp(ip, g.n0, g.per0) * n12; };
  double uo = 0.0, ur = 0.0, bx0 = 0.0, bx1 = 0.0, bx2 = 0.0, br0 = 0.0, br1 = 0.0, br2 = 0.0;
  auto load_plane = [&](int ip) {
    const long long base = plane_base(ip);
    uo = a.ukm1[base + off_own];
    bx0 = a.b0[base + off_own];
    bx1 = a.b1[base + off_own];
    bx2 = a.b2[base + off_own];
    ur = a.ukm1[base + off_ring];
    br0 = a.b0[base + off_ring];
    br1 = a.b1[base + off_ring];
    br2 = a.b2[base + off_ring];
  };
  // Tensor stage of plane ip (its u and b in registers): u into the ring,
  // D11 / D22 / D12 of plane ip, pair sums of plane ip - 1.  Carries the
  // own cell's tensor (and the halo cell's D01, D02) to the next plane.
  Dten cd{};                      // own cell, previous plane
  double cr01 = 0.0, cr02 = 0.0;  // halo cell, previous plane
  double p01 = 0.0, p02 = 0.0;    // own pair sums of plane ip - 1
  auto tensor_stage = [&](int ip) {
    const Dten d = spitzer_tensor(uo, bx0, bx1, bx2, a.kappa0);
    s_u[ip & 3][e] = uo;
    double *q = &s_q[(ip + 3) % 3][0][0];  // ip >= -1
    q[Q11 * QP + e] = d.d11;
    q[Q22 * QP + e] = d.d22;
    q[Q12 * QP + e] = d.d12;
    double *p = &s_p[(ip - 1) & 1][0][0];
    p01 = cd.d01 + d.d01;
    p02 = cd.d02 + d.d02;
    p[P01 * QP + e] = p01;
    p[P02 * QP + e] = p02;
    if (has_ring) {
      const Dten r = spitzer_tensor(ur, br0, br1, br2, a.kappa0);
      s_u[ip & 3][e_ring] = ur;
      q[Q11 * QP + e_ring] = r.d11;
      q[Q22 * QP + e_ring] = r.d22;
      q[Q12 * QP + e_ring] = r.d12;
      p[P01 * QP + e_ring] = cr01 + r.d01;
      p[P02 * QP + e_ring] = cr02 + r.d02;
      cr01 = r.d01;
      cr02 = r.d02;
    }
    cd = d;
    return d;
  };

  const int j = j0 + tj, k = k0 + tk;
  const bool active = j < g.n1 && k < g.n2;
  const int jc = min(j, g.n1 - 1), kc = min(k, g.n2 - 1);
  const ThetaGeo gj = theta_geo(g, jc);
  const PhiGeo gk = phi_geo(g, kc);

  // Weights joining planes ip and ip + 1 (pair sums of plane ip in LDS; the
  // own cell's in p01 / p02).
  double K01o = 0.0, K01m = 0.0, K02o = 0.0, K02m = 0.0;
  auto cross_weights = [&](int ip, const PlaneFac &f) {
    const double *p = &s_p[ip & 1][0][0];
    const double c = f.vs * 0.0625;
    K01o = (c * gj.s1p) * gk.v2 * (p01 + p[P01 * QP + e + QK]);
    K01m = (c * gj.s1m) * gk.v2 * (p[P01 * QP + e - QK] + p01);
    K02o = (c * gj.v1) * gk.s2p * (p02 + p[P02 * QP + e + 1]);
    K02m = (c * gj.v1) * gk.s2m * (p[P02 * QP + e - 1] + p02);
  };

  // ---- prologue: tensors of planes i0 - 1 and i0, weights of plane i0 - 1 ----
  load_plane(i0 - 1);
  const Dten dprev = tensor_stage(i0 - 1);  // (its pair sums, of plane i0 - 2, are unused)
  load_plane(i0);
  Dten dcur = tensor_stage(i0);
  load_plane(i0 + 1);
  __syncthreads();
  double pw0, pk01, pk01B, pk02, pk02C;
  {
    const PlaneFac f = plane_fac(g, wrapclamp(i0 - 1, g.n0, g.per0));
    pw0 = (f.p0 * gj.a01) * gk.a02 * (0.5 * (dprev.d00 + dcur.d00));
    cross_weights(i0 - 1, f);
    pk01 = K01o;
    pk01B = K01m;
    pk02 = K02o;
    pk02C = K02m;
  }

  ThreadGeo<double> tg;
  tg.B = nbr(jc, g.n1, g.per1);
  tg.C = nbr(kc, g.n2, g.per2);
  tg.t11m = T1u(g, T_IL11, tg.B.m);
  tg.t11 = T1u(g, T_IL11, jc);
  tg.t21m = T1u(g, T_IL21, tg.B.m);
  tg.t21 = T1u(g, T_IL21, jc);
  tg.t21p = T1u(g, T_IL21, tg.B.p);
  tg.t22m = T2(g, T_IL22, tg.C.m);
  tg.t22 = T2(g, T_IL22, kc);
  tg.v12 = gj.v1 * gk.v2;
  Grid gs = g;  // the row without its Dirichlet terms (added below from kappa(u))
  gs.dir_lo = gs.dir_hi = 0;

  for (int i = i0; i < i1; ++i) {
    const long long cc = (long long)(i * g.n1 + jc) * g.n2 + kc;
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (MODE == NL_RK) {
      x0 = a.ukm2[cc];
      x1 = a.u0[cc];
      x2 = a.F0[cc];
    }
    // tensor stage of plane i + 1, then the loads for plane i + 2
    const Dten dn = tensor_stage(i + 1);
    if (i + 2 <= i1) load_plane(i + 2);
    __syncthreads();

    // row of plane i
    const PlaneFac f = plane_fac(g, i);
    cross_weights(i, f);
    const double *q = &s_q[i % 3][0][0];
    const double *q11 = q + Q11 * QP, *q22 = q + Q22 * QP, *q12 = q + Q12 * QP;
    RowCoef<double> W;
    const double d11 = q11[e], d22 = q22[e], d12 = q12[e];
    W.w0p = (f.p0 * gj.a01) * gk.a02 * (0.5 * (dcur.d00 + dn.d00));
    W.w0m = pw0;
    W.w1p = (f.p1 * gj.a11) * gk.a12 * (0.5 * (d11 + q11[e + QK]));
    W.w1m = (f.p1 * gj.a11m) * gk.a12 * (0.5 * (q11[e - QK] + d11));
    W.w2p = (f.p2 * gj.a21) * gk.a22 * (0.5 * (d22 + q22[e + 1]));
    W.w2m = (f.p2 * gj.a21) * gk.a22m * (0.5 * (q22[e - 1] + d22));
    W.K01[0] = K01o;
    W.K01[1] = pk01;
    W.K01[2] = K01m;
    W.K01[3] = pk01B;
    W.K02[0] = K02o;
    W.K02[1] = pk02;
    W.K02[2] = K02m;
    W.K02[3] = pk02C;
    {
      const double c = f.v * 0.0625;
      const double dJ = q12[e + QK], dK = q12[e + 1], dJK = q12[e + QK + 1];
      const double dJm = q12[e - QK], dKm = q12[e - 1], dJmK = q12[e - QK + 1];
      const double dJKm = q12[e + QK - 1], dJmKm = q12[e - QK - 1];
      W.K12[0] = (c * gj.s1p) * gk.s2p * (d12 + dJ + dK + dJK);
      W.K12[1] = (c * gj.s1m) * gk.s2p * (dJm + d12 + dJmK + dK);
      W.K12[2] = (c * gj.s1p) * gk.s2m * (dKm + dJKm + d12 + dJ);
      W.K12[3] = (c * gj.s1m) * gk.s2m * (dJmKm + dKm + dJm + d12);
    }
    if (active) {
      PlaneGeo<double> pg;
      pg.A = nbr(i, g.n0, g.per0);
      pg.s00m = T0u(g, T_IL00, pg.A.m);
      pg.s00 = T0u(g, T_IL00, i);
      pg.s10m = T0u(g, T_IL10, pg.A.m);
      pg.s10 = T0u(g, T_IL10, i);
      pg.s10p = T0u(g, T_IL10, pg.A.p);
      pg.s20m = T0u(g, T_IL20, pg.A.m);
      pg.s20 = T0u(g, T_IL20, i);
      pg.s20p = T0u(g, T_IL20, pg.A.p);
      pg.v0 = f.v;
      const double *sm = s_u[(i - 1) & 3], *s0 = s_u[i & 3], *sp = s_u[(i + 1) & 3];
      auto U = [&](int di, int dj, int dk) -> double {
        const double *s = di < 0 ? sm : (di > 0 ? sp : s0);
        return s[e + dj * QK + dk];
      };
      double su = apply_S<OP_SPITZER, true, double, double>(gs, C, W, U, i, j, k, pg, tg);
      const double uc = s0[e];
      // Dirichlet faces on axis 0: w_b = A_b D_00(c) / (centre-to-face distance)
      const int bi = j * g.n2 + k;
      if (g.dir_lo && i == 0)
        su += g.ab_lo * (gj.a01 * gk.a02) * dcur.d00 / g.db_lo * (C.ub_lo[bi] - uc);
      if (g.dir_hi && i == g.n0 - 1)
        su += g.ab_hi * (gj.a01 * gk.a02) * dcur.d00 / g.db_hi * (C.ub_hi[bi] - uc);
      const double F = su / (f.v * tg.v12);
      const long long c = (long long)(i * g.n1 + j) * g.n2 + k;
      if (MODE == NL_F) {
        a.out[c] = F;
      } else if (MODE == NL_RK1) {
        a.F0[c] = F;
        a.out[c] = uc + a.mut_dt * F;
      } else {
        a.out[c] = a.mu * uc + a.nu * x0 + (1.0 - a.mu - a.nu) * x1 + a.mut_dt * F +
                   a.gt_dt * x2;
      }
    }
    pw0 = W.w0p;
    pk01 = K01o;
    pk01B = K01m;
    pk02 = K02o;
    pk02C = K02m;
    dcur = dn;
  }
}

int chunk_nl(const sts_ctx *c) {
  const long long tiles = (long long)((c->n2 + NK - 1) / NK) * ((c->n1 + NJ - 1) / NJ);
  long long ci = tiles * c->n0 / STS_NL_WG;
  if (ci < 2) ci = 2;
  if (ci > 32) ci = 32;
  return (int)std::min<long long>(ci, c->n0);
}

}  // namespace

// mode 0: out = F(u); mode 1: F0 = F(u_0), out = u_0 + mut_dt F0;
// mode 2: out = mu u_{k-1} + nu u_{k-2} + (1 - mu - nu) u_0 + mut_dt F(u_{k-1}) + gt_dt F0
void launch_stage_nl(const sts_ctx *c, int mode, const double *ukm1, const double *ukm2,
                     const double *u0, double *F0, double *out, double mu, double nu,
                     double mut_dt, double gt_dt, double kappa0, const double *b0,
                     const double *b1, const double *b2) {
  STS_PROF(c, "launch_stage_nl");
  NlArgs a{ukm1, ukm2, u0, b0, b1, b2, F0, out, kappa0, mu, nu, mut_dt, gt_dt};
  const Coef k = c->coef();
  CoefS<double> C{};
  C.wb_lo = k.wb_lo;
  C.wb_hi = k.wb_hi;
  C.ub_lo = k.ub_lo;
  C.ub_hi = k.ub_hi;
  const int CI = chunk_nl(c), nchunk = (c->n0 + CI - 1) / CI;
  const dim3 grid(((c->n2 + NK - 1) / NK) * ((c->n1 + NJ - 1) / NJ) * nchunk);
  const dim3 block(NK, NJ);
  if (mode == NL_F)
    hipLaunchKernelGGL(k_march_nl<NL_F>, grid, block, 0, c->stream, c->grid(), C, a, CI);
  else if (mode == NL_RK1)
    hipLaunchKernelGGL(k_march_nl<NL_RK1>, grid, block, 0, c->stream, c->grid(), C, a, CI);
  else
    hipLaunchKernelGGL(k_march_nl<NL_RK>, grid, block, 0, c->stream, c->grid(), C, a, CI);
}

}  // namespace sts
