// RKL2 stages of the conduction term with the Spitzer diffusivity taken from
// the stage value itself instead of the step's start (RKL2 only evaluates F,
// so it can apply the nonlinear operator; Sec. 2.4, Sec. 3.1):
//   F(u) = V^-1 (S(kappa(u)) u + g(kappa(u))),  kappa(u) = kappa0 max(u, 0)^{5/2},
//   D = kappa b b^T (Eq. mhd:e1), b fixed over the step,
// with S, g the 19-point energy-form operator (face weights A Dbar_aa / dl,
// edge weights W_e Dbar_ab; means over the face's two / the edge's four cells).
//
// No coefficient arrays are read or written: a workgroup marches a chunk of
// r-planes of a TJ x TK tile and, per plane, forms the coefficients in LDS
// from u and b.  Per plane i, three phases separated by two barriers:
//   P1  D(i+1) = kappa(u) b b^T on the tile + one halo cell (LDS); each thread
//       keeps the tensors of its own cells in registers;
//   P2  the coefficients at the edge / face origins of plane i (tile + the
//       low halo row and column; LDS): w1, w2, K12 lie in plane i and were
//       formed from D(i) one plane earlier (carried), w0, K01, K02 join
//       planes i and i+1 and combine a carried plane-i partial sum with
//       D(i+1); the next-but-one u plane is staged into the ring;
//   P3  the row of each tile cell from its own and its -1 neighbours'
//       coefficients (coefficients of plane i-1 carried in registers), fused
//       with the RKL2 stage recurrence.
// Per cell and stage: u_{k-1}, b (3 arrays), u_{k-2}, u_0, F0 read and u_k
// written, 64 B, against 88 B when the six coefficient arrays are stored.
#include "k_row.h"

#include <algorithm>

namespace sts {

namespace {

#ifndef STS_NL_WG
#define STS_NL_WG 2048
#endif

constexpr int NK = 64, NJ = 4, NNT = NK * NJ;          // tile = threads
constexpr int QK = NK + 2, QJ = NJ + 2, QP = QK * QJ;  // plane + one halo cell
constexpr int OK = NK + 1, OJ = NJ + 1, OP = OK * OJ;  // origins: tile + low halo
constexpr int NRING = QP - NNT;                        // 140 halo cells of a plane
constexpr int NLOW = OP - NNT;                         // 69 low-halo origins

enum { NL_F = 0, NL_RK1 = 1, NL_RK = 2 };
enum { D01, D02, D11, D22, D12, ND };          // LDS tensor components
enum { C_W1, C_W2, C_K01, C_K02, C_K12, NC };  // LDS origin coefficients
// low-halo origin state kept in LDS: carried partial sums and coefficients,
// then the origin's geometry factors
enum { L_B01, L_B02, L_W1, L_W2, L_K12, L_G1, L_G2, L_G01, L_G02, L_G12, NL_LOW };

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

// (hj, hk) of halo cell r of a plane: first the 69 low-halo origins (row
// hj = 0 for hk < 65, then column hk = 0 for hj = 1..4), then the rest.
__device__ __forceinline__ void ring_cell(int r, int &hj, int &hk) {
  if (r < OK) {
    hj = 0;
    hk = r;
  } else if (r < NLOW) {
    hj = r - NK;
    hk = 0;
  } else if (r == NLOW) {
    hj = 0;
    hk = NK + 1;
  } else if (r < NLOW + 1 + QK) {
    hj = NJ + 1;
    hk = r - NLOW - 1;
  } else {
    hj = r - (NLOW + QK);
    hk = NK + 1;
  }
}

// Geometry factors of an origin at (j, k) (in-plane parts; the r-parts are
// per-plane scalars):  w0 = A00 IL00 * [A01 A02],  w1 = A10 IL10 * [A11 IL11 A12],
// w2 = A20 IL20 * [A21 IL21 A22 IL22],  K01 = (V0 + V0+) * [(V1 + V1+) V2] / 16,
// K02 = (V0 + V0+) * [V1 (V2 + V2+)] / 16,  K12 = V0 * [(V1 + V1+)(V2 + V2+)] / 16.
struct OriginGeo {
  double g0, g1, g2, g01, g02, g12;
};

__device__ __forceinline__ OriginGeo origin_geo(const Grid &g, int j, int k) {
  const Nb B = nbr(j, g.n1, g.per1), C = nbr(k, g.n2, g.per2);
  OriginGeo o;
  o.g0 = T1(g, T_A01, j) * T2(g, T_A02, k);
  o.g1 = T1(g, T_A11, j) * T1(g, T_IL11, j) * T2(g, T_A12, k);
  o.g2 = T1(g, T_A21, j) * T1(g, T_IL21, j) * T2(g, T_A22, k) * T2(g, T_IL22, k);
  const double v1s = T1(g, T_V1, j) + T1(g, T_V1, B.p);
  const double v2s = T2(g, T_V2, k) + T2(g, T_V2, C.p);
  o.g01 = v1s * T2(g, T_V2, k);
  o.g02 = T1(g, T_V1, j) * v2s;
  o.g12 = v1s * v2s;
  return o;
}

struct PlaneFac {
  double p0, p1, p2;  // A00 IL00, A10 IL10, A20 IL20
  double v, vs;       // V0, V0 + V0 of the +1 plane
};

__device__ __forceinline__ PlaneFac plane_fac(const Grid &g, int i) {
  const Nb A = nbr(i, g.n0, g.per0);
  PlaneFac f;
  f.p0 = T0(g, T_A00, i) * T0(g, T_IL00, i);
  f.p1 = T0(g, T_A10, i) * T0(g, T_IL10, i);
  f.p2 = T0(g, T_A20, i) * T0(g, T_IL20, i);
  f.v = T0(g, T_V0, i);
  f.vs = f.v + T0(g, T_V0, A.p);
  return f;
}

template <int MODE>
__global__ void __launch_bounds__(NNT) k_march_nl(Grid g, CoefS<double> C, NlArgs a, int CI,
                                                   int nchunk) {
  __shared__ double s_u[4][QP];
  __shared__ double s_d[ND][QP];
  __shared__ double s_c[NC][OP];
  __shared__ double s_lo[NL_LOW][NLOW];

  const int tk = threadIdx.x, tj = threadIdx.y, tid = tj * NK + tk;
  // XCD-aware order (workgroup w runs on XCD w % 8; each XCD gets a
  // contiguous range of the logical (chunk, row-tile, column-tile) order)
  const int nwg = gridDim.x, w = blockIdx.x;
  const int q8 = nwg >> 3, r8 = nwg & 7, x8 = w & 7, s8 = w >> 3;
  const int L = x8 < r8 ? x8 * (q8 + 1) + s8 : r8 * (q8 + 1) + (x8 - r8) * q8 + s8;
  const int ntk = (g.n2 + NK - 1) / NK, ntj = (g.n1 + NJ - 1) / NJ;
  const int bx = L % ntk, by = (L / ntk) % ntj, chunk = L / (ntk * ntj);
  const int k0 = bx * NK, j0 = by * NJ;
  const int i0 = chunk * CI, i1 = min(i0 + CI, g.n0);
  (void)nchunk;
  const long long n12 = (long long)g.n1 * g.n2;

  // cells of this thread in a plane: its own (slot 0) and halo cell tid (slot 1)
  const bool has_ring = tid < NRING, has_low = tid < NLOW;
  int rhj, rhk;
  ring_cell(has_ring ? tid : 0, rhj, rhk);
  const int e_own = (tj + 1) * QK + (tk + 1), e_ring = rhj * QK + rhk;
  const int o_own = (tj + 1) * OK + (tk + 1), o_low = rhj * OK + rhk;
  const int jw = wrapclamp(j0 + tj, g.n1, g.per1), kw = wrapclamp(k0 + tk, g.n2, g.per2);
  const int jr = wrapclamp(j0 - 1 + rhj, g.n1, g.per1), kr = wrapclamp(k0 - 1 + rhk, g.n2, g.per2);
  const int off_own = jw * g.n2 + kw, off_ring = jr * g.n2 + kr;

  const OriginGeo og = origin_geo(g, jw, kw);
  if (has_low) {
    const OriginGeo lg = origin_geo(g, jr, kr);
    s_lo[L_G1][tid] = lg.g1;
    s_lo[L_G2][tid] = lg.g2;
    s_lo[L_G01][tid] = lg.g01;
    s_lo[L_G02][tid] = lg.g02;
    s_lo[L_G12][tid] = lg.g12;
  }

  auto plane_base = [&](int ip) { return (long long)wrapclamp(ip, g.n0, g.per0) * n12; };
  auto load_u = [&](int ip, double &vo, double &vr) {
    const long long base = plane_base(ip);
    vo = a.ukm1[base + off_own];
    vr = has_ring ? a.ukm1[base + off_ring] : 0.0;
  };
  auto store_u = [&](int ip, double vo, double vr) {
    s_u[ip & 3][e_own] = vo;
    if (has_ring) s_u[ip & 3][e_ring] = vr;
  };
  struct Bv {
    double x, y, z, rx, ry, rz;
  };
  auto load_b = [&](int ip, Bv &b) {
    const long long base = plane_base(ip);
    b.x = a.b0[base + off_own];
    b.y = a.b1[base + off_own];
    b.z = a.b2[base + off_own];
    if (has_ring) {
      b.rx = a.b0[base + off_ring];
      b.ry = a.b1[base + off_ring];
      b.rz = a.b2[base + off_ring];
    }
  };
  // P1: tensors of plane ip (u of that plane already in the ring)
  Dten dn, dr;
  auto phase1 = [&](int ip, const Bv &b) {
    dn = spitzer_tensor(s_u[ip & 3][e_own], b.x, b.y, b.z, a.kappa0);
    s_d[D01][e_own] = dn.d01;
    s_d[D02][e_own] = dn.d02;
    s_d[D11][e_own] = dn.d11;
    s_d[D22][e_own] = dn.d22;
    s_d[D12][e_own] = dn.d12;
    if (has_ring) {
      dr = spitzer_tensor(s_u[ip & 3][e_ring], b.rx, b.ry, b.rz, a.kappa0);
      s_d[D01][e_ring] = dr.d01;
      s_d[D02][e_ring] = dr.d02;
      s_d[D11][e_ring] = dr.d11;
      s_d[D22][e_ring] = dr.d22;
      s_d[D12][e_ring] = dr.d12;
    }
  };
  // In-plane sums at an origin (e: its plane index) from the tensors in LDS:
  // D01 over (j, j+1), D02 over (k, k+1), and the in-plane coefficients.
  struct Sums {
    double b01, b02, w1, w2, k12;
  };
  auto sums = [&](int e, const Dten &d, const PlaneFac &f, double g1, double g2,
                  double g12) {
    Sums r;
    r.b01 = d.d01 + s_d[D01][e + QK];
    r.b02 = d.d02 + s_d[D02][e + 1];
    r.w1 = f.p1 * g1 * (0.5 * (d.d11 + s_d[D11][e + QK]));
    r.w2 = f.p2 * g2 * (0.5 * (d.d22 + s_d[D22][e + 1]));
    r.k12 = f.v * g12 *
            (0.0625 * (d.d12 + s_d[D12][e + QK] + s_d[D12][e + 1] + s_d[D12][e + QK + 1]));
    return r;
  };
  // carried state of the own origin: plane-i partial sums and coefficients
  double ca = 0.0;  // D00 of the own cell
  Sums cs{0.0, 0.0, 0.0, 0.0, 0.0};
  // P2 at plane ip (dn / dr hold the tensors of plane ip + 1) -> origin
  // coefficients of plane ip into s_c; carries move to plane ip + 1.
  // With first: only the carries of plane ip + 1 are formed (from plane ip+1 = ip0).
  double w0_own = 0.0, d00_own = 0.0;
  auto phase2 = [&](int ip, bool first) {
    const PlaneFac fn = plane_fac(g, wrapclamp(ip + 1, g.n0, g.per0));
    const Sums sn = sums(e_own, dn, fn, og.g1, og.g2, og.g12);
    if (!first) {
      const PlaneFac f = plane_fac(g, wrapclamp(ip, g.n0, g.per0));
      w0_own = f.p0 * og.g0 * (0.5 * (ca + dn.d00));
      d00_own = ca;
      s_c[C_W1][o_own] = cs.w1;
      s_c[C_W2][o_own] = cs.w2;
      s_c[C_K01][o_own] = f.vs * og.g01 * (0.0625 * (cs.b01 + sn.b01));
      s_c[C_K02][o_own] = f.vs * og.g02 * (0.0625 * (cs.b02 + sn.b02));
      s_c[C_K12][o_own] = cs.k12;
    }
    ca = dn.d00;
    cs = sn;
    if (has_low) {
      const Sums sl = sums(e_ring, dr, fn, s_lo[L_G1][tid], s_lo[L_G2][tid], s_lo[L_G12][tid]);
      if (!first) {
        const PlaneFac f = plane_fac(g, wrapclamp(ip, g.n0, g.per0));
        s_c[C_W1][o_low] = s_lo[L_W1][tid];
        s_c[C_W2][o_low] = s_lo[L_W2][tid];
        s_c[C_K01][o_low] = f.vs * s_lo[L_G01][tid] * (0.0625 * (s_lo[L_B01][tid] + sl.b01));
        s_c[C_K02][o_low] = f.vs * s_lo[L_G02][tid] * (0.0625 * (s_lo[L_B02][tid] + sl.b02));
        s_c[C_K12][o_low] = s_lo[L_K12][tid];
      }
      s_lo[L_B01][tid] = sl.b01;
      s_lo[L_B02][tid] = sl.b02;
      s_lo[L_W1][tid] = sl.w1;
      s_lo[L_W2][tid] = sl.w2;
      s_lo[L_K12][tid] = sl.k12;
    }
  };

  // ---- prologue: ring planes i0-1, i0, i0+1; origins of plane i0-1 ----
  {
    double vo, vr;
    load_u(i0 - 1, vo, vr);
    store_u(i0 - 1, vo, vr);
    load_u(i0, vo, vr);
    store_u(i0, vo, vr);
    load_u(i0 + 1, vo, vr);
    store_u(i0 + 1, vo, vr);
  }
  Bv bq;
  load_b(i0 - 1, bq);
  phase1(i0 - 1, bq);
  __syncthreads();
  phase2(i0 - 2, true);  // carries of plane i0 - 1
  __syncthreads();
  load_b(i0, bq);
  phase1(i0, bq);
  __syncthreads();
  phase2(i0 - 1, false);  // origins of plane i0 - 1; carries of plane i0
  __syncthreads();
  double pw0 = w0_own;
  double pk01 = s_c[C_K01][o_own], pk02 = s_c[C_K02][o_own];
  double pk01B = s_c[C_K01][o_own - OK], pk02C = s_c[C_K02][o_own - 1];

  const int j = j0 + tj, k = k0 + tk;
  const bool active = j < g.n1 && k < g.n2;
  const int jc = min(j, g.n1 - 1), kc = min(k, g.n2 - 1);
  ThreadGeo<double> tg;
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
  const double ab = T1(g, T_A01, jc) * T2(g, T_A02, kc);
  Grid gs = g;  // the row without its Dirichlet terms (added below from kappa(u))
  gs.dir_lo = gs.dir_hi = 0;

  double vo, vr;  // u of plane i + 2, loaded one iteration ahead
  if (i0 + 2 <= i1) load_u(i0 + 2, vo, vr);

  for (int i = i0; i < i1; ++i) {
    double von = 0.0, vrn = 0.0;
    if (i + 3 <= i1) load_u(i + 3, von, vrn);
    load_b(i + 1, bq);
    const long long cc = (long long)(i * g.n1 + jc) * g.n2 + kc;
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (MODE == NL_RK) {
      x0 = a.ukm2[cc];
      x1 = a.u0[cc];
      x2 = a.F0[cc];
    }
    phase1(i + 1, bq);
    __syncthreads();
    phase2(i, false);
    if (i + 2 <= i1) store_u(i + 2, vo, vr);
    __syncthreads();

    RowCoef<double> W;
    W.w0p = w0_own;
    W.w0m = pw0;
    W.w1p = s_c[C_W1][o_own];
    W.w1m = s_c[C_W1][o_own - OK];
    W.w2p = s_c[C_W2][o_own];
    W.w2m = s_c[C_W2][o_own - 1];
    W.K01[0] = s_c[C_K01][o_own];
    W.K01[1] = pk01;
    W.K01[2] = s_c[C_K01][o_own - OK];
    W.K01[3] = pk01B;
    W.K02[0] = s_c[C_K02][o_own];
    W.K02[1] = pk02;
    W.K02[2] = s_c[C_K02][o_own - 1];
    W.K02[3] = pk02C;
    W.K12[0] = s_c[C_K12][o_own];
    W.K12[1] = s_c[C_K12][o_own - OK];
    W.K12[2] = s_c[C_K12][o_own - 1];
    W.K12[3] = s_c[C_K12][o_own - OK - 1];
    if (active) {
      PlaneGeo<double> pg;
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
      const int base = (tj + 1) * QK + (tk + 1);
      const double *sm = s_u[(i - 1) & 3], *s0 = s_u[i & 3], *sp = s_u[(i + 1) & 3];
      auto U = [&](int di, int dj, int dk) -> double {
        const double *s = di < 0 ? sm : (di > 0 ? sp : s0);
        return s[base + dj * QK + dk];
      };
      double su = apply_S<OP_SPITZER, true, double, double>(gs, C, W, U, i, j, k, pg, tg);
      const double uc = s0[base];
      // Dirichlet faces on axis 0: w_b = A_b D_00(c) / (centre-to-face distance)
      const int bi = j * g.n2 + k;
      if (g.dir_lo && i == 0)
        su += g.ab_lo * ab * d00_own / g.db_lo * (C.ub_lo[bi] - uc);
      if (g.dir_hi && i == g.n0 - 1)
        su += g.ab_hi * ab * d00_own / g.db_hi * (C.ub_hi[bi] - uc);
      const double F = su / (pg.v0 * tg.v12);
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
    pw0 = w0_own;
    pk01 = W.K01[0];
    pk02 = W.K02[0];
    pk01B = W.K01[2];
    pk02C = W.K02[2];
    vo = von;
    vr = vrn;
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
    hipLaunchKernelGGL(k_march_nl<NL_F>, grid, block, 0, c->stream, c->grid(), C, a, CI, nchunk);
  else if (mode == NL_RK1)
    hipLaunchKernelGGL(k_march_nl<NL_RK1>, grid, block, 0, c->stream, c->grid(), C, a, CI,
                       nchunk);
  else
    hipLaunchKernelGGL(k_march_nl<NL_RK>, grid, block, 0, c->stream, c->grid(), C, a, CI,
                       nchunk);
}

}  // namespace sts
