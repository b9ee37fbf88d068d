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
#include "k_reduce.h"
#include "k_row.h"

#include <algorithm>
#include <type_traits>

namespace sts {

namespace {

#ifndef STS_MARCH_TJ
#define STS_MARCH_TJ 4
#endif
#ifndef STS_MARCH_WG
#define STS_MARCH_WG 1024  // about one round of 4 workgroups per CU
#endif
// The stencil-input plane staged into LDS at the end of iteration i is
// loaded after that plane's per-cell operands and on every lane and
// iteration: vector loads complete in order, so the row's wait for its
// operands does not wait for the prefetch, which stays in flight across the
// row.
constexpr int TK = 64, TJ = STS_MARCH_TJ, NT = TK * TJ;
// the in-sweep PCG reductions (block_sum_parts) assume 256-thread workgroups
static_assert(NT == 256, "march workgroups must have 256 threads");
constexpr int HK = TK + 2, HJ = TJ + 2, PL = HK * HJ;  // one LDS plane (tile + halo)
constexpr int NLOAD = (PL + NT - 1) / NT;

enum {
  M_F = 0,      // out = F(u)
  M_RK1 = 1,    // RKL2 stage 1: F0 = F(u_0), out = u_0 + mu~_1 dt F0
  M_RK = 2,     // RKL2 stage k >= 2
  M_PA = 3,     // PCG pass A: p, y = A p, partial p.y
  M_RES = 4,    // r = b - A x, partial r.r, b.b
  M_RESN = 5,   // partial norms of b - A x only
  M_F0F = 6,    // FP32 form: F0 = F(u_0) evaluated in FP64, stored FP32
  M_DK = 7,     // FP32 form stage k: delta_k from delta_{k-1}, delta_{k-2}, F0
  M_DLAST = 8   // FP32 form last stage: u^{n+1} = u_0 + delta_s (FP64)
};

template <class T>
struct LoadU {
  using value_type = T;
  const T *__restrict__ u;
  __device__ __forceinline__ void prepare() {}
  __device__ __forceinline__ T operator()(long long idx) const { return u[idx]; }
};

// p = z + beta p_old, with z = M^-1 r stored by the previous pass (Jacobi:
// r / A_ii from pass B or the initialisation; block ILU0: the substitution).
template <class T>
struct LoadP {
  using value_type = T;
  const T *__restrict__ z;
  const T *__restrict__ pold;
  const PcgScalars *sc;
  int first;
  T beta;
  __device__ __forceinline__ void prepare() { beta = first ? T(0) : T(sc->beta); }
  __device__ __forceinline__ void set_beta(double b) { beta = T(b); }
  __device__ __forceinline__ T operator()(long long idx) const {
    return first ? z[idx] : z[idx] + beta * pold[idx];
  }
};

// Operands of the consumer of F; their element types depend on the mode.
struct Args {
  void *out;           // F, u_k, delta_k, p (pass A), r (residual), u^{n+1}
  void *F0;            // RKL2 F(u_0)
  const void *ukm2;    // RKL2 u_{k-2} / delta_{k-2}
  const double *u0;    // RKL2 u_0 (FP64)
  const double *b;     // residual: right-hand side
  void *y;             // pass A: A p
  double *part;        // per-workgroup partial sums (two regions of cap)
  long long cap;
  double mu, nu, mut_dt, gt_dt, dt;
  PcgScalars *sc;
  const double *pb;  // pass A after a fused pass B: its partials (r.z, r.r), else null
  int npb;           // their count per region (regions cap apart)
  int iters;         // iterations completed before this sweep
};

#ifndef STS_MARCH_WPE
#define STS_MARCH_WPE 4  // waves per SIMD the register allocation must allow
#endif
template <int OP, int MODE, class Loader, class CT>
__global__ void __launch_bounds__(NT, STS_MARCH_WPE)
    k_march(Grid g, CoefS<CT> C, Loader ld, Args a, int CI, int nchunk, long long ncell) {
  using R = typename Loader::value_type;
  if (MODE == M_PA && a.sc->done) return;
  __shared__ R s_u[4][PL];
  __shared__ R s_cf[3][TJ][TK];  // w1, k01, k12 of the tile's rows (cross-lane modes)
  if constexpr (MODE == M_PA) {
    if (a.pb) {
      // the previous iteration's stopping test and this one's beta, from the
      // fused pass B's partials (identical in every workgroup)
      double beta;
      if (pcg_decide(a.pb, a.npb, a.cap, a.iters, a.sc, blockIdx.x == 0,
                     (int)(threadIdx.y * TK + threadIdx.x), &beta))
        return;
      ld.set_beta(beta);
    } else {
      ld.prepare();
    }
  } else {
    ld.prepare();
  }
  // a wavefront is one tile row (blockDim.x = 64): theta-dependent values
  // are uniform across it
  const int tk = threadIdx.x, tj = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int tid = tj * TK + tk;
  // XCD-aware order: workgroup w runs on XCD w % 8; each XCD gets a
  // contiguous range of the logical (chunk, row-tile, column-tile) order.
  const int nwg = gridDim.x, w = wg_index(g.wg_rev);
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
  auto load_plane = [&](int ip, R *v) {
    const long long base = off + (long long)wrapclamp(ip, g.n0, g.per0) * n12;
#pragma unroll
    for (int q = 0; q < NLOAD; ++q) v[q] = ld(base + hoff[q]);
  };
  auto store_plane = [&](int ip, const R *v) {
    R *s = s_u[ip & 3];
#pragma unroll
    for (int q = 0; q < NLOAD; ++q)
      if (tid + q * NT < PL) s[tid + q * NT] = v[q];
  };
  R v[NLOAD];
  load_plane(i0 - 1, v);
  store_plane(i0 - 1, v);
  load_plane(i0, v);
  store_plane(i0, v);
  load_plane(i0 + 1, v);
  store_plane(i0 + 1, v);

  const int j = j0 + tj, k = k0 + tk;
  const bool active = j < g.n1 && k < g.n2;
  const int jc = min(j, g.n1 - 1), kc = min(k, g.n2 - 1);
  ThreadGeo<R> tg;
  tg.B = nbr(jc, g.n1, g.per1);
  tg.C = nbr(kc, g.n2, g.per2);
  tg.t11m = T1u(g, T_IL11, tg.B.m);
  tg.t11 = T1u(g, T_IL11, jc);
  tg.t21m = T1u(g, T_IL21, tg.B.m);
  tg.t21 = T1u(g, T_IL21, jc);
  tg.t21p = T1u(g, T_IL21, tg.B.p);
  tg.t22m = T2(g, T_IL22, tg.C.m);
  tg.t22 = T2(g, T_IL22, kc);
  tg.v12 = T1(g, T_V1, jc) * T2(g, T_V2, kc);
  const R iv12 = R(1) / tg.v12;
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
  // Per-plane loads of this thread, issued one plane ahead of their use:
  // the conduction coefficients of the cell and of its (j-1), (k-1) and
  // (j-1, k-1) neighbours in the same plane, and the consumer's operands.
  // Coefficients of the previous plane are carried in registers.  Inactive
  // threads load at their clamped cell, so every address is in the grid.
  struct Loads {
    R w0, w1, w2, k01, k02, k12;
    R w1B, k01B, k12B, w2C, k02C, k12C, k12BC;
    R x0, x2;   // RKL2: u_{k-2}, F0; FP32 stages: delta_{k-2}, F0
    double x1;  // RKL2 / last FP32 stage: u_0; residuals: b
  };
  // own-cell streams (HBM) of plane ip
  auto load_own = [&](int ip, Loads &L) {
    const int c = (ip * g.n1 + jc) * g.n2 + kc;
    if (OP == OP_SPITZER) {
      L.w0 = R(C.w0[c]);
      L.w1 = R(C.w1[c]);
      L.w2 = R(C.w2[c]);
      L.k01 = R(C.k01[c]);
      L.k02 = R(C.k02[c]);
      L.k12 = R(C.k12[c]);
    }
    const long long cc = off + c;
    if (MODE == M_RK || MODE == M_DK || MODE == M_DLAST) {
      // FP64 stages stream these operands non-temporally; the FP32 stages
      // measured slower that way
      if (MODE == M_RK) {
        L.x0 = stream_ld(&((const R *)a.ukm2)[cc]);
        L.x2 = stream_ld(&((const R *)a.F0)[cc]);
      } else {
        L.x0 = ((const R *)a.ukm2)[cc];
        L.x2 = ((const R *)a.F0)[cc];
      }
    }
    if (MODE == M_RK) L.x1 = stream_ld(&a.u0[cc]);
    if (MODE == M_DLAST) L.x1 = a.u0[cc];
    if (MODE == M_RES || MODE == M_RESN) L.x1 = a.b[cc];
  };
  // Same-plane neighbour coefficients of plane ip.  Every one of them is
  // some thread's own value, passed between threads: the (k - 1) neighbours
  // by a whole-wave DPP shift (a wavefront is 64 consecutive k of one row;
  // lane 0 reads the column left of the tile through the scalar unit), the
  // (j - 1) neighbours through LDS from the wavefront of the row above (the
  // first row loads them).  This needs the own values first and a barrier;
  // measured at 256 x 256 x 512: -8 % per RKL2 stage and -4.4 % per
  // Jacobi-PCG iteration (pass A with cached coefficient loads, which beat
  // non-temporal ones with or without the exchange).  The FP32 form's pass
  // A measured +1.7 % with it and keeps the loads.
  constexpr bool xlane = OP == OP_SPITZER && (MODE != M_PA || sizeof(R) == 8);
  auto load_nbr = [&](int ip, Loads &L) {
    if (OP == OP_SPITZER) {
      const int c = (ip * g.n1 + jc) * g.n2 + kc;
      const int cB = c + tg.dJm;
      if constexpr (xlane) {
        if (tj < TJ - 1) {
          s_cf[0][tj][tk] = L.w1;
          s_cf[1][tj][tk] = L.k01;
          s_cf[2][tj][tk] = L.k12;
        }
        if (tj == 0) {
          L.w1B = R(C.w1[cB]);
          L.k01B = R(C.k01[cB]);
          L.k12B = R(C.k12[cB]);
        }
        __syncthreads();
        if (tj > 0) {
          L.w1B = s_cf[0][tj - 1][tk];
          L.k01B = s_cf[1][tj - 1][tk];
          L.k12B = s_cf[2][tj - 1][tk];
        }
        const int cC0 = __builtin_amdgcn_readfirstlane(c + tg.dKm);
        const int cBC0 = __builtin_amdgcn_readfirstlane(cB + tg.dKm);
        L.w2C = wave_shr1(L.w2, R(uniform_ld(C.w2, cC0)));
        L.k02C = wave_shr1(L.k02, R(uniform_ld(C.k02, cC0)));
        L.k12C = wave_shr1(L.k12, R(uniform_ld(C.k12, cC0)));
        L.k12BC = wave_shr1(L.k12B, R(uniform_ld(C.k12, cBC0)));
      } else {
        const int cC = c + tg.dKm;
        L.w1B = R(C.w1[cB]);
        L.k01B = R(C.k01[cB]);
        L.k12B = R(C.k12[cB]);
        L.w2C = R(C.w2[cC]);
        L.k02C = R(C.k02[cC]);
        L.k12C = R(C.k12[cC]);
        L.k12BC = R(C.k12[cB + tg.dKm]);
      }
    }
  };
  // Conduction: the part of the row of the cell of plane i that the faces and
  // edges joining planes i - 1 and i contribute, evaluated with plane i - 1
  // (r_terms) and carried in a register.  At the chunk start it is formed
  // here from plane i0 - 1 (its coefficients loaded, its u in the ring).
  const int base = (tj + 1) * HK + (tk + 1);
  R carry = R(0);
  R pw0 = R(0), pk01 = R(0), pk02 = R(0), pk01B = R(0), pk02C = R(0);
  const Nb A0 = nbr(i0, g.n0, g.per0);
  if (OP == OP_SPITZER && A0.hm) {
    const int cA = (A0.m * g.n1 + jc) * g.n2 + kc;
    pw0 = R(C.w0[cA]);
    pk01 = R(C.k01[cA]);
    pk02 = R(C.k02[cA]);
    pk01B = R(C.k01[cA + tg.dJm]);
    pk02C = R(C.k02[cA + tg.dKm]);
  }
  Loads cur;
  double acc_a = 0.0, acc_b = 0.0;
  __syncthreads();
  if (OP == OP_SPITZER && A0.hm && active) {
    const R *sl = s_u[(i0 - 1) & 3], *sh = s_u[i0 & 3];
    auto Ul = [&](int dj, int dk) -> R { return sl[base + dj * HK + dk]; };
    auto Uh = [&](int dj, int dk) -> R { return sh[base + dj * HK + dk]; };
    const int ip = A0.m;
    const R K01q[2] = {tg.B.hp ? pk01 : R(0), tg.B.hm ? pk01B : R(0)};
    const R K02q[2] = {tg.C.hp ? pk02 : R(0), tg.C.hm ? pk02C : R(0)};
    R lo;
    r_terms<R>(Ul, Uh, pw0, K01q, K02q, R(0.25) * R(T0u(g, T_IL00, ip)), R(T0u(g, T_IL10, ip)),
               R(T0u(g, T_IL10, i0)), R(T0u(g, T_IL20, ip)), R(T0u(g, T_IL20, i0)), tg, lo,
               carry);
  }

  for (int i = i0; i < i1; ++i) {
    const bool pre = i + 2 <= i1;
    load_own(i, cur);
    if (!xlane) load_nbr(i, cur);
    load_plane(i + 2, v);  // clamped / wrapped plane index: always in the grid
    if (xlane) load_nbr(i, cur);  // waits for the own values and the other rows
    // The RKL2 stage output is stored after the LDS ring update below: the
    // vector-memory counter also counts stores, so a store issued before the
    // update would make its wait for the prefetched plane wait for the store
    // as well (measured: -2 % per stage).
    R st_a = R(0);
    long long st_c = 0;
    if (active) {
      PlaneGeo<R> pg;
      pg.A = nbr(i, g.n0, g.per0);
      pg.s00 = T0u(g, T_IL00, i);
      pg.s10 = T0u(g, T_IL10, i);
      pg.s20 = T0u(g, T_IL20, i);
      pg.v0 = T0u(g, T_V0, i);
      if (OP == OP_ISOTROPIC) {
        pg.s00m = T0u(g, T_IL00, pg.A.m);
        pg.a00 = T0u(g, T_A00, i);
        pg.a00m = T0u(g, T_A00, pg.A.m);
        pg.a10 = T0u(g, T_A10, i);
        pg.a20 = T0u(g, T_A20, i);
      }
      const R *sm = s_u[(i - 1) & 3], *s0 = s_u[i & 3], *sp = s_u[(i + 1) & 3];
      auto U = [&](int di, int dj, int dk) -> R {
        const R *s = di < 0 ? sm : (di > 0 ? sp : s0);
        return s[base + dj * HK + dk];
      };
      RowCoef<R> W;
      if (OP == OP_SPITZER) {
        W.w1p = cur.w1;
        W.w1m = cur.w1B;
        W.w2p = cur.w2;
        W.w2m = cur.w2C;
        W.K12[0] = cur.k12;
        W.K12[1] = cur.k12B;
        W.K12[2] = cur.k12C;
        W.K12[3] = cur.k12BC;
      }
      const int c = (i * g.n1 + j) * g.n2 + k;
      const long long cc = off + c;
      constexpr bool with_g = MODE == M_F || MODE == M_RK1 || MODE == M_RK || MODE == M_F0F;
      R su;
      if (OP == OP_SPITZER) {
        auto Ul = [&](int dj, int dk) -> R { return s0[base + dj * HK + dk]; };
        auto Uh = [&](int dj, int dk) -> R { return sp[base + dj * HK + dk]; };
        const bool hp = pg.A.hp;
        const R K01q[2] = {hp && tg.B.hp ? cur.k01 : R(0), hp && tg.B.hm ? cur.k01B : R(0)};
        const R K02q[2] = {hp && tg.C.hp ? cur.k02 : R(0), hp && tg.C.hm ? cur.k02C : R(0)};
        R lo, hi;
        r_terms<R>(Ul, Uh, cur.w0, K01q, K02q, R(0.25) * pg.s00, pg.s10,
                   R(T0u(g, T_IL10, pg.A.p)), pg.s20, R(T0u(g, T_IL20, pg.A.p)), tg, lo, hi);
        su = carry + lo + inplane_S<R>(W, Ul, pg.s10, pg.s20, tg) +
             dirichlet_terms<with_g, R, CT>(g, C, i, j, k, s0[base]);
        carry = hi;
      } else {
        su = apply_S<OP, with_g, R, CT>(g, C, W, U, i, j, k, pg, tg);
      }
      const R V = pg.v0 * tg.v12;
      const R iV = R(T0u(g, T_IV0, i)) * iv12;
      const R uc = s0[base];
      if (MODE == M_F) {
        ((R *)a.out)[cc] = su * iV;
      } else if (MODE == M_F0F) {
        const float F = (float)(su * iV);
        ((float *)a.F0)[cc] = F;
        if (a.out) ((float *)a.out)[cc] = (float)a.mut_dt * F;  // delta_1 = mu~_1 dt F0
      } else if (MODE == M_RK1) {
        const R F = su * iV;
        stream_st(&((R *)a.F0)[cc], F);
        stream_st(&((R *)a.out)[cc], uc + R(a.mut_dt) * F);
      } else if (MODE == M_RK) {
        const R F = su * iV;
        st_a = R(a.mu) * uc + R(a.nu) * cur.x0 + (R(1) - R(a.mu) - R(a.nu)) * R(cur.x1) +
               R(a.mut_dt) * F + R(a.gt_dt) * cur.x2;
        st_c = cc;
      } else if (MODE == M_DK || MODE == M_DLAST) {
        // delta_k = mu delta_{k-1} + nu delta_{k-2} + mu~ dt M delta_{k-1}
        //           + (mu~ + gamma~) dt F0      (gt_dt carries (mu~ + gamma~) dt)
        const R d = R(a.mu) * uc + R(a.nu) * cur.x0 + R(a.mut_dt) * (su * iV) +
                    R(a.gt_dt) * cur.x2;
        if (MODE == M_DK)
          ((R *)a.out)[cc] = d;
        else
          ((double *)a.out)[cc] = cur.x1 + (double)d;
      } else if (MODE == M_PA) {
        const R yv = V * uc - R(a.dt) * su;
        if (OP == OP_SPITZER && sizeof(R) == 8) {
          stream_st(&((R *)a.out)[cc], uc);
          stream_st(&((R *)a.y)[cc], yv);
        } else {
          ((R *)a.out)[cc] = uc;
          ((R *)a.y)[cc] = yv;
        }
        acc_a += (double)uc * (double)yv;
      } else {  // residual r = b - A x
        const double bv = cur.x1;
        const double rv = bv - (double)(V * uc - R(a.dt) * su);
        if (MODE == M_RES) ((double *)a.out)[cc] = rv;
        acc_a += rv * rv;
        acc_b += bv * bv;
      }
    }
    if (pre) store_plane(i + 2, v);
    if (MODE == M_RK && active) stream_st(&((R *)a.out)[st_c], st_a);
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

template <class CT>
CoefS<CT> coef_of(const sts_ctx *c) {
  const Coef k = c->coef();
  CoefS<CT> s;
  const CT *w = (const CT *)(std::is_same<CT, float>::value ? (const void *)c->d_wf
                                                              : (const void *)c->d_w);
  const long long n = c->ncell;
  s.w0 = w;
  s.w1 = w ? w + n : nullptr;
  s.w2 = w ? w + 2 * n : nullptr;
  s.k01 = w ? w + 3 * n : nullptr;
  s.k02 = w ? w + 4 * n : nullptr;
  s.k12 = w ? w + 5 * n : nullptr;
  s.wb_lo = k.wb_lo;
  s.wb_hi = k.wb_hi;
  s.ub_lo = k.ub_lo;
  s.ub_hi = k.ub_hi;
  s.nu = k.nu;
  return s;
}

template <int OP, int MODE, class CT, class Loader>
void launch(const sts_ctx *c, int ncomp, const Loader &ld, const Args &a) {
  int CI, nchunk;
  const dim3 grid = march_grid(c, ncomp, &CI, &nchunk);
  hipLaunchKernelGGL((k_march<OP, MODE, Loader, CT>), grid, dim3(TK, TJ), 0, c->stream,
                     c->grid(), coef_of<CT>(c), ld, a, CI, nchunk, c->ncell);
}

template <int MODE, class Loader>
void launch_op(const sts_ctx *c, int ncomp, const Loader &ld, const Args &a) {
  if (c->op == OP_SPITZER)
    launch<OP_SPITZER, MODE, double>(c, ncomp, ld, a);
  else
    launch<OP_ISOTROPIC, MODE, double>(c, ncomp, ld, a);
}

}  // namespace

int stencil_parts(const sts_ctx *c) {
  int CI, nchunk;
  const dim3 g = march_grid(c, 1, &CI, &nchunk);
  return (int)(g.x * g.y * g.z);
}

void launch_stage(const sts_ctx *c, int mode, int ncomp, const double *ukm1, const double *ukm2,
                  const double *u0, double *F0, double *out, double mu, double nu, double mut_dt,
                  double gt_dt) {
  STS_PROF(c, mode == 0 ? "stage_F" : (mode == 1 ? "stage_rk_first" : "stage_rk"));
  Args a{};
  a.out = out;
  a.F0 = F0;
  a.ukm2 = ukm2;
  a.u0 = u0;
  a.mu = mu;
  a.nu = nu;
  a.mut_dt = mut_dt;
  a.gt_dt = gt_dt;
  const LoadU<double> ld{ukm1};
  if (mode == 0)
    launch_op<M_F>(c, ncomp, ld, a);
  else if (mode == 1)
    launch_op<M_RK1>(c, ncomp, ld, a);
  else
    launch_op<M_RK>(c, ncomp, ld, a);
}

void launch_pass_a(const sts_ctx *c, double dt, const double *z, const double *pold,
                   double *pnew, double *y, double *part, const PcgScalars *sc, int first,
                   const double *pb, int npb, int iters) {
  STS_PROF(c, "launch_pass_a");
  Args a{};
  a.out = pnew;
  a.y = y;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  a.sc = (PcgScalars *)sc;
  a.pb = first ? nullptr : pb;
  a.npb = npb;
  a.iters = iters;
  const LoadP<double> ld{z, pold, sc, first, 0.0};
  launch_op<M_PA>(c, 1, ld, a);
}

void launch_residual_init(const sts_ctx *c, const double *b, const double *x, double dt,
                          const double *, const double *, double *r, double *, double *part) {
  STS_PROF(c, "launch_residual_init");
  Args a{};
  a.out = r;
  a.b = b;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  launch_op<M_RES>(c, 1, LoadU<double>{x}, a);
}

void launch_true_residual(const sts_ctx *c, const double *b, const double *x, double dt,
                          double *part) {
  STS_PROF(c, "launch_true_residual");
  Args a{};
  a.b = b;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  launch_op<M_RESN>(c, 1, LoadU<double>{x}, a);
}

}  // namespace sts

namespace sts {

// ---------------------------------------------------------------------------
// FP32 form (coefficients stored FP32; d_wf).  The stage arithmetic is FP32;
// F(u_0) and the outer residual evaluate the stencil in FP64 from the FP64
// state with the FP32 coefficients widened.
// ---------------------------------------------------------------------------
namespace {
template <int MODE, class Loader>
void launch_f32(const sts_ctx *c, int ncomp, const Loader &ld, const Args &a) {
  if (c->op == OP_SPITZER)
    launch<OP_SPITZER, MODE, float>(c, ncomp, ld, a);
  else
    launch<OP_ISOTROPIC, MODE, float>(c, ncomp, ld, a);
}
}  // namespace

void f32_F0(const sts_ctx *c, int ncomp, const double *u0, float *F0, float *d1, double mut_dt) {
  STS_PROF(c, "f32_F0");
  Args a{};
  a.F0 = F0;
  a.out = d1;
  a.mut_dt = mut_dt;
  launch_f32<M_F0F>(c, ncomp, LoadU<double>{u0}, a);
}

void f32_apply(const sts_ctx *c, int ncomp, const double *u, double *Fu) {
  STS_PROF(c, "f32_apply");
  Args a{};
  a.out = Fu;
  launch_f32<M_F>(c, ncomp, LoadU<double>{u}, a);
}

void f32_stage(const sts_ctx *c, int last, int ncomp, const float *dkm1, const float *dkm2,
               const float *F0, void *out, const double *u0, double mu, double nu, double mut_dt,
               double g_dt) {
  STS_PROF(c, "f32_stage");
  Args a{};
  a.out = out;
  a.ukm2 = dkm2;
  a.F0 = const_cast<float *>(F0);
  a.u0 = u0;
  a.mu = mu;
  a.nu = nu;
  a.mut_dt = mut_dt;
  a.gt_dt = g_dt;
  if (last)
    launch_f32<M_DLAST>(c, ncomp, LoadU<float>{dkm1}, a);
  else
    launch_f32<M_DK>(c, ncomp, LoadU<float>{dkm1}, a);
}

void f32_pass_a(const sts_ctx *c, double dt, const float *z, const float *pold, float *pnew,
                float *y, double *part, const PcgScalars *sc, int first, const double *pb,
                int npb, int iters) {
  STS_PROF(c, "f32_pass_a");
  Args a{};
  a.out = pnew;
  a.y = y;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  a.sc = (PcgScalars *)sc;
  a.pb = first ? nullptr : pb;
  a.npb = npb;
  a.iters = iters;
  const LoadP<float> ld{z, pold, sc, first, 0.0f};
  launch_f32<M_PA>(c, 1, ld, a);
}

void f32_residual(const sts_ctx *c, const double *b, const double *x, double dt, double *r,
                  double *part) {
  STS_PROF(c, "f32_residual");
  Args a{};
  a.out = r;
  a.b = b;
  a.part = part;
  a.cap = c->red_cap;
  a.dt = dt;
  if (r)
    launch_f32<M_RES>(c, 1, LoadU<double>{x}, a);
  else
    launch_f32<M_RESN>(c, 1, LoadU<double>{x}, a);
}

}  // namespace sts
