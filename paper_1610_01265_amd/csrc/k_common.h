// Device helpers: grid indexing, separable geometry and the 19-point
// finite-volume operator of the lagged conduction term.
//
// The operator is S u = -dE/du of the discrete energy
//   E(u) = 1/2 sum_faces w_f (u_c' - u_c)^2 + sum_edges K_e X_e Y_e
//          + 1/2 sum_Dirichlet faces w_b (u_b - u_c)^2,
// where an edge in the (a, b) plane with origin cell e00 joins the cells
// e00, e10 = e00 + e_a, e01 = e00 + e_b, e11 = e00 + e_a + e_b, and
//   X = 1/2 [(u10 - u00)/dl_a(e00) + (u11 - u01)/dl_a(e01)]
//   Y = 1/2 [(u01 - u00)/dl_b(e00) + (u11 - u10)/dl_b(e10)].
// This is the cell-centred reading of the 19-point anisotropic conduction
// stencil (the paper's operators have p = 19 nonzeros per row, Appendix B);
// differentiating E gives, for the cell at role (p, q) of an edge,
//   (S u)_c += K/2 [ s_a Y / dl_a(face of c) + s_b X / dl_b(face of c) ],
// s_a = +1 if p = 0 else -1, s_b = +1 if q = 0 else -1.
#pragma once

#include "sts_internal.h"

namespace sts {

struct Nb {
  int m, p;    // index of the -1 / +1 neighbour (clamped into range when absent)
  bool hm, hp; // neighbour exists
};

__device__ __forceinline__ Nb nbr(int i, int n, int per) {
  Nb r;
  r.m = i - 1;
  r.p = i + 1;
  r.hm = true;
  r.hp = true;
  if (r.m < 0) {
    if (per) r.m = n - 1;
    else { r.m = 0; r.hm = false; }
  }
  if (r.p >= n) {
    if (per) r.p = 0;
    else { r.p = n - 1; r.hp = false; }
  }
  return r;
}

// Operands the FP64 RKL2 stage reads or writes once per sweep (u_{k-2}, u_0,
// F0, u_k), and the own-cell coefficients and outputs (p, A p) of the FP64
// conduction PCG pass A, are accessed non-temporally, leaving the caches to
// the halo and neighbour-coefficient re-reads (STS_NT=0 turns this off).
// Measured per kernel: the FP32 stages, the viscosity pass A and the
// element-wise PCG pass B ran slower this way.
#ifndef STS_NT
#define STS_NT 1
#endif
template <class T>
__device__ __forceinline__ T stream_ld(const T *p) {
  if (STS_NT) return __builtin_nontemporal_load(p);
  return *p;
}
// Lane l of a wavefront receives v from lane l - 1 (DPP wave_shr:1, a
// whole-wave shift); lane 0 receives lane0.  Every lane must be active.
__device__ __forceinline__ float wave_shr1(float v, float lane0) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(lane0), __float_as_int(v),
                                                    0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double wave_shr1(double v, double lane0) {
  const unsigned long long a = (unsigned long long)__double_as_longlong(v);
  const unsigned long long o = (unsigned long long)__double_as_longlong(lane0);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)a,
                                                            0x138, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32),
                                                            (int)(unsigned)(a >> 32), 0x138, 0xf,
                                                            0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// A load whose index is the same in every lane, through the scalar unit
// (for data that no kernel writes while the launch runs).
template <class T>
__device__ __forceinline__ T uniform_ld(const T *p, int idx) {
  return ((const __attribute__((address_space(4))) T *)p)[idx];
}
template <class T>
__device__ __forceinline__ void stream_st(T *p, T v) {
  if (STS_NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

__device__ __forceinline__ double T0(const Grid &g, int t, int i) { return g.t0[t * g.n0 + i]; }
__device__ __forceinline__ double T1(const Grid &g, int t, int j) { return g.t1[t * g.n1 + j]; }
__device__ __forceinline__ double T2(const Grid &g, int t, int k) { return g.t2[t * g.n2 + k]; }

__device__ __forceinline__ double vol(const Grid &g, int i, int j, int k) {
  return T0(g, T_V0, i) * T1(g, T_V1, j) * T2(g, T_V2, k);
}
__device__ __forceinline__ double il0(const Grid &g, int i) { return T0(g, T_IL00, i); }
__device__ __forceinline__ double il1(const Grid &g, int i, int j) {
  return T0(g, T_IL10, i) * T1(g, T_IL11, j);
}
__device__ __forceinline__ double il2(const Grid &g, int i, int j, int k) {
  return T0(g, T_IL20, i) * T1(g, T_IL21, j) * T2(g, T_IL22, k);
}
__device__ __forceinline__ double area0(const Grid &g, int i, int j, int k) {
  return T0(g, T_A00, i) * T1(g, T_A01, j) * T2(g, T_A02, k);
}
__device__ __forceinline__ double area1(const Grid &g, int i, int j, int k) {
  return T0(g, T_A10, i) * T1(g, T_A11, j) * T2(g, T_A12, k);
}
__device__ __forceinline__ double area2(const Grid &g, int i, int j, int k) {
  return T0(g, T_A20, i) * T1(g, T_A21, j) * T2(g, T_A22, k);
}

__device__ __forceinline__ int lin(const Grid &g, int i, int j, int k) {
  return (i * g.n1 + j) * g.n2 + k;
}

// Geometry of one edge touching cell (i, j, k), the cell being at role (p, q).
struct EdgeGeo {
  int e00;        // linear index of the edge origin (valid when ex)
  bool ex;        // the edge exists (all four cells in the domain)
  double ia0, ia1, ib0, ib1;  // 1/dl_a(e00), 1/dl_a(e01), 1/dl_b(e00), 1/dl_b(e10)
};

// PLANE 0: (a, b) = (0, 1); PLANE 1: (0, 2); PLANE 2: (1, 2)
template <int PLANE>
__device__ __forceinline__ EdgeGeo edge_geo(const Grid &g, int i, int j, int k, const Nb &A,
                                            const Nb &B, const Nb &C, int p, int q) {
  EdgeGeo e;
  if (PLANE == 0) {
    const int ei = p ? A.m : i, e10i = p ? i : A.p, ej = q ? B.m : j;
    e.ex = (p ? A.hm : A.hp) && (q ? B.hm : B.hp);
    e.ia0 = e.ia1 = il0(g, ei);
    e.ib0 = il1(g, ei, ej);
    e.ib1 = il1(g, e10i, ej);
    e.e00 = lin(g, ei, ej, k);
  } else if (PLANE == 1) {
    const int ei = p ? A.m : i, e10i = p ? i : A.p, ek = q ? C.m : k;
    e.ex = (p ? A.hm : A.hp) && (q ? C.hm : C.hp);
    e.ia0 = e.ia1 = il0(g, ei);
    e.ib0 = il2(g, ei, j, ek);
    e.ib1 = il2(g, e10i, j, ek);
    e.e00 = lin(g, ei, j, ek);
  } else {
    const int ej = p ? B.m : j, e10j = p ? j : B.p, ek = q ? C.m : k;
    e.ex = (p ? B.hm : B.hp) && (q ? C.hm : C.hp);
    e.ia0 = e.ia1 = il1(g, i, ej);
    e.ib0 = il2(g, i, ej, ek);
    e.ib1 = il2(g, i, e10j, ek);
    e.e00 = lin(g, i, ej, ek);
  }
  return e;
}

// Contribution of one edge to (S u)_c for the cell at role (p, q).
__device__ __forceinline__ double edge_term(double K, double u00, double u10, double u01,
                                            double u11, const EdgeGeo &e, int p, int q) {
  const double X = 0.5 * ((u10 - u00) * e.ia0 + (u11 - u01) * e.ia1);
  const double Y = 0.5 * ((u01 - u00) * e.ib0 + (u11 - u10) * e.ib1);
  const double ya = (q ? e.ia1 : e.ia0) * Y;
  const double xb = (p ? e.ib1 : e.ib0) * X;
  return 0.5 * K * ((p ? -ya : ya) + (q ? -xb : xb));
}

// Row c of S as a 3x3x3 array row[(dx+1)*9 + (dy+1)*3 + (dz+1)] = S[c, c+d]
// (only the 19 stencil entries can be non-zero).  OP: 1 conduction, 2 isotropic.
__device__ __forceinline__ void add_edge_row(double *row, int sa, int sb, double K,
                                             const EdgeGeo &e, int p, int q) {
  const double am = (p ? 0.5 : -0.5) * (q ? e.ia1 : e.ia0);
  const double bm = (q ? 0.5 : -0.5) * (p ? e.ib1 : e.ib0);
#pragma unroll
  for (int pp = 0; pp < 2; ++pp)
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      const double an = (pp ? 0.5 : -0.5) * (qq ? e.ia1 : e.ia0);
      const double bn = (qq ? 0.5 : -0.5) * (pp ? e.ib1 : e.ib0);
      row[13 + (pp - p) * sa + (qq - q) * sb] -= K * (am * bn + bm * an);
    }
}

template <int OP>
__device__ __forceinline__ void row27(const Grid &g, const Coef &C, int i, int j, int k,
                                      double *row) {
#pragma unroll
  for (int t = 0; t < 27; ++t) row[t] = 0.0;
  const Nb A = nbr(i, g.n0, g.per0), B = nbr(j, g.n1, g.per1), Cn = nbr(k, g.n2, g.per2);
  const int c = lin(g, i, j, k);
  double wp0, wm0, wp1, wm1, wp2, wm2;
  if (OP == OP_SPITZER) {
    wp0 = C.w0[c];
    wm0 = A.hm ? C.w0[lin(g, A.m, j, k)] : 0.0;
    wp1 = C.w1[c];
    wm1 = B.hm ? C.w1[lin(g, i, B.m, k)] : 0.0;
    wp2 = C.w2[c];
    wm2 = Cn.hm ? C.w2[lin(g, i, j, Cn.m)] : 0.0;
  } else {
    wp0 = C.nu * area0(g, i, j, k) * il0(g, i);
    wm0 = A.hm ? C.nu * area0(g, A.m, j, k) * il0(g, A.m) : 0.0;
    wp1 = C.nu * area1(g, i, j, k) * il1(g, i, j);
    wm1 = B.hm ? C.nu * area1(g, i, B.m, k) * il1(g, i, B.m) : 0.0;
    wp2 = C.nu * area2(g, i, j, k) * il2(g, i, j, k);
    wm2 = Cn.hm ? C.nu * area2(g, i, j, Cn.m) * il2(g, i, j, Cn.m) : 0.0;
  }
  row[13 + 9] += wp0;
  row[13 - 9] += wm0;
  row[13 + 3] += wp1;
  row[13 - 3] += wm1;
  row[13 + 1] += wp2;
  row[13 - 1] += wm2;
  row[13] -= wp0 + wm0 + wp1 + wm1 + wp2 + wm2;
  if (OP == OP_SPITZER) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        EdgeGeo e = edge_geo<0>(g, i, j, k, A, B, Cn, p, q);
        if (e.ex) add_edge_row(row, 9, 3, C.k01[e.e00], e, p, q);
        e = edge_geo<1>(g, i, j, k, A, B, Cn, p, q);
        if (e.ex) add_edge_row(row, 9, 1, C.k02[e.e00], e, p, q);
        e = edge_geo<2>(g, i, j, k, A, B, Cn, p, q);
        if (e.ex) add_edge_row(row, 3, 1, C.k12[e.e00], e, p, q);
      }
  }
  if (g.dir_lo && i == 0) row[13] -= C.wb_lo[j * g.n2 + k];
  if (g.dir_hi && i == g.n0 - 1) row[13] -= C.wb_hi[j * g.n2 + k];
}

}  // namespace sts
