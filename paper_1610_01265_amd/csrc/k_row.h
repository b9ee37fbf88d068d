// Row of the 19-point conduction operator (and of the 7-point isotropic
// operator) evaluated from a stencil-input window and per-cell face / edge
// coefficients, shared by the plane-marching kernels.
#pragma once

#include "k_common.h"

namespace sts {

namespace {

// Table reads at a wavefront-uniform index, through the constant address
// space so that they become scalar loads: as vector loads they would join the
// in-order count of outstanding vector loads, and waiting for them would also
// wait for every load issued before them (the next plane's prefetch).
typedef const __attribute__((address_space(4))) double cdouble;
__device__ __forceinline__ double T0u(const Grid &g, int t, int i) {
  return ((cdouble *)g.t0)[t * g.n0 + i];
}
__device__ __forceinline__ double T1u(const Grid &g, int t, int j) {
  return ((cdouble *)g.t1)[t * g.n1 + j];
}

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

// Coefficient arrays of the conduction operator in storage type CT.
template <class CT>
struct CoefS {
  const CT *w0, *w1, *w2, *k01, *k02, *k12;
  const double *wb_lo, *wb_hi, *ub_lo, *ub_hi;
  double nu;
};

template <class R>
struct PlaneGeo {
  Nb A;
  R s00m, s00, s10m, s10, s10p, s20m, s20, s20p, v0;
  R a00m, a00;  // isotropic: A00[i-1], A00[i]
  R a10, a20;   // isotropic: A10[i], A20[i]
};

template <class R>
struct ThreadGeo {
  Nb B, C;
  R t11m, t11, t21m, t21, t21p, t22m, t22, v12;
  R a01, a02, a01m, a11, a11m, a12, a21, a22, a22m;  // isotropic area factors
  int dJm, dKm;
};

template <class R>
struct EdgeG {
  R ia0, ia1, ib0, ib1;
};

// Contribution of one edge to (S u)_c for the cell at role (p, q).
template <class R>
__device__ __forceinline__ R edge_term_r(R K, R u00, R u10, R u01, R u11, const EdgeG<R> &e,
                                         int p, int q) {
  const R h = R(0.5);
  const R X = h * ((u10 - u00) * e.ia0 + (u11 - u01) * e.ia1);
  const R Y = h * ((u01 - u00) * e.ib0 + (u11 - u10) * e.ib1);
  const R ya = (q ? e.ia1 : e.ia0) * Y;
  const R xb = (p ? e.ib1 : e.ib0) * X;
  return h * K * ((p ? -ya : ya) + (q ? -xb : xb));
}

// Coefficients of one cell's row of the conduction operator: its own +face
// and edge coefficients and those of its -1 neighbours.  Edge order (p, q):
// (0,0), (1,0), (0,1), (1,1) (p / q = 1: the edge's origin is one cell back
// along the plane's first / second axis).
template <class R>
struct RowCoef {
  R w0p, w0m, w1p, w1m, w2p, w2m;
  R K01[4], K02[4], K12[4];
};

// (S u)_c (+ g_c when WITH_G), u read through U(di, dj, dk); arithmetic in R.
template <int OP, bool WITH_G, class R, class CT, class UF>
__device__ __forceinline__ R apply_S(const Grid &g, const CoefS<CT> &C, const RowCoef<R> &W,
                                     const UF &U, int i, int j, int k,
                                     const PlaneGeo<R> &pg, const ThreadGeo<R> &tg) {
  const R u0 = U(0, 0, 0);
  const R zero = R(0);
  R acc;
  if (OP == OP_SPITZER) {
    acc = W.w0p * (U(1, 0, 0) - u0) + (pg.A.hm ? W.w0m : zero) * (U(-1, 0, 0) - u0);
    acc += W.w1p * (U(0, 1, 0) - u0) + (tg.B.hm ? W.w1m : zero) * (U(0, -1, 0) - u0);
    acc += W.w2p * (U(0, 0, 1) - u0) + (tg.C.hm ? W.w2m : zero) * (U(0, 0, -1) - u0);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int r = p + 2 * q;
        // plane (0, 1)
        {
          const bool ex = (p ? pg.A.hm : pg.A.hp) && (q ? tg.B.hm : tg.B.hp);
          EdgeG<R> e;
          e.ia0 = e.ia1 = p ? pg.s00m : pg.s00;
          const R tj = q ? tg.t11m : tg.t11;
          e.ib0 = (p ? pg.s10m : pg.s10) * tj;
          e.ib1 = (p ? pg.s10 : pg.s10p) * tj;
          acc += edge_term_r<R>(ex ? W.K01[r] : zero, U(-p, -q, 0), U(1 - p, -q, 0),
                                U(-p, 1 - q, 0), U(1 - p, 1 - q, 0), e, p, q);
        }
        // plane (0, 2)
        {
          const bool ex = (p ? pg.A.hm : pg.A.hp) && (q ? tg.C.hm : tg.C.hp);
          EdgeG<R> e;
          e.ia0 = e.ia1 = p ? pg.s00m : pg.s00;
          const R tk = q ? tg.t22m : tg.t22;
          e.ib0 = (p ? pg.s20m : pg.s20) * tg.t21 * tk;
          e.ib1 = (p ? pg.s20 : pg.s20p) * tg.t21 * tk;
          acc += edge_term_r<R>(ex ? W.K02[r] : zero, U(-p, 0, -q), U(1 - p, 0, -q),
                                U(-p, 0, 1 - q), U(1 - p, 0, 1 - q), e, p, q);
        }
        // plane (1, 2)
        {
          const bool ex = (p ? tg.B.hm : tg.B.hp) && (q ? tg.C.hm : tg.C.hp);
          EdgeG<R> e;
          e.ia0 = e.ia1 = pg.s10 * (p ? tg.t11m : tg.t11);
          const R tk = q ? tg.t22m : tg.t22;
          e.ib0 = pg.s20 * (p ? tg.t21m : tg.t21) * tk;
          e.ib1 = pg.s20 * (p ? tg.t21 : tg.t21p) * tk;
          acc += edge_term_r<R>(ex ? W.K12[r] : zero, U(0, -p, -q), U(0, 1 - p, -q),
                                U(0, -p, 1 - q), U(0, 1 - p, 1 - q), e, p, q);
        }
      }
  } else {
    // nu * (area / distance) on each face, from the separable tables
    const R w0p = pg.a00 * tg.a01 * tg.a02 * pg.s00;
    const R w0m = pg.a00m * tg.a01 * tg.a02 * pg.s00m;
    const R w1p = pg.a10 * tg.a11 * tg.a12 * (pg.s10 * tg.t11);
    const R w1m = pg.a10 * tg.a11m * tg.a12 * (pg.s10 * tg.t11m);
    const R w2p = pg.a20 * tg.a21 * tg.a22 * (pg.s20 * tg.t21 * tg.t22);
    const R w2m = pg.a20 * tg.a21 * tg.a22m * (pg.s20 * tg.t21 * tg.t22m);
    acc = w0p * (U(1, 0, 0) - u0) + (pg.A.hm ? w0m : zero) * (U(-1, 0, 0) - u0);
    acc += w1p * (U(0, 1, 0) - u0) + (tg.B.hm ? w1m : zero) * (U(0, -1, 0) - u0);
    acc += w2p * (U(0, 0, 1) - u0) + (tg.C.hm ? w2m : zero) * (U(0, 0, -1) - u0);
    acc *= R(C.nu);
  }
  if ((g.dir_lo && i == 0) || (g.dir_hi && i == g.n0 - 1)) {
    const int bi = j * g.n2 + k;
    const bool lo = g.dir_lo && i == 0;
    const R wb = lo ? C.wb_lo[bi] : C.wb_hi[bi];
    const R ub = lo ? C.ub_lo[bi] : C.ub_hi[bi];
    acc += WITH_G ? wb * (ub - u0) : -wb * u0;
    if (g.dir_lo && g.dir_hi && i == 0 && i == g.n0 - 1) {  // single radial cell
      const R wh = C.wb_hi[bi], uh = C.ub_hi[bi];
      acc += WITH_G ? wh * (uh - u0) : -wh * u0;
    }
  }
  return acc;
}

}  // namespace

}  // namespace sts
