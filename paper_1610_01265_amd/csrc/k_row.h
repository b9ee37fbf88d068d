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

// Dirichlet faces of a cell on a Dirichlet side of axis 0: -w_b u_c, plus the
// boundary term g_c = w_b u_b when WITH_G.
template <bool WITH_G, class R, class CT>
__device__ __forceinline__ R dirichlet_terms(const Grid &g, const CoefS<CT> &C, int i, int j,
                                             int k, R u0) {
  R acc = R(0);
  if ((g.dir_lo && i == 0) || (g.dir_hi && i == g.n0 - 1)) {
    const int bi = j * g.n2 + k;
    const bool lo = g.dir_lo && i == 0;
    const R wb = lo ? C.wb_lo[bi] : C.wb_hi[bi];
    const R ub = lo ? C.ub_lo[bi] : C.ub_hi[bi];
    acc = WITH_G ? wb * (ub - u0) : -wb * u0;
    if (g.dir_lo && g.dir_hi && i == 0 && i == g.n0 - 1) {  // single radial cell
      const R wh = C.wb_hi[bi], uh = C.ub_hi[bi];
      acc += WITH_G ? wh * (uh - u0) : -wh * u0;
    }
  }
  return acc;
}

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
  return acc + dirichlet_terms<WITH_G, R, CT>(g, C, i, j, k, u0);
}

// The march form of the conduction row.  The terms that join plane ip to
// plane ip + 1 in the column of cell (j, k) -- its +r face and the four edges
// of the (r, theta) and (r, phi) planes with origin (ip, j - q, k) and
// (ip, j, k - q), q = 0, 1 -- are evaluated once, for both cells they touch:
// `lo` is their part of (S u) for the cell of plane ip, `hi` their part for
// the cell of plane ip + 1 (added to that cell's row when the march reaches
// it).  With X' = (u10 - u00) + (u11 - u01) and Y' = (u01 - u00)/dl_b(e00) +
// (u11 - u10)/dl_b(e10), an edge adds K/(4 dl_a) [s_a Y' + s_b X'/dl_b(face)]
// to each of its cells (the edge term of the energy form, with dl_a the same
// for both a-faces of an (r, .) or (theta, phi) edge).  Ul(dj, dk) reads plane
// ip, Uh(dj, dk) plane ip + 1; K01q[q], K02q[q] are the edge coefficients,
// already zero for absent edges; qia = 1/(4 dl_r(ip)).
template <class R, class UL, class UH>
__device__ __forceinline__ void r_terms(const UL &Ul, const UH &Uh, R w, const R K01q[2],
                                        const R K02q[2], R qia, R s10lo, R s10hi, R s20lo,
                                        R s20hi, const ThreadGeo<R> &tg, R &lo, R &hi) {
  const R f = w * (Uh(0, 0) - Ul(0, 0));
  lo = f;
  hi = -f;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    // (r, theta) edge, origin row j - q
    {
      const R a00 = Ul(-q, 0), a01 = Ul(1 - q, 0), a10 = Uh(-q, 0), a11 = Uh(1 - q, 0);
      const R tj = q ? tg.t11m : tg.t11;
      const R ib0 = s10lo * tj, ib1 = s10hi * tj;
      const R X = (a10 - a00) + (a11 - a01);
      const R Y = (a01 - a00) * ib0 + (a11 - a10) * ib1;
      const R t = K01q[q] * qia;
      lo += t * (q ? Y - ib0 * X : Y + ib0 * X);
      hi -= t * (q ? Y + ib1 * X : Y - ib1 * X);
    }
    // (r, phi) edge, origin column k - q
    {
      const R a00 = Ul(0, -q), a01 = Ul(0, 1 - q), a10 = Uh(0, -q), a11 = Uh(0, 1 - q);
      const R tk = tg.t21 * (q ? tg.t22m : tg.t22);
      const R ib0 = s20lo * tk, ib1 = s20hi * tk;
      const R X = (a10 - a00) + (a11 - a01);
      const R Y = (a01 - a00) * ib0 + (a11 - a10) * ib1;
      const R t = K02q[q] * qia;
      lo += t * (q ? Y - ib0 * X : Y + ib0 * X);
      hi -= t * (q ? Y + ib1 * X : Y - ib1 * X);
    }
  }
}

// The in-plane part of the conduction row of cell (i, j, k): its theta and
// phi faces and the four (theta, phi) edges around it.  U(dj, dk) reads plane
// i; W.K12 holds the edge coefficients in the order of RowCoef (absent edges
// masked here); s10 = 1/r_i-factor of dl_theta, s20 that of dl_phi.
template <class R, class UF>
__device__ __forceinline__ R inplane_S(const RowCoef<R> &W, const UF &U, R s10, R s20,
                                       const ThreadGeo<R> &tg) {
  const R u0 = U(0, 0);
  const R zero = R(0);
  R acc = W.w1p * (U(1, 0) - u0) + (tg.B.hm ? W.w1m : zero) * (U(-1, 0) - u0);
  acc += W.w2p * (U(0, 1) - u0) + (tg.C.hm ? W.w2m : zero) * (U(0, -1) - u0);
  const R qs = R(0.25) * s10 * s20;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const R cp = qs * (p ? tg.t11m : tg.t11);  // s20 / (4 dl_theta)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const bool ex = (p ? tg.B.hm : tg.B.hp) && (q ? tg.C.hm : tg.C.hp);
      const R u00 = U(-p, -q), u10 = U(1 - p, -q), u01 = U(-p, 1 - q), u11 = U(1 - p, 1 - q);
      const R tk = q ? tg.t22m : tg.t22;
      const R P0 = (p ? tg.t21m : tg.t21) * tk, P1 = (p ? tg.t21 : tg.t21p) * tk;
      const R X = (u10 - u00) + (u11 - u01);
      const R Y = (u01 - u00) * P0 + (u11 - u10) * P1;
      const R Pp = p ? P1 : P0;
      const R t = (ex ? W.K12[p + 2 * q] : zero) * cp;
      const R v = q ? -(Pp * X) : Pp * X;
      acc += t * (p ? v - Y : v + Y);
    }
  }
  return acc;
}

}  // namespace

}  // namespace sts
