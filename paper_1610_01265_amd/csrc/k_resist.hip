// Resistive diffusion of the vector potential, -eta curl curl A (Eq. mhd:a,
// boxed; eta stands for c^2 eta / 4 pi), on cell edges.
//
// Unknowns are the line integrals E = A . dl along the cell edges, stored as
// one vector [E_r | E_t | E_p]: E_r[n0][m1][m2] on r-edges, E_t[m0][n1][m2]
// on theta-edges, E_p[m0][m1][n2] on phi-edges, with m_a = n_a on a periodic
// axis and n_a + 1 otherwise.  Face fluxes by Stokes' theorem (normals +r,
// +theta, +phi, right-hand rule):
//   Phi_r(i,j,k) = E_t(i,j,k) + E_p(i,j+1,k) - E_t(i,j,k+1) - E_p(i,j,k)
//   Phi_t(i,j,k) = E_r(i,j,k+1) - E_r(i,j,k) - E_p(i+1,j,k) + E_p(i,j,k)
//   Phi_p(i,j,k) = E_t(i+1,j,k) - E_t(i,j,k) - E_r(i,j+1,k) + E_r(i,j,k),
// so the fluxes leaving a cell cancel (div B = 0).  With face weights
// w = l* / S (centre distance across the face over its area) and edge masses
// H = S* / L (dual-face area over edge length), the operator is
//   F(E) = -eta H^-1 C^T diag(w) C E
// on interior edges; edges lying in a non-periodic boundary surface hold
// their values.  Every weight is a product of three 1D tables.
//
// Kernels: one fused sweep for the operators applied every iteration (F, the
// BE matvec with the p . y partial, the initial residual), whose face values
// never leave registers; and, for the set-up operators, a face sweep w C E
// (or the face weights, or the Gershgorin face counts) into memory followed
// by an edge sweep C^T (w Phi) fused with its consumer (the Gershgorin rows,
// the BE right-hand side with the diagonal).
#include "k_common.h"
#include "k_reduce.h"

#include <algorithm>

namespace sts {

namespace {

constexpr int RX = 64, RY = 4, RT = RX * RY;
static_assert(RT == 256, "the in-sweep PCG decision of k_rpa sums with 256 threads");

struct RDims {
  int n0, n1, n2, m0, m1, m2, per0, per1, per2;
  long long ne[3], nf[3];  // edges / faces per component
  const double *tab;       // 18 one-dimensional weight tables
  int off[18];
  int gx, gy, gz;          // tiles along phi, theta; runs of r-planes
  int cgy, cgz;            // the fused sweep's theta tiles and runs
  int rev;                 // debug: reversed workgroup order
};

// The workgroup's tile: (phi tile, theta tile, run of r-planes), phi tiles
// fastest, and its partial-sum slot L.  (An XCD-aware order, giving each XCD
// a contiguous range of tiles, measured no faster here: the cache lines a
// tile shares with its neighbours are few once the plane carries below are
// in registers.)  The reversed-order self-check reverses the order; the work
// and the partial slot go with L.
struct RTile {
  int L, k, j, i0, i1;
};
__device__ __forceinline__ RTile rtile(const RDims &d) {
  RTile t;
  t.L = wg_index(d.rev);
  const int bx = t.L % d.gx, by = (t.L / d.gx) % d.gy, bz = t.L / (d.gx * d.gy);
  t.k = bx * RX + threadIdx.x;
  t.j = by * RY + threadIdx.y;
  const int per = (d.m0 + d.gz - 1) / d.gz;
  t.i0 = min(d.m0, bz * per);
  t.i1 = min(d.m0, t.i0 + per);
  return t;
}

enum { R_H = 0, T_H = 3, P_H = 6, R_W = 9, T_W = 12, P_W = 15 };  // + axis

__device__ __forceinline__ double tb(const RDims &d, int t, int idx) {
  return d.tab[d.off[t] + idx];
}

// fixed-edge predicates (an edge in a non-periodic boundary surface)
__device__ __forceinline__ bool fixed_r(const RDims &d, int j, int k) {
  return (!d.per1 && (j == 0 || j == d.n1)) || (!d.per2 && (k == 0 || k == d.n2));
}
__device__ __forceinline__ bool fixed_t(const RDims &d, int i, int k) {
  return (!d.per0 && (i == 0 || i == d.n0)) || (!d.per2 && (k == 0 || k == d.n2));
}
__device__ __forceinline__ bool fixed_p(const RDims &d, int i, int j) {
  return (!d.per0 && (i == 0 || i == d.n0)) || (!d.per1 && (j == 0 || j == d.n1));
}

__device__ __forceinline__ int nxt(int x, int n, int per) { return per && x + 1 == n ? 0 : x + 1; }
__device__ __forceinline__ int prv(int x, int n, int per) { return per && x == 0 ? n - 1 : x - 1; }

__device__ __forceinline__ long long ir(const RDims &d, int i, int j, int k) {
  return ((long long)i * d.m1 + j) * d.m2 + k;
}
__device__ __forceinline__ long long it(const RDims &d, int i, int j, int k) {
  return d.ne[0] + ((long long)i * d.n1 + j) * d.m2 + k;
}
__device__ __forceinline__ long long ip(const RDims &d, int i, int j, int k) {
  return d.ne[0] + d.ne[1] + ((long long)i * d.m1 + j) * d.n2 + k;
}

// MASK: 0 all edges, 1 interior edges only, 2 fixed edges only
template <int MASK>
__device__ __forceinline__ double ev(const double *E, long long idx, bool fixed) {
  if (MASK == 1 && fixed) return 0.0;
  if (MASK == 2 && !fixed) return 0.0;
  return E[idx];
}

// Per face (component order r, t, p): KIND 0: Phi~ = w C E; KIND 1: w times
// the number of the face's interior edges (Gershgorin rows); KIND 2: w.
enum { RK_FLUX = 0, RK_COUNT = 1, RK_WEIGHT = 2 };

template <int KIND>
__device__ __forceinline__ double face_val(bool f1, bool f2, bool f3, bool f4, double flux) {
  if (KIND == RK_WEIGHT) return 1.0;
  if (KIND == RK_COUNT) return (!f1) + (!f2) + (!f3) + (!f4);
  return flux;
}

template <int MASK, int KIND>
__global__ void __launch_bounds__(RT) k_rcurl(RDims d, const double *__restrict__ E,
                                              double *__restrict__ Phi) {
  // threads: phi index across lanes, theta across threads; each workgroup
  // takes a contiguous run of r-planes and forms the three kinds of face of a
  // plane in one step.  E_t and E_p of plane i + 1 at (j, k), read for the
  // theta and phi faces, are plane i's own values one step later: they are
  // kept in registers, not read again.
  const RTile tl = rtile(d);
  const int k = tl.k, j = tl.j, i0 = tl.i0, i1 = tl.i1;
  constexpr bool rd = KIND == RK_FLUX;
  const bool ep_in = j < d.m1 && k < d.n2, et_in = j < d.n1 && k < d.m2;
  const int kp = nxt(k, d.n2, d.per2), jp = nxt(j, d.n1, d.per1);
  double *Pr = Phi, *Pt = Phi + d.nf[0], *Pp = Phi + d.nf[0] + d.nf[1];
  double ep = 0.0, et = 0.0;  // E_p(i, j, k), E_t(i, j, k) (masked)
  if (rd && i0 < i1) {
    if (ep_in) ep = ev<MASK>(E, ip(d, i0, j, k), fixed_p(d, i0, j));
    if (et_in) et = ev<MASK>(E, it(d, i0, j, k), fixed_t(d, i0, k));
  }
  for (int i = i0; i < i1; ++i) {
    const int iq = nxt(i, d.n0, d.per0);
    double epn = 0.0, etn = 0.0, er = 0.0;  // E_p(i+1), E_t(i+1), E_r(i) at (j, k)
    if (rd && i < d.n0) {
      if (ep_in) epn = ev<MASK>(E, ip(d, iq, j, k), fixed_p(d, iq, j));
      if (et_in) etn = ev<MASK>(E, it(d, iq, j, k), fixed_t(d, iq, k));
      if (j < d.m1 && k < d.m2) er = ev<MASK>(E, ir(d, i, j, k), fixed_r(d, j, k));
    }
    if (j < d.n1 && k < d.n2) {  // r-face (i < m0, j < n1, k < n2)
      const bool f1 = fixed_t(d, i, k), f2 = fixed_p(d, i, jp), f3 = fixed_t(d, i, kp),
                 f4 = fixed_p(d, i, j);
      double flux = 0.0;
      if (rd)
        flux = et + ev<MASK>(E, ip(d, i, jp, k), f2) - ev<MASK>(E, it(d, i, j, kp), f3) - ep;
      const double w = tb(d, R_W, i) * tb(d, R_W + 1, j) * tb(d, R_W + 2, k);
      Pr[((long long)i * d.n1 + j) * d.n2 + k] = w * face_val<KIND>(f1, f2, f3, f4, flux);
    }
    if (i < d.n0) {
      if (j < d.m1 && k < d.n2) {  // t-face (i < n0, j < m1, k < n2)
        const bool f1 = fixed_r(d, j, kp), f2 = fixed_r(d, j, k), f3 = fixed_p(d, iq, j),
                   f4 = fixed_p(d, i, j);
        double flux = 0.0;
        if (rd) flux = ev<MASK>(E, ir(d, i, j, kp), f1) - er - epn + ep;
        const double w = tb(d, T_W, i) * tb(d, T_W + 1, j) * tb(d, T_W + 2, k);
        Pt[((long long)i * d.m1 + j) * d.n2 + k] = w * face_val<KIND>(f1, f2, f3, f4, flux);
      }
      if (j < d.n1 && k < d.m2) {  // p-face (i < n0, j < n1, k < m2)
        const int jq = jp;
        const bool f1 = fixed_t(d, iq, k), f2 = fixed_t(d, i, k), f3 = fixed_r(d, jq, k),
                   f4 = fixed_r(d, j, k);
        double flux = 0.0;
        if (rd) flux = etn - et - ev<MASK>(E, ir(d, i, jq, k), f3) + er;
        const double w = tb(d, P_W, i) * tb(d, P_W + 1, j) * tb(d, P_W + 2, k);
        Pp[((long long)i * d.n1 + j) * d.m2 + k] = w * face_val<KIND>(f1, f2, f3, f4, flux);
      }
    }
    ep = epn;
    et = etn;
  }
}

// Consumers of s = (C^T Phi~)_e, per edge (GERSH: the unsigned sum of the
// face values, rows of the Gershgorin bound; RHS also sums the face weights).
enum { RC_F = 0, RC_AY = 1, RC_RHS = 2, RC_RES = 3, RC_GERSH = 4 };

struct RArgs {
  const double *in;  // F: unused; AY: p; RHS: E^n; RES: x
  const double *b;   // RES: rhs
  double *out;       // F: F(E); AY: y; RHS: b; RES: r; GERSH: unused
  double *out2;      // RHS: 1 / diag; RES: unused
  double *xfix;      // RHS: x, whose fixed edges take E^n
  double *part;      // per-workgroup partials (p . y, b . b, r . r) or row maxima
  double eta, dt;
};

// per edge e: s = (C^T Phi~)_e, wsum the diagonal's face sum, pv = in[e]
template <int MODE>
__device__ __forceinline__ void consume(const RArgs &a, long long e, bool fixed, double h,
                                        double s, double wsum, double pv, double &acc1) {
  if (MODE == RC_F) {
    a.out[e] = fixed ? 0.0 : -a.eta * s / h;
  } else if (MODE == RC_AY) {
    const double yv = fixed ? 0.0 : h * pv + a.dt * a.eta * s;
    a.out[e] = yv;
    acc1 += pv * yv;
  } else if (MODE == RC_RHS) {
    const double en = pv;
    const double bv = fixed ? 0.0 : h * en - a.dt * a.eta * s;
    a.out[e] = bv;
    a.out2[e] = fixed ? 0.0 : 1.0 / (h + a.dt * a.eta * wsum);
    if (fixed) a.xfix[e] = en;
    acc1 += bv * bv;
  } else if (MODE == RC_RES) {
    const double rv = fixed ? 0.0 : a.b[e] - (h * pv + a.dt * a.eta * s);
    a.out[e] = rv;
    acc1 += rv * rv;
  } else {  // Gershgorin row of eta H^-1 K
    if (!fixed) acc1 = fmax(acc1, a.eta * wsum / h);
  }
}

template <int MODE>
__global__ void __launch_bounds__(RT) k_rcurlT(RDims d, const double *__restrict__ Phi,
                                               const double *__restrict__ Wf, RArgs a) {
  // the face values (F) and the values summed for the diagonal (X: face
  // counts for GERSH, weights for RHS), each in the three face arrays
  constexpr bool flux = MODE != RC_GERSH, diag = MODE == RC_GERSH || MODE == RC_RHS;
  const double *X = MODE == RC_GERSH ? Phi : Wf;
  const double *Fr = Phi, *Ft = Phi + d.nf[0], *Fp = Phi + d.nf[0] + d.nf[1];
  const double *Xr = X, *Xt = X + d.nf[0], *Xp = X + d.nf[0] + d.nf[1];
  double acc1 = 0.0, acc2 = 0.0;
  // as the face kernel: a contiguous run of r-planes, the three kinds of edge
  // of a plane in one step.  The faces at (j, k) of plane i are read once for
  // the three edges; the theta and phi faces of plane i - 1 are the previous
  // step's (read at the run's start).
  const RTile tl = rtile(d);
  const int k = tl.k, j = tl.j, i0 = tl.i0, i1 = tl.i1;
  const int km = prv(k, d.n2, d.per2), jm = prv(j, d.n1, d.per1);
  const bool r_in = j < d.n1 && k < d.n2, t_in = j < d.m1 && k < d.n2,
             p_in = j < d.n1 && k < d.m2;
  double ftm = 0.0, fpm = 0.0, xtm = 0.0, xpm = 0.0;  // plane i - 1
  if (i0 < i1) {
    const int im = prv(i0, d.n0, d.per0);
    if (im >= 0) {
      const long long qt = ((long long)im * d.m1 + j) * d.n2 + k,
                      qp = ((long long)im * d.n1 + j) * d.m2 + k;
      if (t_in) {
        if (flux) ftm = Ft[qt];
        if (diag) xtm = Xt[qt];
      }
      if (p_in) {
        if (flux) fpm = Fp[qp];
        if (diag) xpm = Xp[qp];
      }
    }
  }
  for (int i = i0; i < i1; ++i) {
    // faces (i, j, k) of each kind
    const long long qr = ((long long)i * d.n1 + j) * d.n2 + k,
                    qt = ((long long)i * d.m1 + j) * d.n2 + k,
                    qp = ((long long)i * d.n1 + j) * d.m2 + k;
    double fr = 0.0, ft = 0.0, fp = 0.0, xr = 0.0, xt = 0.0, xp = 0.0;
    if (r_in) {
      if (flux) fr = Fr[qr];
      if (diag) xr = Xr[qr];
    }
    if (i < d.n0 && t_in) {
      if (flux) ft = Ft[qt];
      if (diag) xt = Xt[qt];
    }
    if (i < d.n0 && p_in) {
      if (flux) fp = Fp[qp];
      if (diag) xp = Xp[qp];
    }
    // faces of each edge: (flux index, sign) x 4; an interior edge's faces
    // are all in range
    if (i < d.n0 && j < d.m1 && k < d.m2) {  // r-edge (i < n0, j < m1, k < m2)
      const long long e = ((long long)i * d.m1 + j) * d.m2 + k;
      const bool fixed = fixed_r(d, j, k);
      const double h = tb(d, R_H, i) * tb(d, R_H + 1, j) * tb(d, R_H + 2, k);
      double s = 0.0, wsum = 0.0;
      if (!fixed) {
        const long long t0 = ((long long)i * d.m1 + j) * d.n2;   // Ft(i, j, .)
        const long long p1 = ((long long)i * d.n1 + jm) * d.m2;  // Fp(i, j-1, .)
        if (diag) wsum = xt + Xt[t0 + km] + xp + Xp[p1 + k];
        if (flux) s = -ft + Ft[t0 + km] + fp - Fp[p1 + k];
      }
      consume<MODE>(a, e, fixed, h, s, wsum, MODE == RC_F || MODE == RC_GERSH ? 0.0 : a.in[e],
                    acc1);
    }
    if (j < d.n1 && k < d.m2) {  // t-edge (i < m0, j < n1, k < m2)
      const long long e = d.ne[0] + ((long long)i * d.n1 + j) * d.m2 + k;
      const bool fixed = fixed_t(d, i, k);
      const double h = tb(d, T_H, i) * tb(d, T_H + 1, j) * tb(d, T_H + 2, k);
      double s = 0.0, wsum = 0.0;
      if (!fixed) {
        const long long r0 = ((long long)i * d.n1 + j) * d.n2;  // Fr(i, j, .)
        if (diag) wsum = xr + Xr[r0 + km] + xp + xpm;
        if (flux) s = fr - Fr[r0 + km] - fp + fpm;
      }
      consume<MODE>(a, e, fixed, h, s, wsum, MODE == RC_F || MODE == RC_GERSH ? 0.0 : a.in[e],
                    acc1);
    }
    if (j < d.m1 && k < d.n2) {  // p-edge (i < m0, j < m1, k < n2)
      const long long e = d.ne[0] + d.ne[1] + ((long long)i * d.m1 + j) * d.n2 + k;
      const bool fixed = fixed_p(d, i, j);
      const double h = tb(d, P_H, i) * tb(d, P_H + 1, j) * tb(d, P_H + 2, k);
      double s = 0.0, wsum = 0.0;
      if (!fixed) {
        const long long r1 = ((long long)i * d.n1 + jm) * d.n2;  // Fr(i, j-1, .)
        if (diag) wsum = xr + Xr[r1 + k] + xt + xtm;
        if (flux) s = -fr + Fr[r1 + k] + ft - ftm;
      }
      consume<MODE>(a, e, fixed, h, s, wsum, MODE == RC_F || MODE == RC_GERSH ? 0.0 : a.in[e],
                    acc1);
    }
    ftm = ft;
    fpm = fp;
    xtm = xt;
    xpm = xp;
  }
  const int tid = threadIdx.y * RX + threadIdx.x;
  const int wg = tl.L;
  if (MODE == RC_GERSH) {
    __shared__ double red[RT];
    red[tid] = acc1;
    __syncthreads();
    for (int hh = RT / 2; hh > 0; hh >>= 1) {
      if (tid < hh) red[tid] = fmax(red[tid], red[tid + hh]);
      __syncthreads();
    }
    if (tid == 0) a.part[wg] = red[0];
  } else if (MODE != RC_F) {
    wg_sum2<RT>(acc1, acc2, tid, a.part + wg, nullptr);
  }
}

// ---------------------------------------------------------------------------
// Fused sweep for the operators applied every iteration (F, the BE matvec
// with its p . y partial, the initial residual): the face values are formed
// and summed onto the edges without leaving registers, so the sweep reads E
// once and writes one value per edge.
//
// A wavefront owns a strip of CR theta rows x 64 phi lanes and marches over a
// run of r-planes; within a plane it walks its rows in order.  Each edge needs
// the faces at its own (i, j, k) and at one neighbour below in phi (k - 1), in
// theta (j - 1) or in r (i - 1):
//   k - 1: the lane below, by a whole-wavefront DPP shift; lane 0's value
//          (column k0 - 1, the tile to the left) is formed for all CR rows at
//          once by lanes 0..CR-1 and read out per row;
//   j - 1: the previous row's faces; row 0's come from a halo row formed
//          first (row ja - 1);
//   i - 1: kept per row from the previous plane (formed at the run's start).
// E_p and E_t of plane i + 1 at (j, k) are plane i + 1's own values one plane
// later, and E_r(i, j + 1) is the next row's: a strip reads each of its own
// values once (the halo row and column come on top: 1.6x the algorithmic
// bytes in all at 256 x 256 x 512).  Face values and edge sums are the same
// expressions, in the same order, as the two-sweep form's.
template <int CR>
struct RccGeom {
  static constexpr int ROWS = CR * (RT / RX);  // theta rows of a workgroup tile
};

// v unchanged, hidden from the optimiser (a wavefront-uniform value, kept in an
// SGPR): the table loads indexed by it stay in the plane loop instead of
// being hoisted out of it for every row at once (which overflows the SGPRs)
__device__ __forceinline__ int opaque_s(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int MODE, int CR>
__global__ void __launch_bounds__(RT) k_rcc(RDims d, const double *__restrict__ E, RArgs a) {
  constexpr bool MASKED = MODE == RC_RES;  // RES: x's interior edges only
  const int lane = threadIdx.x;
  const int L = wg_index(d.rev);
  const int bx = L % d.gx, by = (L / d.gx) % d.cgy, bz = L / (d.gx * d.cgy);
  const int k0 = bx * RX, k = k0 + lane;
  const int ja = __builtin_amdgcn_readfirstlane(by * RccGeom<CR>::ROWS + (int)threadIdx.y * CR);
  const int nrow = max(0, min(CR, d.m1 - ja));
  const int per = (d.m0 + d.cgz - 1) / d.cgz;
  const int i0 = min(d.m0, bz * per), i1 = min(d.m0, i0 + per);
  const int n1 = d.n1, m1 = d.m1, n2 = d.n2, m2 = d.m2, n0 = d.n0;
  const int kp = nxt(k, n2, d.per2);
  // the column left of the tile and the row below the strip, where they
  // exist (else every edge that would use them is fixed)
  const bool colh = k0 > 0 || d.per2, rowh = nrow > 0 && (ja > 0 || d.per1);
  const int kh = prv(k0, n2, d.per2), jh = prv(ja, n1, d.per1);
  const bool kn = k < n2, km_ = k < m2;
  // phi factors of the weights, constant per lane
  const double wr2 = kn ? tb(d, R_W + 2, k) : 0.0, wt2 = kn ? tb(d, T_W + 2, k) : 0.0,
               wp2 = km_ ? tb(d, P_W + 2, k) : 0.0, hr2 = km_ ? tb(d, R_H + 2, k) : 0.0,
               ht2 = km_ ? tb(d, T_H + 2, k) : 0.0, hp2 = kn ? tb(d, P_H + 2, k) : 0.0;
  // plane starts of the three components (a plane's own offsets fit an int)
  const long long sr = (long long)m1 * m2, st = (long long)n1 * m2, sp = (long long)m1 * n2;
  const double *Er = E, *Et = E + d.ne[0], *Ep = E + d.ne[0] + d.ne[1];
  // masked, bounds-checked loads: component at plane pointer P, offset o
  auto ldr = [&](const double *P, int j, int kk, bool in) {
    return in && !(MASKED && fixed_r(d, j, kk)) ? P[j * m2 + kk] : 0.0;
  };
  auto ldt = [&](const double *P, int i, int j, int kk, bool in) {
    return in && !(MASKED && fixed_t(d, i, kk)) ? P[j * m2 + kk] : 0.0;
  };
  auto ldp = [&](const double *P, int i, int j, int kk, bool in) {
    return in && !(MASKED && fixed_p(d, i, j)) ? P[j * n2 + kk] : 0.0;
  };
  double acc1 = 0.0, acc2 = 0.0;

  double ep[CR], et[CR], ftm[CR], fpm[CR];  // E_p, E_t of plane i; F_t, F_p of plane i - 1
  if (i0 < i1) {
    const int im = prv(i0, n0, d.per0);
    const double *Pti = Et + i0 * st, *Ppi = Ep + i0 * sp;
#pragma unroll
    for (int r = 0; r < CR; ++r) {
      const int j = ja + r;
      ep[r] = et[r] = ftm[r] = fpm[r] = 0.0;
      if (r >= nrow) continue;
      ep[r] = ldp(Ppi, i0, j, k, j < m1 && kn);
      et[r] = ldt(Pti, i0, j, k, j < n1 && km_);
      if (im >= 0) {  // faces of plane i0 - 1 (nxt(im) = i0)
        const int jq = nxt(j, n1, d.per1);
        const double *Prm = Er + im * sr, *Ptm = Et + im * st, *Ppm = Ep + im * sp;
        const double erm = ldr(Prm, j, k, j < m1 && km_);
        if (j < m1 && kn)
          ftm[r] = uniform_ld(d.tab, d.off[T_W] + im) * uniform_ld(d.tab, d.off[T_W + 1] + j) *
                   wt2 * (ldr(Prm, j, kp, true) - erm - ep[r] + ldp(Ppm, im, j, k, true));
        if (j < n1 && km_)
          fpm[r] = uniform_ld(d.tab, d.off[P_W] + im) * uniform_ld(d.tab, d.off[P_W + 1] + j) *
                   wp2 * (et[r] - ldt(Ptm, im, j, k, true) - ldr(Prm, jq, k, true) + erm);
      }
    }
  }
  for (int i = i0; i < i1; ++i) {
    const int iq = nxt(i, n0, d.per0);
    const bool ilt = i < n0;
    // r factors of the weights (wavefront-uniform)
    const double wr0 = uniform_ld(d.tab, d.off[R_W] + i),
                 wt0 = ilt ? uniform_ld(d.tab, d.off[T_W] + i) : 0.0,
                 wp0 = ilt ? uniform_ld(d.tab, d.off[P_W] + i) : 0.0,
                 hr0 = ilt ? uniform_ld(d.tab, d.off[R_H] + i) : 0.0,
                 ht0 = uniform_ld(d.tab, d.off[T_H] + i), hp0 = uniform_ld(d.tab, d.off[P_H] + i);
    const double *Pr = Er + i * sr, *Pt = Et + i * st, *Pp = Ep + i * sp;
    const double *Ptq = Et + iq * st, *Ppq = Ep + iq * sp;
    const long long orr = i * sr, ort = d.ne[0] + i * st, orp = d.ne[0] + d.ne[1] + i * sp;
    double er = ldr(Pr, ja, k, ilt && ja < m1 && km_);  // E_r(i, j, k) of the current row
    // halo row jh = ja - 1: F_r and F_p there (the j - 1 faces of row 0)
    double frj = 0.0, fpj = 0.0;
    if (rowh) {
      const double eth = ldt(Pt, i, jh, k, jh < n1 && km_);
      if (jh < n1 && kn)
        frj = wr0 * uniform_ld(d.tab, d.off[R_W + 1] + jh) * wr2 *
              (eth + ep[0] - ldt(Pt, i, jh, kp, true) - ldp(Pp, i, jh, k, true));
      if (ilt && jh < n1 && km_)
        fpj = wp0 * uniform_ld(d.tab, d.off[P_W + 1] + jh) * wp2 *
              (ldt(Ptq, iq, jh, k, true) - eth - er + ldr(Pr, jh, k, true));
    }
    // column halo kh = k0 - 1: lane l < nrow forms F_r and F_t of row ja + l
    double frc = 0.0, ftc = 0.0;
    if (colh && lane < nrow) {
      const int j = ja + lane, jq = nxt(j, n1, d.per1);
      const double epc = ldp(Pp, i, j, kh, true);
      if (j < n1)
        frc = wr0 * tb(d, R_W + 1, j) * tb(d, R_W + 2, kh) *
              (ldt(Pt, i, j, kh, true) + ldp(Pp, i, jq, kh, true) - ldt(Pt, i, j, k0, true) - epc);
      if (ilt && j < m1)
        ftc = wt0 * tb(d, T_W + 1, j) * tb(d, T_W + 2, kh) *
              (ldr(Pr, j, k0, true) - ldr(Pr, j, kh, true) - ldp(Ppq, iq, j, kh, true) + epc);
    }
#pragma unroll
    for (int r = 0; r < CR; ++r) {
      if (r >= nrow) break;
      const int j = opaque_s(ja + r), jq = nxt(j, n1, d.per1);
      // this row's loads: the next row's E_r, plane i + 1's E_p and E_t
      const double ern = ldr(Pr, jq, k, ilt && jq < m1 && km_);
      const double epn = ldp(Ppq, iq, j, k, ilt && j < m1 && kn);
      const double etn = ldt(Ptq, iq, j, k, ilt && j < n1 && km_);
      const double epq =
          r + 1 < nrow ? ep[r + 1 < CR ? r + 1 : r] : ldp(Pp, i, jq, k, jq < m1 && kn);
      const double fr = (j < n1 && kn)
                            ? wr0 * uniform_ld(d.tab, d.off[R_W + 1] + j) * wr2 *
                                  (et[r] + epq - ldt(Pt, i, j, kp, true) - ep[r])
                            : 0.0;
      const double ft = (ilt && j < m1 && kn)
                            ? wt0 * uniform_ld(d.tab, d.off[T_W + 1] + j) * wt2 *
                                  (ldr(Pr, j, kp, true) - er - epn + ep[r])
                            : 0.0;
      const double fp = (ilt && j < n1 && km_)
                            ? wp0 * uniform_ld(d.tab, d.off[P_W + 1] + j) * wp2 *
                                  (etn - et[r] - ern + er)
                            : 0.0;
      const double frk = wave_shr1(fr, readlane_d(frc, r)),  // F_r(i, j, k - 1)
          ftk = wave_shr1(ft, readlane_d(ftc, r));           // F_t(i, j, k - 1)
      if (ilt && j < m1 && km_) {  // r-edge
        const bool fixed = fixed_r(d, j, k);
        const double s = fixed ? 0.0 : -ft + ftk + fp - fpj;
        consume<MODE>(a, orr + (j * m2 + k), fixed,
                      hr0 * uniform_ld(d.tab, d.off[R_H + 1] + j) * hr2, s, 0.0, er, acc1);
      }
      if (j < n1 && km_) {  // t-edge
        const bool fixed = fixed_t(d, i, k);
        const double s = fixed ? 0.0 : fr - frk - fp + fpm[r];
        consume<MODE>(a, ort + (j * m2 + k), fixed,
                      ht0 * uniform_ld(d.tab, d.off[T_H + 1] + j) * ht2, s, 0.0, et[r], acc1);
      }
      if (j < m1 && kn) {  // p-edge
        const bool fixed = fixed_p(d, i, j);
        const double s = fixed ? 0.0 : -fr + frj + ft - ftm[r];
        consume<MODE>(a, orp + (j * n2 + k), fixed,
                      hp0 * uniform_ld(d.tab, d.off[P_H + 1] + j) * hp2, s, 0.0, ep[r], acc1);
      }
      frj = fr;
      fpj = fp;
      er = ern;
      ftm[r] = ft;
      fpm[r] = fp;
      ep[r] = epn;
      et[r] = etn;
    }
  }
  const int tid = threadIdx.y * RX + threadIdx.x;
  if (MODE != RC_F) wg_sum2<RT>(acc1, acc2, tid, a.part + L, nullptr);
}

// p = z + beta p_old with z = r / diag (beta = 0 on the first iteration).
// pb != null: beta and the previous iteration's stopping test are formed here
// from pass B's partials pb (npb per region, regions cap apart), identically
// in every workgroup (pcg_decide), instead of in a finalize kernel.
__global__ void __launch_bounds__(RT)
    k_rpa(long long n, const double *__restrict__ r, const double *__restrict__ invd,
          const double *__restrict__ pold, double *__restrict__ p, PcgScalars *sc, int first,
          const double *pb, int npb, long long cap, int iters) {
  if (sc->done) return;
  double beta = 0.0;
  if (!first) {
    if (pb) {
      if (pcg_decide(pb, npb, cap, iters, sc, blockIdx.x == 0, (int)threadIdx.x, &beta)) return;
    } else {
      beta = sc->beta;
    }
  }
  for (long long e = (long long)blockIdx.x * RT + threadIdx.x; e < n;
       e += (long long)gridDim.x * RT)
    p[e] = r[e] * invd[e] + (first ? 0.0 : beta * pold[e]);
}

// Tiles: phi x theta (each axis sized for the longest of the three arrays
// along it) x runs of r-planes, one workgroup each.  About 4096 workgroups: enough
// to keep every CU busy through the tail; more would make the PCG sweeps,
// each of whose workgroups sums all of the edge sweep's partials, cost more
// at the smaller grids than the finer split gains.
constexpr int kResWgs = 4096;

dim3 grid3r(const sts_ctx *c) {
  const int m0 = c->n0 + (c->bc[0] == STS_BC_PERIODIC ? 0 : 1),
            m1 = c->n1 + (c->bc[2] == STS_BC_PERIODIC ? 0 : 1),
            m2 = c->n2 + (c->bc[4] == STS_BC_PERIODIC ? 0 : 1);
  const int gx = (m2 + RX - 1) / RX, gy = (m1 + RY - 1) / RY;
  const int gz = std::max(1, std::min(m0, kResWgs / std::max(1, gx * gy)));
  return dim3(gx, gy, gz);
}

// The fused sweep's tiles: strips of kRccRows theta rows, RT / RX strips per
// workgroup, the phi tiles of the two-sweep form, and runs of r-planes: about
// kRccWgs workgroups, but runs of at least kRccRun planes (a run's first
// plane also forms the faces of the plane before it) unless that leaves
// fewer than 1024 workgroups.  Measured at
// 256x256x512 and 128x128x256: 4-row strips beat 2 and 8 (8 rows need 177
// VGPRs); runs of 4 planes beat 8 and 16 at the smaller grid and tie at the
// larger.
constexpr int kRccRows = 4, kRccWgs = 2048, kRccRun = 4;

void rcc_tiles(const sts_ctx *c, int gx, int &cgy, int &cgz) {
  const int m0 = c->n0 + (c->bc[0] == STS_BC_PERIODIC ? 0 : 1),
            m1 = c->n1 + (c->bc[2] == STS_BC_PERIODIC ? 0 : 1);
  const int rows = RccGeom<kRccRows>::ROWS;
  cgy = (m1 + rows - 1) / rows;
  cgz = std::max(1, std::min(kRccWgs / std::max(1, gx * cgy), std::max(1, m0 / kRccRun)));
  // a small grid: runs down to one plane, for parallelism (32x32x64: 47 -> 25
  // us per BE iteration)
  if (gx * cgy * cgz < 1024)
    cgz = std::max(1, std::min(kRccWgs / std::max(1, gx * cgy), m0));
}

template <int MODE>
void rcc_launch(const sts_ctx *c, const RDims &d, const double *E, const RArgs &a) {
  hipLaunchKernelGGL((k_rcc<MODE, kRccRows>), dim3(d.gx * d.cgy * d.cgz), dim3(RX, RY), 0,
                     c->stream, d, E, a);
}

template <int MASK, int KIND>
void curl_launch(const sts_ctx *c, const RDims &d, const double *E, double *Phi) {
  hipLaunchKernelGGL((k_rcurl<MASK, KIND>), dim3(d.gx * d.gy * d.gz), dim3(RX, RY), 0,
                     c->stream, d, E, Phi);
}

}  // namespace

// workgroups of the two-sweep form (the edge sweep's partial sums), also the
// 1D grids' size
int res_parts(const sts_ctx *c) {
  const dim3 g = grid3r(c);
  return (int)(g.x * g.y * g.z);
}

// workgroups (partial sums) of the fused sweep
int res_parts_fused(const sts_ctx *c) {
  const dim3 g = grid3r(c);
  int cgy, cgz;
  rcc_tiles(c, g.x, cgy, cgz);
  return (int)g.x * cgy * cgz;
}

static RDims rdims(const sts_ctx *c) {
  RDims d{};
  d.n0 = c->n0;
  d.n1 = c->n1;
  d.n2 = c->n2;
  d.per0 = c->bc[0] == STS_BC_PERIODIC;
  d.per1 = c->bc[2] == STS_BC_PERIODIC;
  d.per2 = c->bc[4] == STS_BC_PERIODIC;
  d.m0 = d.n0 + !d.per0;
  d.m1 = d.n1 + !d.per1;
  d.m2 = d.n2 + !d.per2;
  for (int q = 0; q < 3; ++q) {
    d.ne[q] = c->res_ne[q];
    d.nf[q] = c->res_nf[q];
  }
  d.tab = c->d_rtab;
  for (int t = 0; t < 18; ++t) d.off[t] = c->res_off[t];
  const dim3 g = grid3r(c);
  d.gx = g.x;
  d.gy = g.y;
  d.gz = g.z;
  rcc_tiles(c, d.gx, d.cgy, d.cgz);
  d.rev = (c->debug & STS_DEBUG_WG_REVERSE) ? 1 : 0;
  return d;
}

template <int MODE>
static void curlT_launch(const sts_ctx *c, const RDims &d, const double *Phi, const double *Wf,
                         const RArgs &a) {
  hipLaunchKernelGGL(k_rcurlT<MODE>, dim3(d.gx * d.gy * d.gz), dim3(RX, RY), 0, c->stream, d,
                     Phi, Wf, a);
}

void launch_res_F(const sts_ctx *c, const double *E, double *FE) {
  STS_PROF(c, "launch_res_F");
  RArgs a{};
  a.out = FE;
  a.eta = c->res_eta;
  rcc_launch<RC_F>(c, rdims(c), E, a);
}

void launch_res_gershgorin(const sts_ctx *c, double *Phi, double *part) {
  STS_PROF(c, "launch_res_gershgorin");
  const RDims d = rdims(c);
  curl_launch<0, RK_COUNT>(c, d, nullptr, Phi);
  RArgs a{};
  a.part = part;
  a.eta = c->res_eta;
  curlT_launch<RC_GERSH>(c, d, Phi, nullptr, a);
}

// b = H E^n - dt eta K E_b on interior edges (E_b: the fixed edges of E^n),
// 1/diag with diag = H + dt eta (sum of the edge's face weights), x's fixed
// edges := E^n's; partial b . b.  Wf receives the face weights.
void launch_res_rhs(const sts_ctx *c, const double *En, double dt, double *x, double *b,
                    double *invd, double *Phi, double *Wf, double *part) {
  STS_PROF(c, "launch_res_rhs");
  const RDims d = rdims(c);
  curl_launch<0, RK_WEIGHT>(c, d, nullptr, Wf);
  curl_launch<2, RK_FLUX>(c, d, En, Phi);
  RArgs a{};
  a.in = En;
  a.out = b;
  a.out2 = invd;
  a.xfix = x;
  a.part = part;
  a.eta = c->res_eta;
  a.dt = dt;
  curlT_launch<RC_RHS>(c, d, Phi, Wf, a);
}

void launch_res_residual(const sts_ctx *c, const double *b, const double *x, double dt,
                         double *r, double *part) {
  STS_PROF(c, "launch_res_residual");
  RArgs a{};
  a.b = b;
  a.out = r;
  a.part = part;
  a.eta = c->res_eta;
  a.dt = dt;
  rcc_launch<RC_RES>(c, rdims(c), x, a);
}

void launch_res_pass_a(const sts_ctx *c, double dt, const double *r, const double *invd,
                       const double *pold, double *p, double *y, double *part,
                       const PcgScalars *sc, int first, const double *pb, int npb, int iters) {
  STS_PROF(c, "launch_res_pass_a");
  const RDims d = rdims(c);
  const long long n = d.ne[0] + d.ne[1] + d.ne[2];
  hipLaunchKernelGGL(k_rpa, dim3(res_parts(c)), dim3(RT), 0, c->stream, n, r, invd, pold, p,
                     const_cast<PcgScalars *>(sc), first, pb, npb, (long long)c->red_cap, iters);
  RArgs a{};
  a.out = y;
  a.part = part;
  a.eta = c->res_eta;
  a.dt = dt;
  rcc_launch<RC_AY>(c, d, p, a);
}

}  // namespace sts
