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
// Kernels: face fluxes w C E (optionally with only the interior or only the
// fixed edges of E), and an edge sweep C^T (w Phi) fused with its consumer
// (F, the BE matvec with the p . y partial, the BE right-hand side with the
// diagonal, the initial residual).
#include "k_common.h"
#include "k_reduce.h"

#include <algorithm>

namespace sts {

namespace {

constexpr int RX = 64, RY = 4, RT = RX * RY;

struct RDims {
  int n0, n1, n2, m0, m1, m2, per0, per1, per2;
  long long ne[3], nf[3];  // edges / faces per component
  const double *tab;       // 18 one-dimensional weight tables
  int off[18];
  int rev;                 // debug: reversed workgroup order
};

// the workgroup's logical 3D index (reversed along each axis in the
// reversed-order self-check; the work and partial slot go with it)
__device__ __forceinline__ int rblk(int b, int n, int rev) { return rev ? n - 1 - b : b; }

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

// the contiguous run [i0, i1) of r-planes of z-block b out of nb over n planes
__device__ __forceinline__ void plane_run(int n, int b, int nb, int &i0, int &i1) {
  const int per = (n + nb - 1) / nb;
  i0 = min(n, b * per);
  i1 = min(n, i0 + per);
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
  // threads: phi index across lanes, theta across threads / blocks; each
  // workgroup takes a contiguous run of r-planes and forms the three kinds of
  // face of a plane together, so the edge values they share (and the next
  // plane's, read again one step later) come from cache
  const int k = rblk(blockIdx.x, gridDim.x, d.rev) * RX + threadIdx.x,
            j = rblk(blockIdx.y, gridDim.y, d.rev) * RY + threadIdx.y;
  int i0, i1;
  plane_run(d.m0, rblk(blockIdx.z, gridDim.z, d.rev), gridDim.z, i0, i1);
  double *Pr = Phi, *Pt = Phi + d.nf[0], *Pp = Phi + d.nf[0] + d.nf[1];
  for (int i = i0; i < i1; ++i) {
    if (j < d.n1 && k < d.n2) {  // r-face (i < m0, j < n1, k < n2)
      const int kp = nxt(k, d.n2, d.per2), jp = nxt(j, d.n1, d.per1);
      const bool f1 = fixed_t(d, i, k), f2 = fixed_p(d, i, jp), f3 = fixed_t(d, i, kp),
                 f4 = fixed_p(d, i, j);
      double flux = 0.0;
      if (KIND == RK_FLUX)
        flux = ev<MASK>(E, it(d, i, j, k), f1) + ev<MASK>(E, ip(d, i, jp, k), f2) -
               ev<MASK>(E, it(d, i, j, kp), f3) - ev<MASK>(E, ip(d, i, j, k), f4);
      const double w = tb(d, R_W, i) * tb(d, R_W + 1, j) * tb(d, R_W + 2, k);
      Pr[((long long)i * d.n1 + j) * d.n2 + k] = w * face_val<KIND>(f1, f2, f3, f4, flux);
    }
    if (i >= d.n0) continue;
    const int iq = nxt(i, d.n0, d.per0);
    if (j < d.m1 && k < d.n2) {  // t-face (i < n0, j < m1, k < n2)
      const int kp = nxt(k, d.n2, d.per2);
      const bool f1 = fixed_r(d, j, kp), f2 = fixed_r(d, j, k), f3 = fixed_p(d, iq, j),
                 f4 = fixed_p(d, i, j);
      double flux = 0.0;
      if (KIND == RK_FLUX)
        flux = ev<MASK>(E, ir(d, i, j, kp), f1) - ev<MASK>(E, ir(d, i, j, k), f2) -
               ev<MASK>(E, ip(d, iq, j, k), f3) + ev<MASK>(E, ip(d, i, j, k), f4);
      const double w = tb(d, T_W, i) * tb(d, T_W + 1, j) * tb(d, T_W + 2, k);
      Pt[((long long)i * d.m1 + j) * d.n2 + k] = w * face_val<KIND>(f1, f2, f3, f4, flux);
    }
    if (j < d.n1 && k < d.m2) {  // p-face (i < n0, j < n1, k < m2)
      const int jq = nxt(j, d.n1, d.per1);
      const bool f1 = fixed_t(d, iq, k), f2 = fixed_t(d, i, k), f3 = fixed_r(d, jq, k),
                 f4 = fixed_r(d, j, k);
      double flux = 0.0;
      if (KIND == RK_FLUX)
        flux = ev<MASK>(E, it(d, iq, j, k), f1) - ev<MASK>(E, it(d, i, j, k), f2) -
               ev<MASK>(E, ir(d, i, jq, k), f3) + ev<MASK>(E, ir(d, i, j, k), f4);
      const double w = tb(d, P_W, i) * tb(d, P_W + 1, j) * tb(d, P_W + 2, k);
      Pp[((long long)i * d.n1 + j) * d.m2 + k] = w * face_val<KIND>(f1, f2, f3, f4, flux);
    }
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

template <int MODE>
__device__ __forceinline__ void consume(const RArgs &a, long long e, bool fixed, double h,
                                        double s, double wsum, double &acc1) {
  if (MODE == RC_F) {
    a.out[e] = fixed ? 0.0 : -a.eta * s / h;
  } else if (MODE == RC_AY) {
    const double pv = a.in[e];
    const double yv = fixed ? 0.0 : h * pv + a.dt * a.eta * s;
    a.out[e] = yv;
    acc1 += pv * yv;
  } else if (MODE == RC_RHS) {
    const double en = a.in[e];
    const double bv = fixed ? 0.0 : h * en - a.dt * a.eta * s;
    a.out[e] = bv;
    a.out2[e] = fixed ? 0.0 : 1.0 / (h + a.dt * a.eta * wsum);
    if (fixed) a.xfix[e] = en;
    acc1 += bv * bv;
  } else if (MODE == RC_RES) {
    const double rv = fixed ? 0.0 : a.b[e] - (h * a.in[e] + a.dt * a.eta * s);
    a.out[e] = rv;
    acc1 += rv * rv;
  } else {  // Gershgorin row of eta H^-1 K
    if (!fixed) acc1 = fmax(acc1, a.eta * wsum / h);
  }
}

template <int MODE>
__global__ void __launch_bounds__(RT) k_rcurlT(RDims d, const double *__restrict__ Phi,
                                               const double *__restrict__ Wf, RArgs a) {
  const double *Fr = Phi, *Ft = Phi + d.nf[0], *Fp = Phi + d.nf[0] + d.nf[1];
  // the values summed for the diagonal: face counts (GERSH) or weights (RHS)
  const double *X = MODE == RC_GERSH ? Phi : Wf;
  const double *Xr = X, *Xt = X + d.nf[0], *Xp = X + d.nf[0] + d.nf[1];
  constexpr bool diag = MODE == RC_GERSH || MODE == RC_RHS;
  double acc1 = 0.0, acc2 = 0.0;
  // as the face kernel: a contiguous run of r-planes, the three kinds of edge
  // of a plane together (faces of plane i - 1 were read one step earlier)
  const int k = rblk(blockIdx.x, gridDim.x, d.rev) * RX + threadIdx.x,
            j = rblk(blockIdx.y, gridDim.y, d.rev) * RY + threadIdx.y;
  int i0, i1;
  plane_run(d.m0, rblk(blockIdx.z, gridDim.z, d.rev), gridDim.z, i0, i1);
  for (int i = i0; i < i1; ++i) {
    const int im = prv(i, d.n0, d.per0);
    // faces of each edge: (flux index, sign) x 4
    if (i < d.n0 && j < d.m1 && k < d.m2) {  // r-edge (i < n0, j < m1, k < m2)
      const long long e = ((long long)i * d.m1 + j) * d.m2 + k;
      const bool fixed = fixed_r(d, j, k);
      const double h = tb(d, R_H, i) * tb(d, R_H + 1, j) * tb(d, R_H + 2, k);
      double s = 0.0, wsum = 0.0;
      if (!fixed) {
        const int km = prv(k, d.n2, d.per2), jm = prv(j, d.n1, d.per1);
        const long long t0 = ((long long)i * d.m1 + j) * d.n2;   // Ft(i, j, .)
        const long long p0 = ((long long)i * d.n1 + j) * d.m2;   // Fp(i, j, .)
        const long long p1 = ((long long)i * d.n1 + jm) * d.m2;  // Fp(i, j-1, .)
        if (diag) wsum = Xt[t0 + k] + Xt[t0 + km] + Xp[p0 + k] + Xp[p1 + k];
        if (MODE != RC_GERSH) s = -Ft[t0 + k] + Ft[t0 + km] + Fp[p0 + k] - Fp[p1 + k];
      }
      consume<MODE>(a, e, fixed, h, s, wsum, acc1);
    }
    if (j < d.n1 && k < d.m2) {  // t-edge (i < m0, j < n1, k < m2)
      const long long e = d.ne[0] + ((long long)i * d.n1 + j) * d.m2 + k;
      const bool fixed = fixed_t(d, i, k);
      const double h = tb(d, T_H, i) * tb(d, T_H + 1, j) * tb(d, T_H + 2, k);
      double s = 0.0, wsum = 0.0;
      if (!fixed) {
        const int km = prv(k, d.n2, d.per2);
        const long long r0 = ((long long)i * d.n1 + j) * d.n2;   // Fr(i, j, .)
        const long long p0 = ((long long)i * d.n1 + j) * d.m2;   // Fp(i, j, .)
        const long long p1 = ((long long)im * d.n1 + j) * d.m2;  // Fp(i-1, j, .)
        if (diag) wsum = Xr[r0 + k] + Xr[r0 + km] + Xp[p0 + k] + Xp[p1 + k];
        if (MODE != RC_GERSH) s = Fr[r0 + k] - Fr[r0 + km] - Fp[p0 + k] + Fp[p1 + k];
      }
      consume<MODE>(a, e, fixed, h, s, wsum, acc1);
    }
    if (j < d.m1 && k < d.n2) {  // p-edge (i < m0, j < m1, k < n2)
      const long long e = d.ne[0] + d.ne[1] + ((long long)i * d.m1 + j) * d.n2 + k;
      const bool fixed = fixed_p(d, i, j);
      const double h = tb(d, P_H, i) * tb(d, P_H + 1, j) * tb(d, P_H + 2, k);
      double s = 0.0, wsum = 0.0;
      if (!fixed) {
        const int jm = prv(j, d.n1, d.per1);
        const long long r0 = ((long long)i * d.n1 + j) * d.n2;   // Fr(i, j, .)
        const long long r1 = ((long long)i * d.n1 + jm) * d.n2;  // Fr(i, j-1, .)
        const long long t0 = ((long long)i * d.m1 + j) * d.n2;   // Ft(i, j, .)
        const long long t1 = ((long long)im * d.m1 + j) * d.n2;  // Ft(i-1, j, .)
        if (diag) wsum = Xr[r0 + k] + Xr[r1 + k] + Xt[t0 + k] + Xt[t1 + k];
        if (MODE != RC_GERSH) s = -Fr[r0 + k] + Fr[r1 + k] + Ft[t0 + k] - Ft[t1 + k];
      }
      consume<MODE>(a, e, fixed, h, s, wsum, acc1);
    }
  }
  const int tid = threadIdx.y * RX + threadIdx.x;
  const int wg = (rblk(blockIdx.z, gridDim.z, d.rev) * gridDim.y +
                  rblk(blockIdx.y, gridDim.y, d.rev)) * gridDim.x +
                 rblk(blockIdx.x, gridDim.x, d.rev);
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

// 3D launch: x over phi, y over theta (each sized for the longest of the three
// arrays along it), z over runs of r-planes.  About 4096 workgroups: enough
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

template <int MASK, int KIND>
void curl_launch(const sts_ctx *c, const RDims &d, const double *E, double *Phi) {
  hipLaunchKernelGGL((k_rcurl<MASK, KIND>), grid3r(c), dim3(RX, RY), 0, c->stream,
                     d, E, Phi);
}

}  // namespace

// workgroups of the edge sweep (its partial sums), also the 1D grids' size
int res_parts(const sts_ctx *c) {
  const dim3 g = grid3r(c);
  return (int)(g.x * g.y * g.z);
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
  d.rev = (c->debug & STS_DEBUG_WG_REVERSE) ? 1 : 0;
  return d;
}

template <int MODE>
static void curlT_launch(const sts_ctx *c, const RDims &d, const double *Phi, const double *Wf,
                         const RArgs &a) {
  hipLaunchKernelGGL(k_rcurlT<MODE>, grid3r(c), dim3(RX, RY), 0, c->stream, d, Phi,
                     Wf, a);
}

void launch_res_F(const sts_ctx *c, const double *E, double *Phi, double *FE) {
  STS_PROF(c, "launch_res_F");
  const RDims d = rdims(c);
  curl_launch<0, RK_FLUX>(c, d, E, Phi);
  RArgs a{};
  a.out = FE;
  a.eta = c->res_eta;
  curlT_launch<RC_F>(c, d, Phi, nullptr, a);
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
                         double *Phi, double *r, double *part) {
  STS_PROF(c, "launch_res_residual");
  const RDims d = rdims(c);
  curl_launch<1, RK_FLUX>(c, d, x, Phi);
  RArgs a{};
  a.in = x;
  a.b = b;
  a.out = r;
  a.part = part;
  a.eta = c->res_eta;
  a.dt = dt;
  curlT_launch<RC_RES>(c, d, Phi, nullptr, a);
}

void launch_res_pass_a(const sts_ctx *c, double dt, const double *r, const double *invd,
                       const double *pold, double *p, double *Phi, double *y, double *part,
                       const PcgScalars *sc, int first, const double *pb, int npb, int iters) {
  STS_PROF(c, "launch_res_pass_a");
  const RDims d = rdims(c);
  const long long n = d.ne[0] + d.ne[1] + d.ne[2];
  hipLaunchKernelGGL(k_rpa, dim3(res_parts(c)), dim3(RT), 0, c->stream, n, r, invd, pold, p,
                     const_cast<PcgScalars *>(sc), first, pb, npb, (long long)c->red_cap, iters);
  curl_launch<0, RK_FLUX>(c, d, p, Phi);
  RArgs a{};
  a.in = p;
  a.out = y;
  a.part = part;
  a.eta = c->res_eta;
  a.dt = dt;
  curlT_launch<RC_AY>(c, d, Phi, nullptr, a);
}

}  // namespace sts
