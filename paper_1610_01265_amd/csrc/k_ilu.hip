// PC2: non-overlapping block ILU0 (Sec. 2.3, Appendix A).
//
// The grid is cut into blocks of B0 x B1 x B2 cells (each <= 8; the last
// block along an axis may be smaller).  Inside a block the BE matrix
// A = V - dt S is restricted to the block (couplings to other blocks and the
// periodic wrap are dropped) and factored by zero-fill ILU on the 19-point
// pattern, rows in lexicographic order (axis 0 slowest, axis 2 fastest).
// Because A is symmetric, the IKJ factorisation of Appendix A yields
// U = D L^T; only the unit-lower L (9 entries per row, one per lower stencil
// neighbour) and the pivots D are stored:
//   L_ik = (A_ik - sum_{m<k} L_im D_m L_km) / D_k,  D_i = A_ii - sum_k L_ik^2 D_k,
// the sums running over the pattern.  The substitution of Appendix A becomes
//   forward  z*_i = r_i - sum_{k<i} L_ik z*_k
//   backward z_i  = z*_i / D_i - sum_{j>i} L_ji z_j.
// Rows are processed by hyperplanes l = 3 i' + 2 j' + k' of the local
// coordinates: every lower neighbour of a cell lies on an earlier hyperplane
// (43 of them for 8^3 blocks).  One wavefront works on one block; lane t owns
// the column (i', j') = (t / 8, t % 8), which holds at most one cell of any
// hyperplane.
//
// Factor layout: fac[block][slot][B0*B1*B2] with slots 0..8 = L, 9 = D, the
// cell index inside a block being (i' B1 + j') B2 + k'.
#include "k_common.h"
#include "k_reduce.h"

namespace sts {

namespace {

// Lower stencil neighbours in ascending lexicographic order.
__constant__ int c_off[9][3] = {{-1, -1, 0}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1}, {-1, 1, 0},
                                {0, -1, -1}, {0, -1, 0},  {0, -1, 1}, {0, 0, -1}};

struct PairTab {
  int n[9];
  int sm[9][8];
  int skm[9][8];
};

// For row i and its lower neighbour k = i + off[sk]: the lower neighbours
// m = i + off[sm] with m < k that are also lower neighbours of k, i.e.
// off[sm] - off[sk] = off[skm] for some lower slot skm.
constexpr PairTab make_pairs() {
  PairTab t{};
  const int off[9][3] = {{-1, -1, 0}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1}, {-1, 1, 0},
                         {0, -1, -1}, {0, -1, 0},  {0, -1, 1}, {0, 0, -1}};
  for (int sk = 0; sk < 9; ++sk) {
    t.n[sk] = 0;
    for (int sm = 0; sm < sk; ++sm) {
      const int d0 = off[sm][0] - off[sk][0], d1 = off[sm][1] - off[sk][1],
                d2 = off[sm][2] - off[sk][2];
      for (int s = 0; s < 9; ++s)
        if (off[s][0] == d0 && off[s][1] == d1 && off[s][2] == d2) {
          t.sm[sk][t.n[sk]] = sm;
          t.skm[sk][t.n[sk]] = s;
          t.n[sk]++;
        }
    }
  }
  return t;
}

__constant__ PairTab c_pairs = make_pairs();

struct BlockGeo {
  int B0, B1, B2, nbj, nbk;
  __device__ __forceinline__ void origin(const Grid &g, int bid, int &o0, int &o1, int &o2,
                                         int &e0, int &e1, int &e2) const {
    const int bk = bid % nbk;
    const int bj = (bid / nbk) % nbj;
    const int bi = bid / (nbk * nbj);
    o0 = bi * B0;
    o1 = bj * B1;
    o2 = bk * B2;
    e0 = min(B0, g.n0 - o0);
    e1 = min(B1, g.n1 - o1);
    e2 = min(B2, g.n2 - o2);
  }
};

constexpr int MAXB = 512;

template <int OP>
__global__ void __launch_bounds__(64)
    k_ilu_factor(Grid g, Coef C, double dt, BlockGeo bg, double *__restrict__ fac, int *bad) {
  __shared__ double sL[9][MAXB];
  __shared__ double sD[MAXB];
  const int bid = blockIdx.x, t = threadIdx.x;
  int o0, o1, o2, e0, e1, e2;
  bg.origin(g, bid, o0, o1, o2, e0, e1, e2);
  const int BS = bg.B0 * bg.B1 * bg.B2;
  const int li = t >> 3, lj = t & 7;
  const bool col = li < e0 && lj < e1;
  const int nlev = 3 * (e0 - 1) + 2 * (e1 - 1) + (e2 - 1) + 1;
  double *fb = fac + (size_t)bid * 10 * BS;
  for (int lev = 0; lev < nlev; ++lev) {
    const int lk = lev - 3 * li - 2 * lj;
    if (col && lk >= 0 && lk < e2) {
      const int gi = o0 + li, gj = o1 + lj, gk = o2 + lk;
      double row[27];
      row27<OP>(g, C, gi, gj, gk, row);
      const int l = (li * bg.B1 + lj) * bg.B2 + lk;
      double Lr[9];
      int nbl[9];
      unsigned valid = 0;
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        const int m0 = li + c_off[s][0], m1 = lj + c_off[s][1], m2 = lk + c_off[s][2];
        nbl[s] = (m0 * bg.B1 + m1) * bg.B2 + m2;
        if (m0 >= 0 && m1 >= 0 && m1 < e1 && m2 >= 0 && m2 < e2) valid |= 1u << s;
      }
      double dii = vol(g, gi, gj, gk) - dt * row[13];
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        Lr[s] = 0.0;
        if (valid & (1u << s)) {
          double a = -dt * row[13 + c_off[s][0] * 9 + c_off[s][1] * 3 + c_off[s][2]];
          const int kk = nbl[s];
          for (int q = 0; q < c_pairs.n[s]; ++q) {
            const int sm = c_pairs.sm[s][q];
            if (valid & (1u << sm)) a -= Lr[sm] * (sD[nbl[sm]] * sL[c_pairs.skm[s][q]][kk]);
          }
          Lr[s] = a / sD[kk];
          dii -= Lr[s] * (sD[kk] * Lr[s]);
        }
      }
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        sL[s][l] = Lr[s];
        fb[s * BS + l] = Lr[s];
      }
      sD[l] = dii;
      fb[9 * BS + l] = dii;
      if (!(dii > 0.0)) atomicOr(bad, 1);
    }
    __syncthreads();
  }
}

// z = (L D L^T)^-1 r on each block.  UPDATE: first x += alpha p, r -= alpha y
// (the PCG pass-B axpys), and reduce r.z and r.r.
template <bool UPDATE>
__global__ void __launch_bounds__(64)
    k_ilu_apply(Grid g, BlockGeo bg, const double *__restrict__ fac, double *__restrict__ x,
                const double *__restrict__ p, double *__restrict__ r,
                const double *__restrict__ y, double *__restrict__ z, double *part,
                long long cap, const PcgScalars *sc) {
  if (UPDATE && sc->done) return;
  __shared__ double sz[MAXB];
  __shared__ double sr[MAXB];
  const int bid = blockIdx.x, t = threadIdx.x;
  int o0, o1, o2, e0, e1, e2;
  bg.origin(g, bid, o0, o1, o2, e0, e1, e2);
  const int B1 = bg.B1, B2 = bg.B2, BS = bg.B0 * B1 * B2;
  const double *fb = fac + (size_t)bid * 10 * BS;
  const double alpha = UPDATE ? sc->alpha : 0.0;
  for (int l = t; l < BS; l += 64) {
    const int li = l / (B1 * B2), rem = l - li * B1 * B2, lj = rem / B2, lk = rem - lj * B2;
    double rv = 0.0;
    if (li < e0 && lj < e1 && lk < e2) {
      const int c = lin(g, o0 + li, o1 + lj, o2 + lk);
      if (UPDATE) {
        x[c] = x[c] + alpha * p[c];
        rv = r[c] - alpha * y[c];
        r[c] = rv;
      } else {
        rv = r[c];
      }
    }
    sr[l] = rv;
    sz[l] = rv;
  }
  __syncthreads();
  const int li = t >> 3, lj = t & 7;
  const bool col = li < e0 && lj < e1;
  const int nlev = 3 * (e0 - 1) + 2 * (e1 - 1) + (e2 - 1) + 1;
  // forward: z*_i = r_i - sum_k L_ik z*_k
  for (int lev = 0; lev < nlev; ++lev) {
    const int lk = lev - 3 * li - 2 * lj;
    if (col && lk >= 0 && lk < e2) {
      const int l = (li * B1 + lj) * B2 + lk;
      double acc = sz[l];
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        const int m0 = li + c_off[s][0], m1 = lj + c_off[s][1], m2 = lk + c_off[s][2];
        if (m0 >= 0 && m1 >= 0 && m1 < e1 && m2 >= 0 && m2 < e2)
          acc -= fb[s * BS + l] * sz[(m0 * B1 + m1) * B2 + m2];
      }
      sz[l] = acc;
    }
    __syncthreads();
  }
  // backward: z_i = z*_i / D_i - sum_j L_ji z_j over upper neighbours j
  for (int lev = nlev - 1; lev >= 0; --lev) {
    const int lk = lev - 3 * li - 2 * lj;
    if (col && lk >= 0 && lk < e2) {
      const int l = (li * B1 + lj) * B2 + lk;
      double acc = sz[l] / fb[9 * BS + l];
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        const int m0 = li - c_off[s][0], m1 = lj - c_off[s][1], m2 = lk - c_off[s][2];
        if (m0 < e0 && m1 >= 0 && m1 < e1 && m2 >= 0 && m2 < e2) {
          const int j = (m0 * B1 + m1) * B2 + m2;
          acc -= fb[s * BS + j] * sz[j];
        }
      }
      sz[l] = acc;
    }
    __syncthreads();
  }
  double rz = 0.0, rr = 0.0;
  for (int l = t; l < BS; l += 64) {
    const int li2 = l / (B1 * B2), rem = l - li2 * B1 * B2, lj2 = rem / B2, lk2 = rem - lj2 * B2;
    if (li2 < e0 && lj2 < e1 && lk2 < e2) {
      const int c = lin(g, o0 + li2, o1 + lj2, o2 + lk2);
      const double zv = sz[l];
      z[c] = zv;
      rz += sr[l] * zv;
      rr += sr[l] * sr[l];
    }
  }
  if (part) {
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (t == 0) {
      part[bid] = rz;
      part[cap + bid] = rr;
    }
  }
}

BlockGeo block_geo(const sts_ctx *c, const int block[3]) {
  BlockGeo bg;
  bg.B0 = block[0];
  bg.B1 = block[1];
  bg.B2 = block[2];
  bg.nbj = (c->n1 + bg.B1 - 1) / bg.B1;
  bg.nbk = (c->n2 + bg.B2 - 1) / bg.B2;
  return bg;
}

}  // namespace

int ilu_nblocks(const sts_ctx *c, const int block[3]) {
  return ((c->n0 + block[0] - 1) / block[0]) * ((c->n1 + block[1] - 1) / block[1]) *
         ((c->n2 + block[2] - 1) / block[2]);
}

int ilu_parts(const sts_ctx *c, const int block[3]) { return ilu_nblocks(c, block); }

void launch_ilu_factor(const sts_ctx *c, double dt, const int block[3], double *fac, int *bad) {
  const int nb = ilu_nblocks(c, block);
  if (c->op == OP_SPITZER)
    hipLaunchKernelGGL(k_ilu_factor<OP_SPITZER>, dim3(nb), dim3(64), 0, c->stream, c->grid(),
                       c->coef(), dt, block_geo(c, block), fac, bad);
  else
    hipLaunchKernelGGL(k_ilu_factor<OP_ISOTROPIC>, dim3(nb), dim3(64), 0, c->stream, c->grid(),
                       c->coef(), dt, block_geo(c, block), fac, bad);
}

void launch_ilu_apply_init(const sts_ctx *c, const int block[3], const double *fac,
                           const double *r, double *z) {
  const int nb = ilu_nblocks(c, block);
  hipLaunchKernelGGL(k_ilu_apply<false>, dim3(nb), dim3(64), 0, c->stream, c->grid(),
                     block_geo(c, block), fac, (double *)nullptr, (const double *)nullptr,
                     const_cast<double *>(r), (const double *)nullptr, z, (double *)nullptr, 0LL,
                     (const PcgScalars *)nullptr);
}

void launch_pass_b_ilu(const sts_ctx *c, const int block[3], const double *fac, double *x,
                       const double *p, double *r, const double *y, double *z, double *part,
                       const PcgScalars *sc) {
  const int nb = ilu_nblocks(c, block);
  hipLaunchKernelGGL(k_ilu_apply<true>, dim3(nb), dim3(64), 0, c->stream, c->grid(),
                     block_geo(c, block), fac, x, p, r, y, z, part, (long long)c->red_cap, sc);
}

}  // namespace sts
