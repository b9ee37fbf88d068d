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
// Factor layout: fac[block][slot][B0*B1*B2] with slots 0..8 = L, 9 = 1/D,
// the cell index inside a block being (i' B1 + j') B2 + k'.
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

// XCD-aware order: workgroup w runs on XCD w % 8.  The returned logical
// index gives each XCD a contiguous range, so neighbouring blocks (which
// share cache lines of the grid-layout arrays along phi) meet in one L2.
__device__ __forceinline__ int xcd_order(int w, int nwg) {
  const int q8 = nwg >> 3, r8 = nwg & 7, x8 = w & 7, s8 = w >> 3;
  return x8 < r8 ? x8 * (q8 + 1) + s8 : r8 * (q8 + 1) + (x8 - r8) * q8 + s8;
}

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

__device__ __forceinline__ bool in_block(int m0, int m1, int m2, int e0, int e1, int e2) {
  return m0 >= 0 && m0 < e0 && m1 >= 0 && m1 < e1 && m2 >= 0 && m2 < e2;
}

// Factorisation.  Phase 1: every lane assembles the block-restricted rows of
// A = V - dt S for 8 cells (fully parallel) into LDS.  Phase 2: hyperplane
// by hyperplane, each lane turns its cell's row into L (in place) and the
// pivot D.  Phase 3: L and 1/D go to HBM.
constexpr int FTH = 256;
template <int OP>
__global__ void __launch_bounds__(FTH)
    k_ilu_factor(Grid g, Coef C, double dt, BlockGeo bg, double *__restrict__ fac, int *bad) {
  __shared__ double sL[9][MAXB];
  __shared__ double sD[MAXB];
  const int bid = xcd_order(wg_index(g.wg_rev), gridDim.x), t = threadIdx.x;
  int o0, o1, o2, e0, e1, e2;
  bg.origin(g, bid, o0, o1, o2, e0, e1, e2);
  const int B1 = bg.B1, B2 = bg.B2, BS = bg.B0 * B1 * B2;
  for (int l = t; l < BS; l += FTH) {
    const int li = l / (B1 * B2), rem = l - li * B1 * B2, lj = rem / B2, lk = rem - lj * B2;
    if (li < e0 && lj < e1 && lk < e2) {
      const int gi = o0 + li, gj = o1 + lj, gk = o2 + lk;
      double row[27];
      row27<OP>(g, C, gi, gj, gk, row);
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        const bool v = in_block(li + c_off[s][0], lj + c_off[s][1], lk + c_off[s][2], e0, e1, e2);
        sL[s][l] = v ? -dt * row[13 + c_off[s][0] * 9 + c_off[s][1] * 3 + c_off[s][2]] : 0.0;
      }
      sD[l] = vol(g, gi, gj, gk) - dt * row[13];
    } else {
#pragma unroll
      for (int s = 0; s < 9; ++s) sL[s][l] = 0.0;
      sD[l] = 1.0;
    }
  }
  __syncthreads();
  // Phase 2 runs on wavefront 0 alone: its LDS operations complete in order,
  // so a wave-level compiler barrier separates the levels.
  const int li = t >> 3, lj = t & 7;
  const bool col = li < e0 && lj < e1;
  const int nlev = 3 * (e0 - 1) + 2 * (e1 - 1) + (e2 - 1) + 1;
  if (t < 64)
  for (int lev = 0; lev < nlev; ++lev) {
    const int lk = lev - 3 * li - 2 * lj;
    if (col && lk >= 0 && lk < e2) {
      const int l = (li * B1 + lj) * B2 + lk;
      int nbl[9];
      unsigned valid = 0;
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        const int m0 = li + c_off[s][0], m1 = lj + c_off[s][1], m2 = lk + c_off[s][2];
        nbl[s] = (m0 * B1 + m1) * B2 + m2;
        if (in_block(m0, m1, m2, e0, e1, e2)) valid |= 1u << s;
      }
      double dii = sD[l];
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        if (valid & (1u << s)) {
          const int kk = nbl[s];
          double a = sL[s][l];
          for (int q = 0; q < c_pairs.n[s]; ++q) {
            const int sm = c_pairs.sm[s][q];
            if (valid & (1u << sm)) a -= sL[sm][l] * (sD[nbl[sm]] * sL[c_pairs.skm[s][q]][kk]);
          }
          const double Lv = a / sD[kk];
          sL[s][l] = Lv;
          dii -= Lv * (sD[kk] * Lv);
        }
      }
      sD[l] = dii;
      if (!(dii > 0.0)) atomicOr(bad, 1);
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  double *fb = fac + (size_t)bid * 10 * BS;
  for (int l = t; l < BS; l += FTH) {
#pragma unroll
    for (int s = 0; s < 9; ++s) fb[s * BS + l] = sL[s][l];
    fb[9 * BS + l] = 1.0 / sD[l];
  }
}

// z = (L D L^T)^-1 r on each block.  UPDATE: first x += alpha p, r -= alpha y
// (the PCG pass-B axpys), and reduce r.z and r.r.  The block's factors are
// staged in LDS once by all four wavefronts (coalesced, loads issued
// unconditionally with clamped indices); wavefront 0 then runs both
// substitution sweeps out of LDS, while the others wait at the barriers.
constexpr int ATH = 256;
template <bool UPDATE>
__global__ void __launch_bounds__(ATH)
    k_ilu_apply(Grid g, BlockGeo bg, const double *__restrict__ fac, double *__restrict__ x,
                const double *__restrict__ p, double *__restrict__ r,
                const double *__restrict__ y, double *__restrict__ z, double *part,
                long long cap, const PcgScalars *sc) {
  if (UPDATE && sc->done) return;
  __shared__ double sL[9][MAXB];
  __shared__ double sI[MAXB];  // 1 / D
  __shared__ double sz[MAXB];
  __shared__ double sr[MAXB];
  const int bid = xcd_order(wg_index(g.wg_rev), gridDim.x), t = threadIdx.x;
  int o0, o1, o2, e0, e1, e2;
  bg.origin(g, bid, o0, o1, o2, e0, e1, e2);
  const int B1 = bg.B1, B2 = bg.B2, BS = bg.B0 * B1 * B2;
  const double *fb = fac + (size_t)bid * 10 * BS;
  const double alpha = UPDATE ? sc->alpha : 0.0;
  constexpr int PER = MAXB / ATH;  // cells per thread in the load / store phases
  // factors -> LDS
#pragma unroll
  for (int s = 0; s < 10; ++s) {
    double v[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) v[m] = fb[s * BS + min(t + ATH * m, BS - 1)];
#pragma unroll
    for (int m = 0; m < PER; ++m)
      if (t + ATH * m < BS) (s < 9 ? sL[s] : sI)[t + ATH * m] = v[m];
  }
  // x, r updates; r -> LDS
  int cidx[PER];
  bool cval[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int l = t + ATH * m;
    const int li = l / (B1 * B2), rem = l - li * B1 * B2, lj = rem / B2, lk = rem - lj * B2;
    cval[m] = l < BS && li < e0 && lj < e1 && lk < e2;
    cidx[m] = lin(g, o0 + min(li, e0 - 1), o1 + min(lj, e1 - 1), o2 + min(lk, e2 - 1));
  }
  double rl[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int c = cidx[m];
    if (UPDATE) {
      const double xv = x[c], pv = p[c], rv = r[c], yv = y[c];
      rl[m] = cval[m] ? rv - alpha * yv : 0.0;
      if (cval[m]) {
        x[c] = xv + alpha * pv;
        r[c] = rl[m];
      }
    } else {
      const double rv = r[c];
      rl[m] = cval[m] ? rv : 0.0;
    }
    const int l = t + ATH * m;
    if (l < BS) {
      sz[l] = rl[m];
      sr[l] = rl[m];
    }
  }
  __syncthreads();
  // Both sweeps run on wavefront 0 alone: a level's rows read z values
  // written at earlier levels by other lanes of the same wavefront, and the
  // LDS operations of one wavefront complete in issue order, so a wave-level
  // compiler barrier (no instruction) between levels is the only ordering
  // needed.  The sweeps are branch-free: L entries of neighbours outside the
  // block are stored as zero, so a neighbour index only has to stay inside
  // the LDS arrays (clamped); the 18 LDS reads of a row are issued before a
  // pairwise sum of the 9 products.
  if (t < 64) {
    const int li = t >> 3, lj = t & 7;
    const bool col = li < e0 && lj < e1;
    const int nlev = 3 * (e0 - 1) + 2 * (e1 - 1) + (e2 - 1) + 1;
    int loff[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) loff[s] = (c_off[s][0] * B1 + c_off[s][1]) * B2 + c_off[s][2];
    auto sum9 = [](const double *lv, const double *zv) {
      const double a = lv[0] * zv[0] + lv[1] * zv[1], b = lv[2] * zv[2] + lv[3] * zv[3];
      const double c = lv[4] * zv[4] + lv[5] * zv[5], d = lv[6] * zv[6] + lv[7] * zv[7];
      return ((a + b) + (c + d)) + lv[8] * zv[8];
    };
    // forward: z*_i = r_i - sum_k L_ik z*_k
    for (int lev = 0; lev < nlev; ++lev) {
      const int lk = lev - 3 * li - 2 * lj;
      if (col && lk >= 0 && lk < e2) {
        const int l = (li * B1 + lj) * B2 + lk;
        double lv[9], zv[9];
#pragma unroll
        for (int s = 0; s < 9; ++s) {
          lv[s] = sL[s][l];
          zv[s] = sz[min(max(l + loff[s], 0), BS - 1)];
        }
        sz[l] = sz[l] - sum9(lv, zv);
      }
      __builtin_amdgcn_wave_barrier();
    }
    // backward: z_i = z*_i / D_i - sum_j L_ji z_j over upper neighbours j
    for (int lev = nlev - 1; lev >= 0; --lev) {
      const int lk = lev - 3 * li - 2 * lj;
      if (col && lk >= 0 && lk < e2) {
        const int l = (li * B1 + lj) * B2 + lk;
        double lv[9], zv[9];
#pragma unroll
        for (int s = 0; s < 9; ++s) {
          const int j = min(max(l - loff[s], 0), BS - 1);
          lv[s] = (l - loff[s] == j) ? sL[s][j] : 0.0;
          zv[s] = sz[j];
        }
        sz[l] = sz[l] * sI[l] - sum9(lv, zv);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  double rz = 0.0, rr = 0.0;
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int l = t + ATH * m;
    if (cval[m]) {
      const double zv = sz[l];
      z[cidx[m]] = zv;
      rz += sr[l] * zv;
      rr += sr[l] * sr[l];
    }
  }
  if (part) wg_sum2<ATH>(rz, rr, t, part + bid, part + cap + bid);
}

// The same apply for 8 x 8 x 8 blocks with compile-time neighbour offsets.
// Every neighbour read is an immediate-offset LDS load off the row's own
// address: z has a zero pad of PADZ entries before and after the block and
// each L row a zero pad of PADZ after it, so no index needs clamping, and an
// upper-neighbour coupling L_ji is read as stored (the factorisation stores
// zero for couplings that leave the block, which covers the pads' role).
// Edge blocks (fewer than 8 cells along an axis) are handled as full 8^3
// blocks whose missing cells have L = 0, 1/D = 1 and r = 0.
constexpr int B8 = 8, BS8 = 512;
constexpr int PADZ = (B8 + 1) * B8 + 1;  // largest |offset| of a lower neighbour
constexpr int LROW = BS8 + PADZ;
// Persistent form: workgroup w takes blocks w, w + G, w + 2G, ... (G =
// gridDim.x, at most the number of workgroups resident at once).  While one
// wavefront runs a block's two substitution sweeps out of LDS, every
// wavefront's loads of the next block's factors and vectors are in flight
// into registers, so HBM latency overlaps the latency-bound sweeps.
struct Blk8 {
  double f[10][BS8 / ATH];  // L (9 slots) and 1/D of this thread's cells
  double xv[BS8 / ATH], pv[BS8 / ATH], rv[BS8 / ATH], yv[BS8 / ATH];
  int c[BS8 / ATH];         // grid index (clamped into the grid)
  bool v[BS8 / ATH];        // cell inside the grid
};

template <bool UPDATE>
__global__ void __launch_bounds__(ATH)
    k_ilu_apply8(Grid g, BlockGeo bg, int nblk, const double *__restrict__ fac,
                 double *__restrict__ x, const double *__restrict__ p, double *__restrict__ r,
                 const double *__restrict__ y, double *__restrict__ z, double *part,
                 long long cap, const PcgScalars *sc) {
  if (UPDATE && sc->done) return;
  __shared__ double sL[9 * LROW];
  __shared__ double sI[BS8];
  __shared__ double szp[PADZ + BS8 + PADZ];
  double *sz = szp + PADZ;
  const int t = threadIdx.x;
  const double alpha = UPDATE ? sc->alpha : 0.0;
  constexpr int PER = BS8 / ATH;
  // pads -> 0 (the per-block staging below never writes them)
  for (int q = t; q < 9 * PADZ; q += ATH) sL[(q / PADZ) * LROW + BS8 + q % PADZ] = 0.0;
  for (int q = t; q < PADZ; q += ATH) {
    szp[q] = 0.0;
    szp[PADZ + BS8 + q] = 0.0;
  }
  auto fetch = [&](int bid, Blk8 &B) {
    int o0, o1, o2, e0, e1, e2;
    bg.origin(g, bid, o0, o1, o2, e0, e1, e2);
    const double *fb = fac + (size_t)bid * 10 * BS8;
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int l = t + ATH * m;
      const int li = l >> 6, lj = (l >> 3) & 7, lk = l & 7;
      B.v[m] = li < e0 && lj < e1 && lk < e2;
      B.c[m] = lin(g, o0 + min(li, e0 - 1), o1 + min(lj, e1 - 1), o2 + min(lk, e2 - 1));
    }
#pragma unroll
    for (int s = 0; s < 10; ++s)
#pragma unroll
      for (int m = 0; m < PER; ++m) B.f[s][m] = fb[s * BS8 + t + ATH * m];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      B.rv[m] = r[B.c[m]];
      if (UPDATE) {
        B.xv[m] = x[B.c[m]];
        B.pv[m] = p[B.c[m]];
        B.yv[m] = y[B.c[m]];
      }
    }
  };
  constexpr int LO[9] = {-72, -65, -64, -63, -56, -9, -8, -7, -1};
  auto sum9 = [](const double *lv, const double *zv) {
    const double a = lv[0] * zv[0] + lv[1] * zv[1], b = lv[2] * zv[2] + lv[3] * zv[3];
    const double c = lv[4] * zv[4] + lv[5] * zv[5], e = lv[6] * zv[6] + lv[7] * zv[7];
    return ((a + b) + (c + e)) + lv[8] * zv[8];
  };
  double rz = 0.0, rr = 0.0;
  Blk8 B;
  const int w = wg_index(g.wg_rev);
  int bid = w;
  if (bid < nblk) fetch(bid, B);
  for (; bid < nblk; bid += gridDim.x) {
    // stage this block: factors -> LDS; x, r updates; r -> LDS (0 outside the grid)
#pragma unroll
    for (int s = 0; s < 10; ++s)
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        if (s < 9)
          sL[s * LROW + t + ATH * m] = B.f[s][m];
        else
          sI[t + ATH * m] = B.f[s][m];
      }
    double rl[PER], xn[PER];
    int cidx[PER];
    bool cval[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      cidx[m] = B.c[m];
      cval[m] = B.v[m];
      if (UPDATE) {
        rl[m] = cval[m] ? B.rv[m] - alpha * B.yv[m] : 0.0;
        xn[m] = B.xv[m] + alpha * B.pv[m];
      } else {
        rl[m] = cval[m] ? B.rv[m] : 0.0;
      }
      sz[t + ATH * m] = rl[m];
    }
    // stores after every prefetched operand is consumed: vector memory
    // counters complete in order, so a store issued earlier would make the
    // wait for a later load also wait for the store
    if (UPDATE) {
#pragma unroll
      for (int m = 0; m < PER; ++m)
        if (cval[m]) {
          x[cidx[m]] = xn[m];
          r[cidx[m]] = rl[m];
        }
    }
    __syncthreads();
    // the next block's loads go out before the sweeps
    if (bid + (int)gridDim.x < nblk) fetch(bid + gridDim.x, B);
    if (t < 64) {
      const int li = t >> 3, lj = t & 7;
      const int d = 3 * li + 2 * lj;
      constexpr int NLEV = 3 * 7 + 2 * 7 + 7 + 1;
      // forward: z*_i = r_i - sum_k L_ik z*_k
      for (int lev = 0; lev < NLEV; ++lev) {
        const int lk = lev - d;
        if (lk >= 0 && lk < B8) {
          const int l = t * B8 + lk;
          const double *zr = sz + l;
          const double *lr = sL + l;
          double lv[9], zv[9];
#pragma unroll
          for (int s = 0; s < 9; ++s) {
            lv[s] = lr[s * LROW];
            zv[s] = zr[LO[s]];
          }
          sz[l] = zr[0] - sum9(lv, zv);
        }
        __builtin_amdgcn_wave_barrier();
      }
      // backward: z_i = z*_i / D_i - sum_j L_ji z_j over upper neighbours j = i - LO[s]
      for (int lev = NLEV - 1; lev >= 0; --lev) {
        const int lk = lev - d;
        if (lk >= 0 && lk < B8) {
          const int l = t * B8 + lk;
          const double *zr = sz + l;
          double lv[9], zv[9];
#pragma unroll
          for (int s = 0; s < 9; ++s) {
            lv[s] = sL[s * LROW + l - LO[s]];
            zv[s] = zr[-LO[s]];
          }
          sz[l] = zr[0] * sI[l] - sum9(lv, zv);
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int l = t + ATH * m;
      if (cval[m]) {
        const double zv = sz[l];
        z[cidx[m]] = zv;
        rz += rl[m] * zv;
        rr += rl[m] * rl[m];
      }
    }
    __syncthreads();  // the LDS is restaged for the next block
  }
  if (part) wg_sum2<ATH>(rz, rr, t, part + w, part + cap + w);
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

// Workgroups of the persistent 8^3 apply: at most three per CU are resident
// (51.5 KB of LDS each) on the 256 CUs; the blocks are spread evenly.
static int ilu8_grid(int nb) {
  constexpr int kResident = 3 * 256;
  const int per = (nb + kResident - 1) / kResident;
  return (nb + per - 1) / per;
}

bool is8(const int block[3]) { return block[0] == 8 && block[1] == 8 && block[2] == 8; }

int ilu_parts(const sts_ctx *c, const int block[3]) {
  const int nb = ilu_nblocks(c, block);
  return is8(block) ? ilu8_grid(nb) : nb;
}

void launch_ilu_factor(const sts_ctx *c, double dt, const int block[3], double *fac, int *bad) {
  STS_PROF(c, "launch_ilu_factor");
  const int nb = ilu_nblocks(c, block);
  if (c->op == OP_SPITZER)
    hipLaunchKernelGGL(k_ilu_factor<OP_SPITZER>, dim3(nb), dim3(FTH), 0, c->stream, c->grid(),
                       c->coef(), dt, block_geo(c, block), fac, bad);
  else
    hipLaunchKernelGGL(k_ilu_factor<OP_ISOTROPIC>, dim3(nb), dim3(FTH), 0, c->stream, c->grid(),
                       c->coef(), dt, block_geo(c, block), fac, bad);
}

void launch_ilu_apply_init(const sts_ctx *c, const int block[3], const double *fac,
                           const double *r, double *z) {
  STS_PROF(c, "launch_ilu_apply_init");
  const int nb = ilu_nblocks(c, block);
  if (is8(block)) {
    hipLaunchKernelGGL(k_ilu_apply8<false>, dim3(ilu8_grid(nb)), dim3(ATH), 0, c->stream,
                       c->grid(), block_geo(c, block), nb, fac, (double *)nullptr,
                       (const double *)nullptr,
                       const_cast<double *>(r), (const double *)nullptr, z, (double *)nullptr,
                       0LL, (const PcgScalars *)nullptr);
    return;
  }
  hipLaunchKernelGGL(k_ilu_apply<false>, dim3(nb), dim3(ATH), 0, c->stream, c->grid(),
                     block_geo(c, block), fac, (double *)nullptr, (const double *)nullptr,
                     const_cast<double *>(r), (const double *)nullptr, z, (double *)nullptr, 0LL,
                     (const PcgScalars *)nullptr);
}

void launch_pass_b_ilu(const sts_ctx *c, const int block[3], const double *fac, double *x,
                       const double *p, double *r, const double *y, double *z, double *part,
                       const PcgScalars *sc) {
  STS_PROF(c, "launch_pass_b_ilu");
  const int nb = ilu_nblocks(c, block);
  if (is8(block)) {
    hipLaunchKernelGGL(k_ilu_apply8<true>, dim3(ilu8_grid(nb)), dim3(ATH), 0, c->stream,
                       c->grid(), block_geo(c, block), nb, fac, x, p, r, y, z, part,
                       (long long)c->red_cap, sc);
    return;
  }
  hipLaunchKernelGGL(k_ilu_apply<true>, dim3(nb), dim3(ATH), 0, c->stream, c->grid(),
                     block_geo(c, block), fac, x, p, r, y, z, part, (long long)c->red_cap, sc);
}

}  // namespace sts
