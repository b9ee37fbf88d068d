// The operator application fused with the RKL2 stage recurrence.
//
// One kernel per stage (Sec. 3, Fig. "rkl2"): each cell gathers its
// 19-point (conduction) or 7-point (viscosity) stencil of u_{k-1}, forms
// F(u_{k-1}) = V^-1 (S u_{k-1} + g) and writes
//   u_k = mu_k u_{k-1} + nu_k u_{k-2} + (1 - mu_k - nu_k) u_0
//         + mu~_k dt F(u_{k-1}) + gamma~_k dt F(u_0)
// in the same pass, so a stage is one sweep over HBM.  u_{k-2}, u_0 and
// F(u_0) are read at the cell itself only, so u_k may overwrite u_{k-2} or
// u_0 in place.
#include "k_common.h"

namespace sts {

namespace {

constexpr int TX = 64, TY = 4;

template <int OP, int MODE>
__global__ void __launch_bounds__(TX *TY)
    k_stage(Grid g, Coef C, long long ncell, const double *__restrict__ ukm1, const double *ukm2,
            const double *u0, double *F0, double *out, double mu, double nu, double mut_dt,
            double gt_dt) {
  const int k = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int comp = blockIdx.z / g.n0;
  const int i = blockIdx.z - comp * g.n0;
  if (k >= g.n2 || j >= g.n1) return;
  const long long off = (long long)comp * ncell;
  const ArrayField f{ukm1 + off};
  const double su = (OP == OP_SPITZER) ? s19<true>(g, C, f, i, j, k) : s7<true>(g, C, f, i, j, k);
  const double F = su / vol(g, i, j, k);
  const long long c = off + lin(g, i, j, k);
  if (MODE == 0) {
    out[c] = F;
  } else if (MODE == 1) {
    F0[c] = F;
    out[c] = ukm1[c] + mut_dt * F;
  } else {
    out[c] = mu * ukm1[c] + nu * ukm2[c] + (1.0 - mu - nu) * u0[c] + mut_dt * F + gt_dt * F0[c];
  }
}

template <int OP>
void launch_op(const sts_ctx *c, int mode, int ncomp, const double *ukm1, const double *ukm2,
               const double *u0, double *F0, double *out, double mu, double nu, double mut_dt,
               double gt_dt) {
  const dim3 grid((c->n2 + TX - 1) / TX, (c->n1 + TY - 1) / TY, c->n0 * ncomp);
  const dim3 blk(TX, TY);
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((k_stage<OP, 0>), grid, blk, 0, c->stream, c->grid(), c->coef(),
                         c->ncell, ukm1, ukm2, u0, F0, out, mu, nu, mut_dt, gt_dt);
      break;
    case 1:
      hipLaunchKernelGGL((k_stage<OP, 1>), grid, blk, 0, c->stream, c->grid(), c->coef(),
                         c->ncell, ukm1, ukm2, u0, F0, out, mu, nu, mut_dt, gt_dt);
      break;
    default:
      hipLaunchKernelGGL((k_stage<OP, 2>), grid, blk, 0, c->stream, c->grid(), c->coef(),
                         c->ncell, ukm1, ukm2, u0, F0, out, mu, nu, mut_dt, gt_dt);
  }
}

}  // namespace

void launch_stage(const sts_ctx *c, int mode, int ncomp, const double *ukm1, const double *ukm2,
                  const double *u0, double *F0, double *out, double mu, double nu, double mut_dt,
                  double gt_dt) {
  if (c->op == OP_SPITZER)
    launch_op<OP_SPITZER>(c, mode, ncomp, ukm1, ukm2, u0, F0, out, mu, nu, mut_dt, gt_dt);
  else
    launch_op<OP_ISOTROPIC>(c, mode, ncomp, ukm1, ukm2, u0, F0, out, mu, nu, mut_dt, gt_dt);
}

}  // namespace sts
