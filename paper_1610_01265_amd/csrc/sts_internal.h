// Internal declarations shared by the host API and the kernel translation
// units of libsts.  Device kernels are launched only through the host
// launchers declared here.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/sts.h"

namespace sts {

// ---------------------------------------------------------------------------
// Separable geometry.  Every geometric factor of the finite-volume operator
// is a product of 1D tables along the three axes (spherical or Cartesian):
//   V      = V0[i] V1[j] V2[k]
//   A_a    = Aa0[i] Aa1[j] Aa2[k]            (area of the +a face of a cell)
//   1/dl_0 = IL00[i]                         (centre distance across +r face)
//   1/dl_1 = IL10[i] IL11[j]
//   1/dl_2 = IL20[i] IL21[j] IL22[k]
// IL00 / IL11 / IL22 hold 0 where the +face does not exist (last cell of a
// non-periodic axis).  Dirichlet faces on axis 0: area AB[s] A01[j] A02[k],
// centre-to-face distance DB[s].
// ---------------------------------------------------------------------------
enum Tab0 { T_V0, T_A00, T_A10, T_A20, T_IL00, T_IL10, T_IL20, T_IV0, NT0 };  // T_IV0 = 1 / T_V0
enum Tab1 { T_V1, T_A01, T_A11, T_A21, T_IL11, T_IL21, NT1 };
enum Tab2 { T_V2, T_A02, T_A12, T_A22, T_IL22, NT2 };

struct Grid {
  int n0, n1, n2;
  int per0, per1, per2;      // periodic flags
  int dir_lo, dir_hi;        // Dirichlet on axis-0 low / high side
  int wg_rev;                // debug: workgroups take their work in reversed order
  const double *t0, *t1, *t2;  // tables: t0[tab * n0 + i] etc.
  double ab_lo, ab_hi, db_lo, db_hi;
};

// Coefficients of the 19-point conduction operator (per-cell arrays) or of
// the isotropic 7-point operator (nu only).
struct Coef {
  const double *w0, *w1, *w2;     // face weights on +a faces of each cell
  const double *k01, *k02, *k12;  // edge weights, edge origin = the cell
  const double *wb_lo, *wb_hi;    // Dirichlet face weights [n1*n2]
  const double *ub_lo, *ub_hi;    // Dirichlet values [n1*n2]
  double nu;                      // isotropic mode
};

enum OpKind { OP_NONE = 0, OP_SPITZER = 1, OP_ISOTROPIC = 2 };

// PCG scalars kept on the device (alpha / beta never leave it).
struct PcgScalars {
  double rr;      // r . z
  double rr_old;
  double alpha, beta;
  double bnorm2;  // ||b||^2
  double rnorm2;  // ||r||^2
  double py;
  double tol2;    // (rtol ||b||)^2
  int done;       // 1 once converged / broken down; later kernels no-op
  int iters;
  int status;     // 0 ok, 1 converged, -4 breakdown
  int maxit;
};

// Per-kernel timing (STS_PROFILE, sts_set_profile): an event pair recorded
// on the context's stream around each launcher's launch.
struct ProfRec {
  const char *name;
  hipEvent_t a, b;
};
class ProfScope {
 public:
  ProfScope(const sts_ctx *c, const char *name);
  ~ProfScope();
  ProfScope(const ProfScope &) = delete;
  ProfScope &operator=(const ProfScope &) = delete;

 private:
  sts_ctx *c_ = nullptr;
  const char *name_ = nullptr;
  hipEvent_t a_ = nullptr;
};
#define STS_PROF(c, name) ::sts::ProfScope sts_prof_scope_(c, name)

// the workgroup's logical index (reversed in the debug order)
__device__ __forceinline__ int wg_index(int rev) {
  return rev ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
}

}  // namespace sts

struct sts_ctx {
  int coord = 0;
  int n0 = 0, n1 = 0, n2 = 0;
  long long ncell = 0;
  int bc[6] = {0, 0, 0, 0, 0, 0};
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // geometry tables
  double *d_t0 = nullptr, *d_t1 = nullptr, *d_t2 = nullptr;
  double ab_lo = 0, ab_hi = 0, db_lo = 0, db_hi = 0;

  // operator
  int op = sts::OP_NONE;
  double nu = 0.0;
  double *d_w = nullptr;      // 6 * ncell: w0 w1 w2 k01 k02 k12
  float *d_wf = nullptr;      // FP32 copy of d_w (precision form)
  int prec = 0;               // 0: FP64, 1: FP32 storage (precision form)
  double *d_sdiag = nullptr;  // S_cc (homogeneous diagonal) per cell
  double *d_bnd = nullptr;    // 4 * n1*n2: wb_lo wb_hi ub_lo ub_hi
  double ub_const[2] = {0.0, 0.0};
  bool ub_array[2] = {false, false};
  double dt_euler = -1.0;     // cached Gershgorin limit (< 0: not computed)

  // workspace
  double *d_rk = nullptr;     // RKL2: F0 and 2 (4 with fused stages) state buffers
  int rk_ncomp = 0;
  float *d_rk32 = nullptr;    // FP32 form RKL2: F0, delta_a, delta_b
  void *d_scratch = nullptr;  // device address of the static scratch array (not owned)
  std::string scratch_err;    // why d_scratch is null, if it is
  int rk32_ncomp = 0;
  float *d_pcg32 = nullptr;   // FP32 form PCG: 1/A_ii, e, r, p0, p1, y, z
  double *d_pcg = nullptr;    // PCG vectors
  double *d_red = nullptr;    // reduction partials
  int red_cap = 0;
  sts::PcgScalars *d_sc = nullptr;
  sts::PcgScalars *h_sc = nullptr;  // pinned mirror
  void *d_gfac = nullptr;     // factored preconditioner G, BF16 [4][ncell]
  bool gfac_set = false;
  double *d_pct = nullptr;    // its PCG work vector t = G^T r
  double *d_pcobj = nullptr;  // sts_pc_objective: w, y, r, q, s, p (6 x ncell)
  sts::PcgScalars *d_sc0 = nullptr;  // all-zero scalars: a stand-alone pass A (y = A p)
  double *d_ilu = nullptr;    // block ILU0 factors
  long long ilu_cap = 0;
  int *d_flag = nullptr;      // device flags (input checks, ILU breakdown)
  double *d_tmp = nullptr;    // small device scratch for host-read scalars

  // resistive diffusion of A on cell edges (set by sts_set_resistivity)
  std::vector<double> hf[3];  // face coordinates (host copy)
  double res_eta = 0.0;       // 0: not set
  long long res_ne[3] = {0, 0, 0}, res_nf[3] = {0, 0, 0};  // edges / faces per component
  int res_off[18] = {};       // offsets of the 18 weight tables in d_rtab
  double *d_rtab = nullptr;
  double *d_rws = nullptr;    // faces x 2, edges x 6 (PCG vectors)
  void *h_pin = nullptr;      // pinned host mirror of flags / scalars (two 128-byte slots)
  int debug = 0;              // STS_DEBUG_* flags (sts_set_debug)
  // per-kernel timing: records and a pool of reusable events
  bool profile = false;
  mutable std::vector<sts::ProfRec> prof;
  mutable std::vector<hipEvent_t> prof_pool;
  hipEvent_t ev[2] = {nullptr, nullptr};  // PCG batch completion (pipelined polls)

  sts::Grid grid() const;
  sts::Coef coef() const;
};

namespace sts {

// geometry / coefficient setup (k_coef.hip)
void launch_spitzer_coef(const sts_ctx *c, const double *T, double kappa0, const double *b0,
                         const double *b1, const double *b2);
void launch_spitzer_coef_f32(const sts_ctx *c, const float *T, double kappa0, const float *b0,
                             const float *b1, const float *b2);
void launch_check_spitzer_f32(const sts_ctx *c, const float *T, const float *b0, const float *b1,
                              const float *b2, int *flag);
void launch_dirichlet_weights(const sts_ctx *c);
void launch_sdiag(const sts_ctx *c);
void launch_gershgorin(const sts_ctx *c, double *partials, int nparts);
int gershgorin_parts(const sts_ctx *c);

// stencil kernels (k_stencil.hip)
// mode 0: out = F(u); mode 1: F0 = F(u0), out = u0 + mut_dt F0;
// mode 2: out = mu ukm1 + nu ukm2 + (1-mu-nu) u0 + mut_dt F(ukm1) + gt_dt F0
void launch_stage(const sts_ctx *c, int mode, int ncomp, const double *ukm1, const double *ukm2,
                  const double *u0, double *F0, double *out, double mu, double nu, double mut_dt,
                  double gt_dt);

// Conduction with kappa = kappa0 max(u, 0)^{5/2} taken from the stencil
// input itself (k_nonlinear.hip); modes as launch_stage, one component.
void launch_stage_nl(const sts_ctx *c, int mode, const double *ukm1, const double *ukm2,
                     const double *u0, double *F0, double *out, double mu, double nu,
                     double mut_dt, double gt_dt, double kappa0, const double *b0,
                     const double *b1, const double *b2);

// Resistive diffusion on edges (k_resist.hip).  Phi / Wf: face-sized scratch
// of the two-sweep form (face sweep, then edge sweep), which the set-up
// operators use; F, the residual and pass A run one fused sweep.
int res_parts(const sts_ctx *c);        // two-sweep form's partials; 1D grids
int res_parts_fused(const sts_ctx *c);  // fused sweep's partials
void launch_res_F(const sts_ctx *c, const double *E, double *FE);
void launch_res_gershgorin(const sts_ctx *c, double *Phi, double *part);
void launch_res_rhs(const sts_ctx *c, const double *En, double dt, double *x, double *b,
                    double *invd, double *Phi, double *Wf, double *part);
void launch_res_residual(const sts_ctx *c, const double *b, const double *x, double dt,
                         double *r, double *part);
// pb != null (and !first): beta and the previous iteration's stopping test
// from a fused pass B's partials pb (npb), the iteration count being `iters`
void launch_res_pass_a(const sts_ctx *c, double dt, const double *r, const double *invd,
                       const double *pold, double *p, double *y, double *part,
                       const PcgScalars *sc, int first, const double *pb = nullptr,
                       int npb = 0, int iters = 0);
// PCG pieces over a vector of n entries (k_pcg.hip)
void launch_init_p_n(const sts_ctx *c, long long n, const double *r, const double *invd,
                     double *p, double *part, int nparts);
// pa != null: alpha from pass A's partials pa (npa) inside the sweep
void launch_pass_b_jacobi_n(const sts_ctx *c, long long n, double *x, const double *p, double *r,
                            const double *y, const double *invd, double *part, int nparts,
                            const PcgScalars *sc, const double *pa = nullptr, int npa = 0);

// FP32 form (k_stencil.hip, k_pcg.hip)
void f32_F0(const sts_ctx *c, int ncomp, const double *u0, float *F0, float *d1, double mut_dt);
void f32_apply(const sts_ctx *c, int ncomp, const double *u, double *Fu);
void f32_stage(const sts_ctx *c, int last, int ncomp, const float *dkm1, const float *dkm2,
               const float *F0, void *out, const double *u0, double mu, double nu, double mut_dt,
               double g_dt);
// pb / pa != null: the in-sweep finalizers, as launch_pass_a and
// launch_pass_b_jacobi_fused
void f32_pass_a(const sts_ctx *c, double dt, const float *z, const float *pold, float *pnew,
                float *y, double *part, const PcgScalars *sc, int first,
                const double *pb = nullptr, int npb = 0, int iters = 0);
void f32_residual(const sts_ctx *c, const double *b, const double *x, double dt, double *r,
                  double *part);
void f32_inner_init(const sts_ctx *c, const double *r64, const double *invd64, float *r,
                    float *invd, float *e, float *z, double *part);
void f32_pass_b(const sts_ctx *c, float *e, const float *p, float *r, const float *y,
                const float *invd, float *z, double *part, const PcgScalars *sc,
                const double *pa = nullptr, int npa = 0);
void f32_add_to(const sts_ctx *c, double *x, const float *e);
void launch_fill_f32(const sts_ctx *c, float *p, long long n, float v);

// PCG (k_pcg.hip).  Partial-sum buffers hold two regions of red_cap values.
int stencil_parts(const sts_ctx *c);  // workgroups of the 3D-tiled kernels
int pass_b_parts(const sts_ctx *c);   // workgroups of the 1D kernels
int pcg_parts(const sts_ctx *c);      // max of the two
void launch_be_rhs(const sts_ctx *c, const double *u_n, double dt, double *b, double *invd,
                   double *part);
void launch_residual_init(const sts_ctx *c, const double *b, const double *x, double dt,
                          const double *invd, const double *zilu, double *r, double *p,
                          double *part);
// zout (may be null): where the Jacobi z = r / A_ii is stored for pass A
void launch_init_p(const sts_ctx *c, const double *r, const double *invd, const double *zilu,
                   double *p, double *part, double *zout);
void launch_finalize_init_n(const sts_ctx *c, const double *pb, int nb, const double *prr,
                            int nrr, const double *prz, int nrz, PcgScalars *sc, double rtol,
                            int maxit);
void launch_finalize_init3(const sts_ctx *c, const double *pb, const double *prr,
                           const double *prz, PcgScalars *sc, double rtol, int maxit);
// pass A: p = z + beta p_old (z stored by the previous pass), y = A p, partial p.y
// pb != null (and !first): the sweep first evaluates the previous
// iteration's end (stopping test, beta) from a fused pass B's partials pb
// (npb per region), the iteration count being `iters`.
void launch_pass_a(const sts_ctx *c, double dt, const double *z, const double *pold,
                   double *pnew, double *y, double *part, const PcgScalars *sc, int first,
                   const double *pb = nullptr, int npb = 0, int iters = 0);
void launch_finalize_alpha(const sts_ctx *c, const double *part, int nparts, PcgScalars *sc);
void launch_finalize_beta(const sts_ctx *c, const double *part, int nparts, PcgScalars *sc);
// Jacobi pass B that forms alpha itself from pass A's partials pa (npa), then
// updates x, r, z (z = r / A_ii, for the next pass A) and writes its partials (r.z, r.r) to part, part + cap; the
// end of its iteration is evaluated by the next fused pass A, or, after the
// last one, by launch_finalize_check.
void launch_pass_b_jacobi_fused(const sts_ctx *c, double *x, const double *p, double *r,
                                const double *y, const double *invd, double *z, double *part,
                                PcgScalars *sc, const double *pa, int npa);
// the same sweep with alpha from sc (written by launch_finalize_alpha)
void launch_pass_b_jacobi(const sts_ctx *c, double *x, const double *p, double *r,
                          const double *y, const double *invd, double *z, double *part,
                          PcgScalars *sc);
void launch_finalize_check(const sts_ctx *c, const double *part, int nparts, int iters,
                           PcgScalars *sc);
// In-sweep finalizers: every pass-B workgroup re-sums pass A's partials and
// every pass-A workgroup pass B's, a cost that grows with the product of the
// two workgroup counts.  Measured per Jacobi iteration: fused 4-5 % faster at
// 128 x 128 x 256 (1024 pass-A workgroups), separate 0.7 % faster at
// 256 x 256 x 512 (8192) and 0.8 % at 1023 x 1024 x 1024 (262144).
constexpr int kFuseMaxParts = 4096;
inline bool fuse_finalizers(const sts_ctx *c, int pass_a_parts) {
  return !(c->debug & STS_DEBUG_SEPARATE_FINALIZE) && pass_a_parts <= kFuseMaxParts;
}
void launch_true_residual(const sts_ctx *c, const double *b, const double *x, double dt,
                          double *part);
void launch_sum2(const sts_ctx *c, const double *part, int nparts, double *out2);
void launch_fill(const sts_ctx *c, double *p, long long n, double v);
void launch_check_spitzer(const sts_ctx *c, const double *T, const double *b0, const double *b1,
                          const double *b2, int *flag);

// block ILU0 (k_ilu.hip)
int ilu_nblocks(const sts_ctx *c, const int block[3]);
void launch_ilu_factor(const sts_ctx *c, double dt, const int block[3], double *fac, int *bad);
void launch_ilu_apply_init(const sts_ctx *c, const int block[3], const double *fac,
                           const double *r, double *z);
void launch_pass_b_ilu(const sts_ctx *c, const int block[3], const double *fac, double *x,
                       const double *p, double *r, const double *y, double *z, double *part,
                       const PcgScalars *sc);
int ilu_parts(const sts_ctx *c, const int block[3]);

// factored preconditioner M^-1 = G G^T (k_pc.hip); g: BF16 [4][ncell]
int pc_parts(const sts_ctx *c);  // workgroups (partials) of the pc kernels
// t = G^T x (- sub, may be null); sc (may be null): no-op once sc->done
void launch_pc_gt(const sts_ctx *c, const void *g, const double *x, const double *sub,
                  double *t, const PcgScalars *sc);
// z = G t; sc (may be null): no-op once sc->done
void launch_pc_g(const sts_ctx *c, const void *g, const double *t, double *z,
                 const PcgScalars *sc);
// factor from network outputs o4 [cells][4] (null: point Jacobi) at dt
void launch_pc_build(const sts_ctx *c, double dt, const float *o4, void *g, int *bad);
void launch_pc_check(const sts_ctx *c, const float *g32, void *g, int *bad);
void launch_pc_pack(const sts_ctx *c, double dt, double lscale, const double *T, double tsh,
                    double tsc, void *x);
void launch_pc_grad(const sts_ctx *c, double dt, const void *g, const double *y,
                    const double *r, const double *s, const double *z, double *dg, void *dout,
                    double *part);
// x += alpha p, r_out = r_in - alpha y, t = G^T r_out (r_in != r_out); partial
// sums t.t and r.r to part, part + cap; pa != null: alpha from pass A's
// partials pa (npa) inside the sweep, else from sc
void launch_pc_xr_gt(const sts_ctx *c, const void *g, double *x, const double *p,
                     const double *rin, double *rout, const double *y, double *t, double *part,
                     PcgScalars *sc, const double *pa, int npa);
// host helpers of the factor network (sts_api.cpp): the factor built from
// network outputs o4 [cells][4] at dt (STS_BREAKDOWN if an entry is not
// finite), and the objective's sweeps at dt for probe z, writing dL/dG (dg)
// and / or the network's output gradient (dout, bf16 [cells][16]) and the
// r.r partials (pc_parts of them) into the context's reduction buffer
sts_status build_pc_factor(sts_ctx *ctx, double dt, const float *o4);
sts_status pc_objective_sweeps(sts_ctx *ctx, double dt, const double *z, double *dg, void *dout);

}  // namespace sts
