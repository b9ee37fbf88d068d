/*
 * sts.h - C ABI of the MI355X library for advancing stiff parabolic operators
 * (anisotropic Spitzer conduction and artificial viscosity) by RKL2 super
 * time-stepping or by backward Euler with preconditioned conjugate gradients,
 * after Caplan, Mikic, Linker & Lionello (2016), "Advancing parabolic operators
 * in thermodynamic MHD models: explicit super time-stepping versus implicit
 * schemes with Krylov solvers".
 *
 * Conventions for every call
 *  - Field arrays are DEVICE pointers owned by the caller, contiguous
 *    [n0][n1][n2] with axis 2 (phi) fastest, FP64 unless stated otherwise.
 *    Axis order is (r, theta, phi) on the spherical shell, (x, y, z) in a box.
 *  - Host arrays are marked HOST.  The library never frees caller memory; it
 *    owns only its workspace (coefficients, solver vectors, factors), which it
 *    allocates at the first call that needs it and frees in sts_destroy.
 *  - All work is enqueued on the context's HIP stream.  Calls that return
 *    host scalars (sts_dt_euler, rkl2_step's s_used is host-known,
 *    be_pcg_solve, sts_be_residual) synchronise that stream before returning.
 *  - Errors are return codes; sts_last_error() gives a text.  Non-finite or
 *    out-of-range arguments give STS_EINVAL and leave outputs untouched.
 *  - A context is not thread-safe; use one per host thread / stream.
 */
#ifndef STS_H
#define STS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sts_ctx sts_ctx; /* opaque */

typedef enum {
  STS_OK = 0,
  STS_NOT_CONVERGED = 1, /* PCG reached maxit; x holds the last iterate        */
  STS_EINVAL = -1,       /* bad argument / shape / non-finite value             */
  STS_EHIP = -2,         /* a HIP runtime call failed                           */
  STS_ENOMEM = -3,       /* device allocation failed                            */
  STS_BREAKDOWN = -4     /* PCG p.Ap <= 0, or an ILU0 pivot <= 0                */
} sts_status;

typedef enum { STS_SPHERICAL = 0, STS_CARTESIAN = 1 } sts_coord;
typedef enum { STS_BC_ZEROFLUX = 0, STS_BC_DIRICHLET = 1, STS_BC_PERIODIC = 2 } sts_bc;
typedef enum { STS_PC_JACOBI = 0, STS_PC_BLOCK_ILU0 = 1 } sts_pc;

/* sts_create - a context for one grid and one operator.
 * Grid (Sec. 4.2 and Table "tab:grid" of the paper: a logically rectangular,
 * non-uniform spherical grid): n0 x n1 x n2 cells whose faces are the HOST
 * arrays f0[n0+1], f1[n1+1], f2[n2+1] (strictly increasing; for the shell
 * r, colatitude theta in (0, pi), longitude phi).  Cell centres are face
 * midpoints.  bc[6] = {axis0-, axis0+, axis1-, axis1+, axis2-, axis2+}:
 * STS_BC_PERIODIC must be set on both sides of an axis (>= 3 cells);
 * STS_BC_DIRICHLET only on the axis-0 sides (values: sts_set_dirichlet,
 * default 0).  stream: a hipStream_t (NULL = the default stream).
 * The device is the current HIP device at this call.  */
sts_status sts_create(sts_ctx **out, int coord, int n0, int n1, int n2,
                      const double *f0, const double *f1, const double *f2,
                      const int bc[6], void *stream);
sts_status sts_destroy(sts_ctx *ctx);
sts_status sts_set_stream(sts_ctx *ctx, void *stream);
const char *sts_last_error(const sts_ctx *ctx);
/* number of cells n0*n1*n2 */
long long sts_num_cells(const sts_ctx *ctx);

/* sts_set_spitzer - lagged-diffusivity conduction operator (Sec. 1; Eq.
 * mhd:e1, blue box): D = kappa0 T^{5/2} b b^T with T (> 0) and the unit
 * vector b = (b0, b1, b2) in the local (r, theta, phi) basis, all device FP64
 * [n0][n1][n2].  The diffusivity is frozen here until the next set_* call.
 * Forms the 3 face and 3 edge coefficient arrays of the 19-point
 * finite-volume operator F(u) = V^-1 (S u + g), S = -Hessian of the discrete
 * energy (face terms + edge cross terms), so that S is exactly symmetric.  */
sts_status sts_set_spitzer(sts_ctx *ctx, const double *T, double kappa0,
                           const double *b0, const double *b1, const double *b2);

/* sts_set_isotropic - viscosity operator nu * Laplacian per velocity
 * component (Eq. mhd:v, blue box, with rho = 1 and uniform nu > 0): the
 * 7-point finite-volume Laplacian whose coefficients are separable geometry
 * times nu (no per-cell coefficient arrays).  */
sts_status sts_set_isotropic(sts_ctx *ctx, double nu);

/* sts_set_spitzer_f32 - the precision form of sts_set_spitzer: T and the unit
 * vector b are device FP32 arrays [n0][n1][n2]; the face / edge coefficients
 * are formed from them (FP64 set-up arithmetic) and stored in FP32.  Until the
 * next set_* call the context runs the FP32 form:
 *  - rkl2_step iterates FP32 increments delta_k = u_k - u_0 (stencil and stage
 *    arithmetic in FP32) and returns u^{n+1} = u_0 + delta_s accumulated in
 *    FP64 (u stays an FP64 array);
 *  - be_pcg_solve (Jacobi only) refines in mixed precision: FP64 outer
 *    residual b - A x (FP32 coefficients widened), FP32-vector inner PCG with
 *    FP64 dot products, alpha / beta and norms, x += correction in FP64;
 *    *iters counts inner iterations, *relres is the FP64 true residual;
 *  - apply_F evaluates F(u) from FP64 u with the FP32 coefficients.
 * The FP32 form targets <= 1e-6 relative error in T against the FP64
 * solution (a stated error of the form, not a parity bound).  */
sts_status sts_set_spitzer_f32(sts_ctx *ctx, const float *T, double kappa0, const float *b0,
                               const float *b1, const float *b2);
/* sts_set_isotropic_f32 - the viscosity operator of sts_set_isotropic run in
 * the FP32 form described above.  */
sts_status sts_set_isotropic_f32(sts_ctx *ctx, double nu);

/* sts_set_dirichlet - boundary values on axis-0 side `side` (0 = low,
 * 1 = high), used if that side is STS_BC_DIRICHLET: `values` is a device
 * FP64 [n1][n2] array copied into the context, or NULL to use the constant
 * `value`.  Takes effect for the operator set by the next set_* call and
 * for the current one.  */
sts_status sts_set_dirichlet(sts_ctx *ctx, int side, const double *values, double value);

/* sts_dt_euler - explicit Euler limit dt_E = 2 / max_i sum_j |M_ij|, M = V^-1 S
 * (Appendix B, Eqs. dteuler and gstb: the Gershgorin bound on |lambda|_max,
 * summed along rows of M).  Synchronises the stream.  */
sts_status sts_dt_euler(sts_ctx *ctx, double *dt_e);

/* apply_F - Fu = F(u) = V^-1 (S u + g) (Eq. pde with the lagged operator), for
 * ncomp independent components stored one after the other
 * (u[ncomp][n0][n1][n2]).  u and Fu must not overlap.  */
sts_status apply_F(sts_ctx *ctx, const double *u, double *Fu, int ncomp);

/* rkl2_step - one RKL2 super-step of length dt (Sec. 3, Fig. "rkl2" and its
 * coefficient block), in place: u holds u^n on entry and u^{n+1} = u_s on
 * return.  s <= 0 selects the minimal stable stage count
 * s = ceil((sqrt(9 + 16 dt/dt_E) - 1)/2) (Eq. rkl2_s; dt_E from sts_dt_euler,
 * computed once per operator); s >= 2 forces s.  *s_used (may be NULL)
 * receives s.  Each stage is one fused stencil + recurrence kernel.  */
sts_status rkl2_step(sts_ctx *ctx, double *u, int ncomp, double dt, int s, int *s_used);

/* be_pcg_solve - one backward-Euler step (Sec. 2.1, Eqs. BE, BE_lin,
 * BE_linsolve) written as (V - dt S) u^{n+1} = V u^n + dt g and solved by the
 * PCG of Fig. "pcg" (Sec. 2.2).  u_n: u^n (read only).  x: on entry the
 * initial guess (pass a copy of u^n for the paper's x0 = u^n), on return the
 * solution; x must not alias u_n.  pc: STS_PC_JACOBI (PC1: diagonal) or
 * STS_PC_BLOCK_ILU0 (PC2: zero-fill ILU on non-overlapping blocks of
 * block[3] cells, each <= 8, couplings across blocks dropped; Sec. 2.3,
 * Appendix A).  Stops when ||b - A x_k||_2 <= rtol ||b||_2 (recursively
 * updated residual) or after maxit iterations.  *iters and *relres (may be
 * NULL) receive the iteration count and the final relative residual.
 * Returns STS_NOT_CONVERGED at maxit and STS_BREAKDOWN if p.Ap <= 0 or a
 * pivot <= 0.  Synchronises the stream.  */
sts_status be_pcg_solve(sts_ctx *ctx, const double *u_n, double *x, double dt, int pc,
                        const int block[3], double rtol, int maxit, int *iters, double *relres);

/* sts_be_residual - true relative residual ||b - A x||_2 / ||b||_2 of the BE
 * system above, computed with FP64 dot products.  Synchronises the stream.  */
sts_status sts_be_residual(sts_ctx *ctx, const double *u_n, const double *x, double dt,
                           double *relres);

#ifdef __cplusplus
}
#endif
#endif /* STS_H */
