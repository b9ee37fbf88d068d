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
typedef enum { STS_PC_JACOBI = 0, STS_PC_BLOCK_ILU0 = 1, STS_PC_FACTOR = 2 } sts_pc;

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

/* Diagnostics (not in the paper).
 * sts_set_profile - per-kernel timing on (on != 0) or off; the environment
 * variable STS_PROFILE (set and not "0") switches it on at sts_create.  While
 * on, every kernel launch of the library is bracketed by a pair of HIP events
 * on the context's stream.
 * sts_profile_summary - writes a text table into buf (HOST, cap bytes): one
 * line per launcher, "calls total_ms avg_us min_us max_us name", by total
 * time; reset != 0 clears the records.  STS_EINVAL if buf is too small.
 * Synchronises the stream.
 * sts_set_debug - flags; STS_DEBUG_WG_REVERSE makes the stencil, PCG,
 * block-ILU0, factor, CNN and resistivity kernels that use LDS or write
 * per-workgroup partial sums take their work in reversed workgroup order (each
 * workgroup still computes the same tiles and partial sums), a self-check
 * that results do not depend on the order in which workgroups run: results
 * are bit for bit those of the normal order.  STS_DEBUG_SEPARATE_FINALIZE
 * makes the Jacobi and factor PCG evaluate alpha, beta and the stopping
 * test in single-workgroup kernels between the sweeps instead of inside
 * them (the same sums in the same order: bit for bit the same iterates), for
 * timing the two forms; without it the in-sweep form is taken up to 4096
 * workgroups of the plane march (beyond, the separate one).  */
enum { STS_DEBUG_WG_REVERSE = 1, STS_DEBUG_SEPARATE_FINALIZE = 2 };
sts_status sts_set_profile(sts_ctx *ctx, int on);
sts_status sts_profile_summary(sts_ctx *ctx, char *buf, long long cap, int reset);
sts_status sts_set_debug(sts_ctx *ctx, int flags);

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

/* rkl2_step_noalloc - rkl2_step for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results (bit for bit) and kernels as
 * rkl2_step; the stage buffers (F0 and two state arrays in FP64, or F0 and two
 * FP32 increments in the precision form) live in a static device array of
 * 96 MiB that each GPU holds from sts_create until the process ends, so the
 * call allocates nothing.  Limits and errors:
 *  - ncell * ncomp <= 4,194,304 in FP64 (8,388,608 in the FP32 form), else
 *    STS_EINVAL (nothing enqueued);
 *  - s <= 0 needs dt_E already computed for the current operator (a prior
 *    sts_dt_euler, rkl2_step or rkl_step call), else STS_EINVAL;
 *  - STS_EHIP if the array's device address could not be resolved.
 * The array is shared by every context on one GPU and keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap in
 * time on one GPU (other streams, other threads) race.  */
sts_status rkl2_step_noalloc(sts_ctx *ctx, double *u, int ncomp, double dt, int s, int *s_used);

/* rkl_step - the super-step with the variants discussed in Sec. 6 (with
 * Fig. "ampfac") and after Eq. rkl2_s, in this order:
 *   euler_fraction in [0, 1): first advance euler_fraction * dt by explicit
 *     Euler sub-steps u += h F(u) of equal length h <= euler_cfl * dt_E
 *     (euler_cfl in (0, 1]; ignored when euler_fraction = 0);
 *   then nsub (>= 1) sub-steps of the remaining time with scheme 2 (RKL2,
 *     Fig. "rkl2") or 1 (RKL1: Y_1 = Y_0 + w1 h F(Y_0), Y_j = mu_j Y_{j-1} +
 *     nu_j Y_{j-2} + mu~_j h F(Y_{j-1}), mu_j = (2j-1)/j, nu_j = -(j-1)/j,
 *     mu~_j = w1 (2j-1)/j, w1 = 2/(s^2+s)), each with the minimal stable s
 *     for its length (RKL2: Eq. rkl2_s; RKL1: s^2 + s >= 2 h/dt_E) plus
 *     extra (>= 0) stages, rounded up to odd if odd != 0.
 * In place on u (ncomp components).  *n_apply (may be NULL) receives the
 * number of operator evaluations.  The FP32 form accepts RKL2 sub-steps only
 * (STS_EINVAL otherwise).  */
sts_status rkl_step(sts_ctx *ctx, double *u, int ncomp, double dt, int scheme, int extra, int odd,
                    int nsub, double euler_fraction, double euler_cfl, int *n_apply);

/* apply_F_nonlinear - Fu = F(u) = V^-1 (S(kappa(u)) u + g(kappa(u))): the
 * conduction operator of sts_set_spitzer with the diffusivity taken from u
 * itself, kappa(u) = kappa0 max(u, 0)^{5/2}, D = kappa b b^T (Eq. mhd:e1,
 * blue box; the operator RKL2 can apply without lagging, Sec. 2.4 and
 * Sec. 3.1).  u, Fu, b0, b1, b2: device FP64 [n0][n1][n2]; b is the unit
 * vector in the local basis; u and Fu must not overlap.  Uses the context's
 * grid, boundaries and Dirichlet values only (no set_* call needed; the
 * stored operator is left as it is).  Non-finite inputs give non-finite
 * outputs; no input check is made.  */
sts_status apply_F_nonlinear(sts_ctx *ctx, const double *u, double *Fu, double kappa0,
                             const double *b0, const double *b1, const double *b2);

/* rkl2_step_nonlinear - one RKL2 super-step (Sec. 3, Fig. "rkl2") of
 * du/dt = F(u) with F the operator of apply_F_nonlinear: every stage takes
 * kappa from its own input u_{k-1}, F0 = F(u^n), b fixed over the step.  In
 * place on u (device FP64, u^n in, u^{n+1} out; one component).  The call
 * first sets the context's operator to the lagged operator at u^n, as
 * sts_set_spitzer(ctx, u, kappa0, b0, b1, b2) does (same input checks: u
 * finite and > 0, b finite; STS_EINVAL otherwise, u untouched); s <= 0 takes
 * the minimal stable s (Eq. rkl2_s) for dt / dt_E of that operator, s >= 2
 * forces s.  *s_used (may be NULL) receives s.  Each stage is one kernel that
 * forms the face / edge coefficients from u_{k-1} and b on the fly.
 * Synchronises the stream (input check; dt_E when s <= 0).  */
sts_status rkl2_step_nonlinear(sts_ctx *ctx, double *u, double dt, double kappa0,
                               const double *b0, const double *b1, const double *b2, int s,
                               int *s_used);

/* be_pcg_solve - one backward-Euler step (Sec. 2.1, Eqs. BE, BE_lin,
 * BE_linsolve) written as (V - dt S) u^{n+1} = V u^n + dt g and solved by the
 * PCG of Fig. "pcg" (Sec. 2.2).  u_n: u^n (read only).  x: on entry the
 * initial guess (pass a copy of u^n for the paper's x0 = u^n), on return the
 * solution; x must not alias u_n.  pc: STS_PC_JACOBI (PC1: diagonal),
 * STS_PC_BLOCK_ILU0 (PC2: zero-fill ILU on non-overlapping blocks of
 * block[3] cells, each <= 8, couplings across blocks dropped; Sec. 2.3,
 * Appendix A) or STS_PC_FACTOR (M^-1 = G G^T with the context's factor G:
 * sts_set_pc_factor or cnn_pc_factor; not in the paper).  Stops when ||b - A x_k||_2 <= rtol ||b||_2 (recursively
 * updated residual) or after maxit iterations.  *iters and *relres (may be
 * NULL) receive the iteration count and the final relative residual.
 * Returns STS_NOT_CONVERGED at maxit and STS_BREAKDOWN if p.Ap <= 0 or a
 * pivot <= 0.  Synchronises the stream.  */
sts_status be_pcg_solve(sts_ctx *ctx, const double *u_n, double *x, double dt, int pc,
                        const int block[3], double rtol, int maxit, int *iters, double *relres);

/* The factored preconditioner M^-1 = G G^T (not in the paper: a third
 * preconditioner for the PCG of Fig. "pcg" beside PC1 and PC2 of Sec. 2.3,
 * whose factor a network can predict, cnn_pc_factor).  G is lower
 * triangular in the cells' lexicographic order: row c holds G[c, c] and
 * G[c, c - e_a] for the -1 neighbours along axes a = 0, 1, 2 that lie in the
 * grid (no wrap across a periodic axis); with a positive diagonal G is
 * nonsingular and M^-1 symmetric positive definite.  Layout: device FP32
 * g[4][n0][n1][n2], g[0] = G[c, c], g[1 + a] = G[c, c - e_a] (entries whose
 * neighbour does not exist are ignored).  The context stores the entries
 * rounded to BF16 (to nearest, ties to even): every application, solve and
 * objective uses the rounded factor; vectors and sums stay FP64.  */

/* sts_set_pc_factor - stores g, rounded to BF16, in the context (used by
 * be_pcg_solve with STS_PC_FACTOR until the next call).  STS_EINVAL if a
 * rounded diagonal entry is not finite and positive or another entry is not
 * finite.  Synchronises.  */
sts_status sts_set_pc_factor(sts_ctx *ctx, const float *g);
/* sts_apply_pc_factor - z = G (G^T r) with the context's factor; r, z device
 * FP64 [n0][n1][n2], not overlapping.  */
sts_status sts_apply_pc_factor(sts_ctx *ctx, const double *r, double *z);
/* sts_pc_objective - the factor's training objective for a probe vector z
 * (device FP64): L = ||G^T A G z - z||_2^2 / N with A = V - dt S of the
 * context's operator (N cells), into *loss (HOST), and, if dg != NULL, its
 * gradient dL/dG[c, m] = 2 (y_c r_m + s_c z_m) / N (w = G z, y = A w,
 * r = G^T y - z, s = A G r) in the layout of g as device FP64 [4][cells]
 * (zero where the entry does not exist).  Synchronises.  */
sts_status sts_pc_objective(sts_ctx *ctx, double dt, const double *z, double *loss, double *dg);

/* Resistive diffusion of the vector potential, dA/dt = -eta curl curl A
 * (Eq. mhd:a, boxed; eta stands for c^2 eta / 4 pi, constant as in the
 * paper's runs), advanced by BE + PCG with PC1 as MAS does for this term
 * (Sec. 4.2).  A is staggered on the cell edges (MAS keeps every vector
 * component staggered so that div B = 0 holds exactly): the unknowns are the
 * line integrals E = A . dl along the edges, one device FP64 vector
 * [E_r | E_t | E_p] with E_r[n0][m1][m2] on r-edges (r_c, th_f, ph_f),
 * E_t[m0][n1][m2] on theta-edges (r_f, th_c, ph_f), E_p[m0][m1][n2] on
 * phi-edges (r_f, th_f, ph_c), m_a = n_a on a periodic axis, n_a + 1
 * otherwise (sts_resistivity_sizes).  Face fluxes Phi = C E by Stokes'
 * theorem (normals +r, +theta, +phi, right-hand rule), energy
 * 1/2 sum_f (l*_f / S_f) Phi_f^2 (S_f face area, l*_f distance between the
 * centres of the cells it separates), edge mass H_e = S*_e / L_e (dual-face
 * area over edge length), all exact for spherical cells:
 *   F(E) = -eta H^-1 C^T diag(l* / S) C E.
 * Edges lying in a non-periodic boundary surface keep their values
 * (tangential E given) and F = 0 there, whatever the scalar boundary kinds.  */

/* sts_set_resistivity - builds the edge / face weight tables for eta > 0
 * (finite); independent of the scalar operator set by sts_set_*.  */
sts_status sts_set_resistivity(sts_ctx *ctx, double eta);
/* sts_resistivity_sizes - sizes[3] = number of E_r, E_t, E_p entries (HOST). */
sts_status sts_resistivity_sizes(const sts_ctx *ctx, long long sizes[3]);
/* apply_F_resistivity - FE = F(E), both device FP64 edge vectors, not
 * overlapping.  */
sts_status apply_F_resistivity(sts_ctx *ctx, const double *E, double *FE);
/* resistivity_dt_euler - 2 / (largest Gershgorin row sum of eta H^-1 K over
 * the interior edges), Appendix B's bound applied to this operator.
 * Synchronises the stream.  */
sts_status resistivity_dt_euler(sts_ctx *ctx, double *dt_e);
/* resistivity_be_pcg_solve - one BE step (H + dt eta C^T W C) E^{n+1} = H E^n
 * on the interior edges (the fixed edges' terms on the right-hand side) by
 * the PCG of Fig. "pcg" with PC1.  E_n: E^n (read only).  E: on entry the
 * initial guess on interior edges (pass a copy of E^n for the paper's
 * x0 = u^n), on return E^{n+1}, its fixed edges set to E^n's; E must not
 * alias E_n.  Stops at ||b - A x||_2 <= rtol ||b||_2 over the interior edges
 * (recursively updated residual) or after maxit iterations; *iters, *relres
 * as be_pcg_solve.  Returns STS_NOT_CONVERGED at maxit, STS_BREAKDOWN if
 * p.Ap <= 0.  Synchronises the stream.  */
sts_status resistivity_be_pcg_solve(sts_ctx *ctx, const double *E_n, double *E, double dt,
                                    double rtol, int maxit, int *iters, double *relres);

/* sts_be_residual - true relative residual ||b - A x||_2 / ||b||_2 of the BE
 * system above, computed with FP64 dot products.  Synchronises the stream.  */
sts_status sts_be_residual(sts_ctx *ctx, const double *u_n, const double *x, double dt,
                           double *relres);

/* ------------------------------------------------------------------------
 * Learned initial guess for the backward-Euler solve.
 *
 * Not part of the paper: the PCG of Fig. "pcg" (Sec. 2.2) starts from an
 * initial guess x_0, which the paper takes as u^n.  This network predicts
 * x_0 from two fields instead.  It is a 3D CNN of `layers` 3x3x3
 * convolutions, 2 -> 16 -> ... -> 16 -> 1 channels, ReLU between layers,
 * "same" padding: zero along axes 0 and 1, circular along axis 2.  Inputs:
 *   channel 0 = dt F(T_prev) * rhs_scale   (the BE increment of one
 *               explicit step, F as in apply_F with the context's operator)
 *   channel 1 = (T_prev - T_shift) * T_scale
 * Output d; the guess is x_0 = T_prev + delta_scale * d.
 * Arithmetic: BF16 weights and activations, FP32 accumulation on the MFMA
 * units (v_mfma_f32_16x16x32_bf16), FP32 master weights and Adam state.
 * Activations are stored channel-last, bf16 [cells][16] (16 channels per
 * cell, unused channels zero); the first layer's 2 inputs and the last
 * layer's 1 output are padded to 16 channels with zero weights.
 *
 * Host weight vector (cnn_set_weights / cnn_get_weights), FP32, per layer l
 * with c_in = (l == 0 ? 2 : 16), c_out = (l == last ? 1 : 16):
 *   W[c_out][c_in][3][3][3]   (kernel offsets a, b, c in -1..1 along axes
 *                              0, 1, 2, at index [a+1][b+1][c+1]; the
 *                              output at a cell sums W * input(cell + (a,b,c)))
 *   bias[c_out]
 * layers = 4 gives 15169 values.  A new network holds zeros.
 * The sts_cnn handle uses its context's grid and stream; destroy it before
 * the context.  It allocates its workspace (about 7 x 32 bytes per cell)
 * at cnn_create.
 * ------------------------------------------------------------------------ */
typedef struct sts_cnn sts_cnn; /* opaque */

/* cnn_create - network of `layers` (2..8) convolutions with `channels` (16)
 * hidden channels on ctx's grid.  */
sts_status cnn_create(sts_cnn **out, sts_ctx *ctx, int layers, int channels);
sts_status cnn_destroy(sts_cnn *net);

/* cnn_num_params - length of the host weight vector.  */
long long cnn_num_params(const sts_cnn *net);

/* cnn_set_weights / cnn_get_weights - copy the FP32 weight vector from / to
 * the HOST array w[n] (n must equal cnn_num_params).  Setting resets the
 * Adam state (moments and step count).  Synchronise the stream.  */
sts_status cnn_set_weights(sts_cnn *net, const float *w, long long n);
sts_status cnn_get_weights(sts_cnn *net, float *w, long long n);

/* cnn_state_size / cnn_get_state / cnn_set_state - the whole training state,
 * for checkpoint and resume (not in the paper): buf (HOST, FP32,
 * cnn_state_size = 3 x layers x 6928 values) holds the padded master
 * parameters, then Adam's first and second moments, each in the padded
 * layout cnn_weight_grad writes; meta (HOST, 8 values) = Adam step count,
 * the four scalings of cnn_set_norm (the factor network uses T_shift and
 * T_scale), beta1, beta2, eps.  Setting checks finiteness, second moments
 * >= 0, zeros at the padding entries and the ranges of cnn_set_norm and
 * cnn_set_adam (STS_EINVAL otherwise); a network set from a state continues
 * training exactly as the one the state was taken from.  Synchronise.  */
long long cnn_state_size(const sts_cnn *net);
sts_status cnn_get_state(sts_cnn *net, float *buf, long long n, double meta[8]);
sts_status cnn_set_state(sts_cnn *net, const float *buf, long long n, const double meta[8]);

/* cnn_set_norm - the four input / output scalings above (finite; the
 * scales nonzero).  Defaults 1, 0, 1, 1.  */
sts_status cnn_set_norm(sts_cnn *net, double rhs_scale, double T_shift, double T_scale,
                        double delta_scale);

/* cnn_moments - mean and root-mean-square of scale * (x - y) over the cells
 * (y may be NULL: read as 0) into the HOST array out[2], FP64 sums in a
 * fixed order.  A helper for choosing the scalings.  Synchronises.  */
sts_status cnn_moments(sts_cnn *net, const double *x, const double *y, double scale,
                       double out[2]);

/* cnn_pack_input - network input x16 (bf16 [cells][16]) from F_prev =
 * F(T_prev) (as apply_F returns it), dt and T_prev, with the set scalings:
 * x16[c][0] = bf16(float(dt F_prev[c] rhs_scale)),
 * x16[c][1] = bf16(float((T_prev[c] - T_shift) T_scale)), others 0.  */
sts_status cnn_pack_input(sts_cnn *net, const double *F_prev, double dt, const double *T_prev,
                          void *x16);

/* cnn_conv - one convolution of layer `layer` with the current weights
 * (rounded to bf16), on in16 (bf16 [cells][16]):
 *   kind 0: out = bf16 [cells][16], ReLU(conv + bias)        (hidden layer)
 *   kind 1: out = FP32 [cells],     channel 0 of conv + bias (output layer)
 *   kind 2: out = bf16 [cells][16], adjoint convolution (input gradient:
 *           transposed channels, mirrored offsets) times (mask16 > 0);
 *           mask16 NULL: no mask
 *   kind 3: out = FP32 [cells][16], conv + bias
 *   kind 4: out = FP32 [cells][16], adjoint convolution, no mask
 *   kind 5: out = FP32 [cells][4],  channels 0..3 of conv + bias (output
 *           layer of the factor network)
 * in16 and out must not overlap.  */
sts_status cnn_conv(sts_cnn *net, int layer, int kind, const void *in16, const void *mask16,
                    void *out);

/* cnn_weight_grad - gradient of a scalar loss with respect to layer
 * `layer`'s padded parameters, given the layer input act16 and the gradient
 * dout16 with respect to its output (both bf16 [cells][16]):
 *   grad[(co*16 + ci)*27 + t] = sum_cells dout16[cell][co] act16[cell + off(t)][ci]
 *   grad[16*16*27 + co]       = sum_cells dout16[cell][co]
 * (t = 9(a+1) + 3(b+1) + (c+1)), grad a DEVICE FP32 array of 6928 values.
 * FP32 sums in a fixed order.  */
sts_status cnn_weight_grad(sts_cnn *net, int layer, const void *act16, const void *dout16,
                           float *grad);

/* cnn_forward - x0 = T_prev + delta_scale * network(F_prev, dt, T_prev).  */
sts_status cnn_forward(sts_cnn *net, const double *F_prev, double dt, const double *T_prev,
                       double *x0);

/* cnn_set_adam - the constants of the Adam optimiser (Kingma & Ba, 2015)
 * used by cnn_train_step and cnn_adam_step: moment decay rates beta1,
 * beta2 in [0, 1) and eps > 0 (defaults 0.9, 0.999, 1e-8; held as FP32).
 * Takes effect at the next step; the moments are kept.  */
sts_status cnn_set_adam(sts_cnn *net, double beta1, double beta2, double eps);

/* cnn_adam_step - one Adam step of the FP32 master parameters with the
 * caller's gradient grad (a DEVICE FP32 array of layers * 6928 values, per
 * layer in the padded layout cnn_weight_grad writes; entries of padding,
 * which has no parameter, are ignored), rate lr > 0.  With t the number of
 * steps taken since cnn_set_weights, including this one:
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   p = p - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 * in FP32, then the bf16 copies of the weights are refreshed.  For a caller
 * that forms the gradient itself (e.g. summed over several samples or
 * devices).  Does not synchronise.  */
sts_status cnn_adam_step(sts_cnn *net, const float *grad, float lr);

/* cnn_train_step - one Adam step (constants of cnn_set_adam, rate lr)
 * on the loss mean_cells (d - (x_star - T_prev) / delta_scale)^2, with
 * gradients by back-propagation through the same kernels.  *loss (may be
 * NULL; then the call does not synchronise) receives the loss before the
 * step.  */
sts_status cnn_train_step(sts_cnn *net, const double *F_prev, double dt, const double *T_prev,
                          const double *x_star, float lr, double *loss);

/* cnn_guess - the initial guess for be_pcg_solve(ctx, T_prev, x0, dt, ...)
 * with the context's current operator: F_prev = F(T_prev), the network's
 * guess, and a fallback: x0 = T_prev instead when the network's guess is
 * non-finite or has a larger BE residual than T_prev.  *used_net (may be
 * NULL) receives 1 if the network's guess was kept; relres[2] (may be NULL)
 * the relative residuals of the network's guess and of T_prev.
 * Synchronises the stream.  */
sts_status cnn_guess(sts_cnn *net, const double *T_prev, double dt, double *x0, int *used_net,
                     double relres[2]);

/* The factor network: a network of the same architecture whose last layer
 * has 4 output channels o = (o0, o1, o2, o3) per cell, which give the factor
 * of the STS_PC_FACTOR preconditioner M^-1 = G G^T (see sts_set_pc_factor):
 *   G[c, c] = d_c exp(o0_c),  G[c, c - e_a] = d_c o_(1+a),c,  d_c = A_cc^-1/2,
 * with A = V - dt S the backward-Euler matrix of the context's operator, so
 * that M^-1 is symmetric positive definite for any outputs and point Jacobi
 * for o = 0 (not in the paper: a learned alternative to PC1 / PC2 of
 * Sec. 2.3).  Its input features (bf16 [cells][16]) are
 *   x[c][0] = log(A_cc / V_c) / log(1 + dt / dt_E),
 *   x[c][1] = (T[c] - T_shift) T_scale, others 0.
 * cnn_num_params, cnn_set_weights, cnn_get_weights, cnn_conv,
 * cnn_weight_grad, cnn_set_adam, cnn_adam_step and cnn_destroy apply as for
 * the initial-guess network (the last layer has 4 output channels);
 * cnn_pack_input, cnn_forward, cnn_train_step and cnn_guess reject it.  */
sts_status cnn_create_pc(sts_cnn **out, sts_ctx *ctx, int layers, int channels);
/* cnn_pc_set_norm - the temperature scalings of the input features.  */
sts_status cnn_pc_set_norm(sts_cnn *net, double T_shift, double T_scale);
/* cnn_pc_factor - the network's factor for the context's current operator
 * at dt, from the temperature T (device FP64), stored as the context's
 * STS_PC_FACTOR factor.  Fallback: if an entry is not finite the context's
 * factor becomes point Jacobi (o = 0) and *used_net (may be NULL) is 0.
 * Synchronises.  */
sts_status cnn_pc_factor(sts_cnn *net, const double *T, double dt, int *used_net);
/* cnn_pc_grad - the gradient of the factor's objective for the probe vector
 * z (device FP64, drawn by the caller) with respect to the network
 * parameters, into grad (device FP32, layers x 6928 values in the padded
 * layout of cnn_weight_grad), by back-propagation through the entry maps
 * and the network: dL/do0 = dL/dG[c, c] G[c, c], dL/do_(1+a) =
 * dL/dG[c, c - e_a] d_c.  Leaves the network's factor set in the context.
 * *loss (may be NULL) receives L.  STS_BREAKDOWN if the factor has a
 * non-finite entry.  */
sts_status cnn_pc_grad(sts_cnn *net, const double *T, double dt, const double *z, float *grad,
                       double *loss);
/* cnn_pc_train_step - one Adam step (constants of cnn_set_adam, rate lr) on
 * the factor's objective for the probe vector z (device FP64, drawn by the
 * caller): L = ||G^T A G z - z||^2 / N at the context's operator and dt
 * (see sts_pc_objective), with the gradient of cnn_pc_grad.  Leaves the
 * step's factor (before the update) set in the context.  *loss (may be
 * NULL) receives L before the step.  STS_BREAKDOWN if the factor has a
 * non-finite entry (no update).  */
sts_status cnn_pc_train_step(sts_cnn *net, const double *T, double dt, const double *z, float lr,
                             double *loss);

#ifdef __cplusplus
}
#endif
#endif /* STS_H */
