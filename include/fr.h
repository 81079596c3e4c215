/*
 * fr.h -- C ABI of the MI355X (gfx950) flux-reconstruction residual library
 * for the artificial compressibility method with hyperbolised diffusion
 * (ACM-HD) on constant-Jacobian tensor-product hexahedra.
 *
 * Method: Trojak, Watson, Witherden, "Hyperbolic Diffusion in Flux
 * Reconstruction: Optimisation through Kernel Fusion within Tensor-Product
 * Elements", arXiv:2107.14027.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State layout ("element-major SoA"): one state array holds
 *     ne * 13 * m^3 scalars,  m = p + 1,  ne = nx * ny * nz,
 * indexed U[e][v][k][j][i] with i (the xi_1 point index) fastest and
 * e = ex + nx * (ey + ny * ez).  Variables v, in order:
 *     P, u, v, w, q_x, q_y, q_z, r_x, r_y, r_z, s_x, s_y, s_z
 * where q = grad u, r = grad v, s = grad w (the auxiliary variables of the
 * hyperbolised diffusion, paper Sec. 2.2, eq. acmhd_nd).  Solution points are
 * the Gauss-Legendre points of each element.  The lattice is periodic in all
 * three directions; element (ex, ey, ez) is the image of the reference cube
 * [-1, 1]^3 under x = J (xi + 1 + 2 (ex, ey, ez)) with one constant Jacobian J.
 *
 * Pointers named U, R, G, Un, ... are DEVICE pointers, owned by the caller,
 * contiguous, at least 16-byte aligned (256 recommended).  Arrays of the
 * plan's working precision are float or double as selected with
 * FR_OPT_PRECISION; arrays typed double are always double.  Every call
 * enqueues its work on the caller's stream `s` (NULL = the null stream) and
 * returns without synchronising, except where stated.  A plan may be used by
 * one stream at a time: calls that overlap on one plan race on its scratch.
 * No call throws across the ABI; failures return a negative fr_status and
 * fr_last_error() (per thread) describes the last one.
 */
#ifndef FR_H
#define FR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ABI-compatible with hipStream_t. */
typedef struct ihipStream_t *fr_stream_t;
typedef struct fr_plan fr_plan;

typedef enum fr_status {
    FR_OK = 0,
    FR_EINVAL = -1,       /* bad argument (NULL, out of range, misaligned)           */
    FR_ENOMEM = -2,       /* device or host allocation failed                        */
    FR_EHIP = -3,         /* a HIP runtime call or kernel launch failed              */
    FR_ENONFINITE = -4,   /* a residual norm became NaN or Inf                        */
    FR_ENOCONV = -5,      /* pseudo-time iteration hit max_iters before the tolerance */
    FR_EUNSUPPORTED = -6  /* option not available for this order / precision          */
} fr_status;

typedef enum fr_option {
    FR_OPT_PRECISION = 1, /* FR_F64 (default) or FR_F32: working precision of the residual */
    FR_OPT_VARIANT = 2,   /* FR_FUSED (default), FR_UNFUSED or FR_MFMA (see fr_residual)   */
    FR_OPT_BLOCK = 3,     /* elements per workgroup of the fused kernel; 0 = tuned default  */
    FR_OPT_PROFILE = 4,   /* 1: record HIP events around every kernel launch (see below)   */
    FR_OPT_GUESS_BASE = 5,/* extrapolation the learned guess corrects: 2 quadratic (default),
                             1 linear                                                      */
    FR_OPT_GRAPH = 6,     /* 1: fr_rk_step and fr_dual_step replay one captured HIP graph per
                             (pseudo-)step instead of launching every kernel; 0 (default):
                             plain launches.  Results are identical either way; the graphs
                             are captured on a stream the plan owns and re-captured when a
                             pointer or scalar baked into them changes.                     */
    FR_OPT_FUSE_STAGE = 7,/* 1 (default): with FR_FUSED, fr_rk_step and fr_dual_step apply each
                             RK4 stage update (and the BDF source and the pseudo-residual
                             norm) in the fused kernel's epilogue, so the residual never goes
                             to memory (not available at p = 6 with a non-diagonal Jacobian,
                             which keeps the separate kernel); 0: residual kernel + separate
                             stage kernel.  The epilogue runs in the residual's own kernel
                             for the point and halo forms (FR_INFO_RESIDUAL_FORM), and then
                             the states are bitwise identical either way; with the line form
                             it runs in the point form's kernel (equal to rounding).  The
                             norm's summation order (per workgroup) differs.                 */
    FR_OPT_PSEUDO = 8,    /* pseudo-time scheme of fr_dual_step and of every fr_pmg level:
                             0 (default) classical RK4 with the fixed step dtau; 1 the RK34
                             embedded pair (Sec. 5; coefficients of Kennedy, Carpenter and
                             Lewis's RK3(2)4[2R+]C) with one pseudo-step per state value,
                             scaled after each step by clamp(0.8 (|e|/tol)^(-1/3), 0.98, 1.01)
                             (e the embedded error estimate, tol the call's tolerance) and
                             kept within [dtau/3, 3 dtau].  The step field persists in the
                             plan between calls with the same dtau.                           */
    FR_OPT_FORM = 9       /* kernel form of the FR_FUSED residual: FR_FORM_POINT a trace
                             kernel, then the batch staged in LDS with the transformed
                             fluxes, every point contracting its own lines; FR_FORM_LINES
                             (diagonal Jacobians only, FR_EUNSUPPORTED otherwise) a trace
                             kernel, then the batch staged in LDS and one lane per element
                             line and direction computing the flux, its own traces, the
                             common fluxes and the six corrected line derivatives in
                             registers; FR_FORM_HALO (diagonal Jacobians only) the line form
                             without a trace kernel: each lane forms the neighbours' traces
                             from their states (the batch's tile, else global memory) with
                             the trace kernel's arithmetic, so its results are bitwise those
                             of FR_FORM_LINES; FR_FORM_AUTO (default) the fastest measured:
                             the halo form with a diagonal Jacobian, else the point form.
                             The point and line forms agree to rounding (not bitwise); the
                             stage epilogue of fr_rk_step /
                             fr_dual_step uses the halo form's kernel when that is the
                             residual's form, else the point form's.                       */
} fr_option;

/* Kernel identifiers for fr_plan_kernel_stats. */
typedef enum fr_kernel {
    FR_K_TRACE = 0,       /* fused path: face-trace projection (stage 1)                  */
    FR_K_FUSED = 1,       /* fused path: stages 2-6                                       */
    FR_K_U_PROJECT = 2,   /* unfused path, Table 1 stage 1                                */
    FR_K_U_FLUX = 3,      /* stage 2                                                      */
    FR_K_U_DIV = 4,       /* stage 3                                                      */
    FR_K_U_COMMON = 5,    /* stage 4                                                      */
    FR_K_U_CORRECT = 6,   /* stage 5                                                      */
    FR_K_U_NEGSRC = 7,    /* stage 6                                                      */
    FR_K_STAGE = 8,       /* RK stage update (time integrators)                           */
    FR_K_COUNT = 9
} fr_kernel;

enum { FR_F64 = 0, FR_F32 = 1 };
enum { FR_FUSED = 0, FR_UNFUSED = 1, FR_MFMA = 2 };
enum { FR_FORM_AUTO = 0, FR_FORM_POINT = 1, FR_FORM_LINES = 2, FR_FORM_HALO = 3 };

/*
 * fr_plan_create -- build the 1D operators (Sec. 2.1: Gauss-Legendre solution
 * points, Lagrange derivative matrix, DG correction functions, and the
 * partially corrected divergence operator of Sec. 3 / Table 1 stage 3) and
 * the constant geometry for a periodic nx*ny*nz lattice of order-p hexahedra.
 *   p          polynomial order, 1..6
 *   nx,ny,nz   lattice size, each >= 1 (1 means the element is its own neighbour)
 *   jac        constant dx/dxi, row-major 3x3 with det > 0; NULL selects the
 *              periodic box [0, 2 pi]^3, i.e. J = diag(pi/nx, pi/ny, pi/nz)
 *   acm_zeta   artificial compressibility parameter zeta > 0 (Sec. 2.2)
 *   hd_relax   {nu, T}: kinematic viscosity nu >= 0 and relaxation time T > 0 of
 *              the hyperbolised diffusion (Sec. 2.2, eq. acmhd_nd)
 * Host memory is allocated; device memory for operators is allocated on the
 * current HIP device, scratch buffers lazily on first use.
 * Returns NULL on error (fr_last_error() says why).  Thread-safe.
 */
fr_plan *fr_plan_create(int p, int nx, int ny, int nz, const double jac[9], double acm_zeta,
                        const double hd_relax[2]);

/* Set / read an fr_option.  Changing the precision or variant frees scratch
 * that no longer applies.  FR_EINVAL for an unknown key or value. */
int fr_plan_set_int(fr_plan *plan, int key, int value);
int fr_plan_get_int(const fr_plan *plan, int key, int *value);
/* Read-only keys of fr_plan_get_int, for the plan's current settings:
 *   FR_INFO_RESIDUAL_FORM  the kernel form fr_residual runs (FR_FORM_POINT,
 *                          FR_FORM_LINES or FR_FORM_HALO; 0 for FR_UNFUSED and
 *                          FR_MFMA)
 *   FR_INFO_STAGE_PATH     how fr_rk_step and fr_dual_step (RK4 pseudo-steps)
 *                          apply each stage update: FR_STAGE_SEPARATE (residual
 *                          kernels, then the separate stage kernel),
 *                          FR_STAGE_POINT (the point form's kernel with the
 *                          epilogue), FR_STAGE_HALO (the halo form's kernel with
 *                          the epilogue).  Explicit FR_OPT_FORM = FR_FORM_POINT or
 *                          FR_FORM_HALO selects that form's epilogue;
 *                          FR_FORM_AUTO takes the fastest measured per order and
 *                          precision; FR_OPT_FUSE_STAGE = 0 the separate kernel. */
enum { FR_INFO_RESIDUAL_FORM = 100, FR_INFO_STAGE_PATH = 101 };
enum { FR_STAGE_SEPARATE = 0, FR_STAGE_POINT = 1, FR_STAGE_HALO = 2 };

/* Release the plan and all device memory it owns (waits for the device). */
void fr_plan_destroy(fr_plan *plan);

/* Number of scalars in one state array, ne * 13 * (p+1)^3. */
size_t fr_state_len(const fr_plan *plan);

/*
 * fr_residual -- R = -div F + S(U), the FR right-hand side of ACM-HD
 * (Table 1, stages 1-6; dU/dtau = R).  U and R are state arrays of the plan's
 * precision, must not overlap.  Interface fluxes: Rusanov on (P, V), mean of
 * the two normal fluxes for the auxiliary variables (Sec. 5).
 * FR_FUSED runs two kernels: a face-trace projection (stage 1) and one fused
 * kernel for stages 2-6 (flux, partially corrected divergence, common flux,
 * correction, source); FR_UNFUSED runs the six stages as six kernels through
 * HBM, as in Table 1.  FR_MFMA is FR_FUSED with the partially corrected
 * divergence and the correction (Table 1 stages 3 and 5; Sec. 4 treats the
 * operator application as a small matrix multiplication) applied on the
 * matrix cores: per direction, the m x (m + 2) block [Dt | g_L' | g_R']
 * multiplies, for a batch of 16 element lines at a time, each line's m values
 * followed by its two common interface values, in single-precision operands
 * with single-precision accumulation (v_mfma_f32_16x16x4f32).  It requires
 * FR_F32 (FR_EUNSUPPORTED in FR_F64); fr_rk_step and fr_dual_step then use the
 * separate stage kernel.  Allocates the plan's trace scratch on first use.
 */
int fr_residual(fr_plan *plan, const void *U, void *R, fr_stream_t s);

/*
 * fr_residual_noalloc -- fr_residual for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and kernels as fr_residual in the
 * FR_FUSED or FR_MFMA variant, but the face traces go to a fixed array of
 * 64 MiB that the library holds on every device it runs on (until the process
 * ends) instead of the plan's scratch; it calls no allocating routine.
 * Limit: 6 * ne * ceil16(7 (p+1)^2) values of the plan's precision must fit in
 * 64 MiB (at p = 3: 12,483 elements in FP64, 24,966 in FP32); larger plans get
 * FR_EINVAL before any work is enqueued, FR_UNFUSED gets FR_EUNSUPPORTED.  The
 * halo form (FR_OPT_FORM) uses no trace array, so it has no limit.  All
 * calls on one device share the array, so calls that overlap in time on one
 * device (two streams, two threads) race; calls ordered on one stream do not.
 * Nothing in the array needs clearing: every call writes each trace it reads.
 */
int fr_residual_noalloc(fr_plan *plan, const void *U, void *R, fr_stream_t s);

/*
 * fr_rk_step -- nsteps classical fourth-order Runge-Kutta steps of size dt of
 * dU/dtau = R(U) on all 13 variables.  U is a double state array updated in
 * place; the stage accumulators are double; in FR_F32 precision each stage
 * state is rounded to float for the residual.  Allocates scratch (three state
 * arrays) on first use.
 */
int fr_rk_step(fr_plan *plan, double *U, double dt, int nsteps, fr_stream_t s);

/*
 * fr_dual_step -- one physical time step by dual time stepping (Sec. 5):
 * pseudo-time RK4 steps of size dtau on dU/dtau = R*(U) with the BDF physical
 * source on the velocity only (Sec. 2.2 time-derivative masks):
 *     R*(U) = R(U) - M_V (3U - 4Un + Unm1) / (2 dt)     (Unm1 != NULL, BDF2)
 *     R*(U) = R(U) - M_V (U - Un) / dt                  (Unm1 == NULL, BDF1)
 * until the root mean square over all points of the three velocity
 * components of R* falls below tol, tested on the first-stage residual of each
 * pseudo-step (every `check_every` steps; 1 = every step).  The BDF terms and
 * the norm are evaluated in double in either precision.
 *   U       in: initial guess, out: last iterate (double state array)
 *   iters   out: completed pseudo-steps;  resid: out: last norm computed
 * Synchronises the stream at every convergence check (the norm is read back).
 * Returns FR_OK, FR_ENOCONV (max_iters reached, U holds the last iterate) or
 * FR_ENONFINITE.
 */
int fr_dual_step(fr_plan *plan, double *U, const double *Un, const double *Unm1, double dt,
                 double dtau, double tol, int max_iters, int check_every, int *iters,
                 double *resid, fr_stream_t s);

/*
 * P-multigrid dual time stepping (Sec. 5: the pseudo-iterations are accelerated
 * by a P-multigrid cycle of (order, pseudo-steps), the pseudo-step growing by a
 * constant factor per level below the finest; the paper's cycle for order 4 is
 * [(4,1), (3,1), (2,1), (1,4), (2,1), (3,1), (4,7)] with a factor of 1.75).
 * Full-approximation scheme: level l solves dU/dtau = R*_l(U) + d_l, with R*_l
 * the pseudo-residual of fr_dual_step on order l whose BDF constant is the
 * restriction of the finest level's, and d_l = 0 on the finest level;
 *   going down from order h to l = h - 1:  r_h = R*_h(U_h) + d_h,
 *     U_l = I U_h (kept as U_l^0),  d_l = I r_h - R*_l(U_l);
 *   going up from l to h:  U_h += P (U_l - U_l^0);
 * I is the L2 projection onto degree l per direction, P the interpolation of
 * the coarse polynomial at the fine points (tensor products per element).
 * Every level takes classical RK4 pseudo-steps of dtau * factor^(P - l).
 *
 * fr_pmg_create -- a cycle for the plan `fine` (borrowed: it must outlive the
 * returned object).  orders/steps hold nlevels entries; the cycle starts and
 * ends on the fine plan's order and consecutive orders differ by one.  With
 * nlevels = 0 and both arrays NULL the paper's cycle shape is used for the
 * fine plan's order P: one pseudo-step per order going down, four on order 1,
 * one per order going up, seven on order P.  factor > 0.  Creates one plan per
 * coarser order and allocates their state arrays on the current device.
 * Returns NULL on error (fr_last_error() says why).
 */
typedef struct fr_pmg fr_pmg;
fr_pmg *fr_pmg_create(fr_plan *fine, int nlevels, const int *orders, const int *steps,
                      double factor);

/*
 * fr_pmg_dual_step -- one physical time step (BDF2, or BDF1 when Unm1 is NULL)
 * by P-multigrid cycles.  Convergence (RMS over all points of the velocity
 * part of the finest level's R* below tol) is tested before the first cycle
 * and after each cycle.  The coarse plans take the fine plan's precision,
 * variant, stage-fusion, pseudo-time-scheme and graph settings.  Arguments as fr_dual_step; cycles: out,
 * completed cycles.  Synchronises the stream once per cycle.  Returns FR_OK,
 * FR_ENOCONV (max_cycles completed, U holds the last iterate) or
 * FR_ENONFINITE.
 */
int fr_pmg_dual_step(fr_pmg *mg, double *U, const double *Un, const double *Unm1, double dt,
                     double dtau, double tol, int max_cycles, int *cycles, double *resid,
                     fr_stream_t s);

/* Release the coarse plans and arrays (waits for the device). */
void fr_pmg_destroy(fr_pmg *mg);

/*
 * Standard ACM with LDG viscous fluxes -- the system the paper compares ACM-HD
 * against (Sec. 2.2, eq. acm_2d in three dimensions; Sec. 5): unknowns
 * (P, u, v, w), dU/dtau + div F = 0 with
 *   F_j = [zeta u_j ; u_i u_j + P delta_ij - nu du_i/dx_j].
 * The viscous term takes the FR route for second-order systems (Sec. 2.1):
 * a corrected velocity gradient with a common solution at the interfaces,
 * then the FR divergence.  Interfaces: Rusanov on the inviscid part (the
 * ACM-HD wave speed), LDG on the viscous part, with L the element on the
 * minus side of a face, R the plus side and n the unit normal along +xi_d:
 *   u^I   = (u_L + u_R)/2 + beta (u_L - u_R)
 *   F_v^I = (F_vL + F_vR).n/2 - beta (F_vL - F_vR).n + tau (u_L - u_R)  (velocity only)
 * The paper's runs use beta = 0.5, tau = 0.1.  The geometry, order, zeta and
 * nu come from the plan (its precision, variant and T are not used: this path
 * is double precision only).  States are U[e][4][m^3] (P, u, v, w), the same
 * element and point order as the ACM-HD state.
 *
 * fr_acm_create -- bind beta and tau (finite, tau >= 0) to the plan (borrowed:
 * it must outlive the object) and allocate the intermediates on the current
 * device: face traces (24 m^2 doubles per element), the gradient (9 m^3) and
 * the common fluxes (12 m^2).  Returns NULL on error (fr_last_error() says why).
 */
typedef struct fr_acm fr_acm;
fr_acm *fr_acm_create(fr_plan *plan, double ldg_beta, double ldg_tau);

/*
 * fr_acm_residual -- R = -div F of the device state U, both [ne][4][m^3]
 * double, 8-byte aligned, R not aliasing U.  Asynchronous on stream s; calls
 * that overlap on one object share its intermediates and race.  Returns
 * FR_EINVAL on bad arguments, else FR_OK or a launch error.
 */
int fr_acm_residual(fr_acm *a, const double *U, double *R, fr_stream_t s);

/*
 * fr_acm_gradient -- the corrected velocity gradient of U:
 * Q[e][3 i + j][m^3] = du_i/dx_j (device, double).  Same rules as
 * fr_acm_residual.
 */
int fr_acm_gradient(fr_acm *a, const double *U, double *Q, fr_stream_t s);

/*
 * fr_acm_dual_step -- one physical time step of this system by dual time
 * stepping (Sec. 5): classical RK4 pseudo-steps of size dtau on
 * dU/dtau = R*(U), with the BDF source on the velocity only,
 *     R*(U) = R(U) - M_V (3U - 4Un + Unm1) / (2 dt)    (Unm1 != NULL, BDF2)
 *     R*(U) = R(U) - M_V (U - Un) / dt                 (Unm1 == NULL, BDF1)
 * until the root mean square over all points of the velocity part of R*
 * falls below tol, tested on the first-stage residual of a pseudo-step every
 * check_every steps (and when max_iters is reached).  U: in the initial
 * guess, out the last iterate; iters, resid: out, completed pseudo-steps and
 * the last norm computed.  Device states as fr_acm_residual; U may alias
 * neither Un nor Unm1.  Allocates four more state-sized arrays and a pinned
 * host word on first use; synchronises the stream at every check.  Returns
 * FR_OK, FR_ENOCONV (U holds the last iterate), FR_ENONFINITE or FR_EINVAL.
 */
int fr_acm_dual_step(fr_acm *a, double *U, const double *Un, const double *Unm1, double dt,
                     double dtau, double tol, int max_iters, int check_every, int *iters,
                     double *resid, fr_stream_t s);

/* Release the intermediates (waits for the device). */
void fr_acm_destroy(fr_acm *a);

/*
 * Linear hexahedra: the ACM-HD residual (as fr_residual, double precision) on
 * elements whose Jacobian varies inside the element, which the paper leaves
 * as future work, noting that linear elements need only their corners
 * (Sec. 6).  Element e is the trilinear image of [-1, 1]^3 with corners
 * corners[e][c][0..2], c = c0 + 2 c1 + 4 c2 (c_d = 0 at xi_d = -1); the
 * metric rows S_d = det J J^{-T} e_d and det J are evaluated from the corners
 * wherever they are needed (nothing per point is stored).  Elements keep the
 * plan's lattice connectivity (neighbours along +-xi_d, periodic) and must be
 * conforming: the plus face of an element and the minus face of its
 * neighbour are the same quadrilateral (a periodic shift of it is allowed:
 * only tangents enter).  The common flux on a face is evaluated once, with
 * the minus-side element's metric.  det J must be positive at every solution
 * point (not checked).  With affine corners the result is fr_residual's.
 *
 * fr_lhex_create -- bind to the plan (borrowed; its order, lattice, zeta, nu
 * and T are used, its Jacobian, precision and variant are not) and allocate
 * the face traces (42 m^2 doubles per element) and common fluxes (39 m^2) on
 * the current device.  Returns NULL on error.
 */
typedef struct fr_lhex fr_lhex;
fr_lhex *fr_lhex_create(fr_plan *plan);

/*
 * fr_lhex_residual -- R = -div F + S(U) of the device state U[ne][13][m^3]
 * (double) on the elements described by the device array corners[ne][8][3]
 * (double).  8-byte aligned; R may not alias U.  Asynchronous on s; calls
 * that overlap on one object race on its intermediates.
 */
int fr_lhex_residual(fr_lhex *h, const double *corners, const double *U, double *R, fr_stream_t s);

/* Release the intermediates (waits for the device). */
void fr_lhex_destroy(fr_lhex *h);

/*
 * fr_diagnostics -- flow diagnostics of a double state U (Sec. 5 follows the
 * Taylor-Green run through them):
 *   out[0] = kinetic energy  (1/|Omega|) int |V|^2 / 2 dx
 *   out[1] = enstrophy       (nu/|Omega|) int omega . omega dx,  omega = curl V
 * with the Gauss quadrature of the solution points (exact for the nodal
 * polynomials' squares) and omega formed from the auxiliary variables,
 * omega = (s_y - r_z, q_z - s_x, r_x - q_y).  out is host memory (2 doubles);
 * synchronises the stream.  Allocates a small scratch on first use.
 */
int fr_diagnostics(fr_plan *plan, const double *U, double *out, fr_stream_t s);

/*
 * fr_guess_extrap -- initial guess for the next physical step by polynomial
 * extrapolation in time of the past states (double state arrays):
 *   order 1: G = 2 Un - Unm1;   order 2: G = 3 Un - 3 Unm1 + Unm2.
 * With FR_GUESS_KEEP_P or-ed into order, the pressure is not extrapolated but
 * taken from Un (it has no physical time derivative; extrapolating the part of
 * it a capped pseudo-iteration left unconverged makes that part grow).
 * Unm2 may be NULL for order 1.  G may alias none of the inputs.
 */
#define FR_GUESS_KEEP_P 0x10
int fr_guess_extrap(fr_plan *plan, const double *Un, const double *Unm1, const double *Unm2,
                    int order, double *G, fr_stream_t s);

/*
 * Learned initial guess (not in the paper: the pseudo-time iteration still
 * decides the converged state, the guess only sets where it starts).
 * A pointwise network 12 -> 64 -> 64 -> 4 with tanh hidden layers predicts a
 * correction to a polynomial extrapolation E of P, u, v, w (the plan option
 * FR_OPT_GUESS_BASE: quadratic E = 3 U^n - 3 U^{n-1} + U^{n-2}, the default, or
 * linear E = 2 U^n - U^{n-1}):
 *   raw features  [U^n_c, U^n_c - U^{n-1}_c, U^n_c - 2 U^{n-1}_c + U^{n-2}_c], c = P,u,v,w
 *   x = (raw - mu) * inv_sd,   y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3
 *   G_c = E_c + y_sd_c * y_c
 * Weights are rounded to bfloat16 for the matrix-core products, which
 * accumulate in float; activations are rounded to bfloat16 between layers.
 *
 * The network lives in one caller-owned DEVICE float array ("state") of
 * fr_mlp_state_floats() entries:
 *   [0, 5252)      parameters W1[64][12], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]
 *                  (row-major, output index first)
 *   [5252, 5280)   normalisation mu[12], inv_sd[12], y_sd[4]
 *   then           Adam first and second moments, 5252 floats each
 * fr_mlp_init writes initial parameters (uniform Glorot W1, W2 from `seed`;
 * W3 = b3 = 0 so that the initial guess equals the extrapolation), identity
 * normalisation and zero moments, and synchronises the stream.
 * Training rows: X[n][12] raw features and Y[n][4] raw targets
 * (U^{n+1}_c minus its extrapolation E_c), float, device memory.
 */
size_t fr_mlp_state_floats(void);
int fr_mlp_init(float *state, uint64_t seed, fr_stream_t s);

/* Raw training rows of the points offset + k*stride (k < n, flat index over
 * (element, point)) from three past states and, if Unp1 != NULL, the step's
 * converged state (else Y = 0). */
int fr_mlp_sample(fr_plan *plan, const double *Un, const double *Unm1, const double *Unm2,
                  const double *Unp1, int64_t offset, int64_t stride, int64_t n, float *X,
                  float *Y, fr_stream_t s);

/* Sets mu, inv_sd of the features and y_sd of the targets in `state` from the
 * column moments of X, Y (deterministic reductions in double). */
int fr_mlp_fit_norm(fr_plan *plan, float *state, const float *X, const float *Y, int64_t n,
                    fr_stream_t s);

/* Network outputs y (normalised units) of raw feature rows: Yout[n][4]. */
int fr_mlp_forward(fr_plan *plan, const float *state, const float *X, int64_t n, float *Yout,
                   fr_stream_t s);

/* Gradient of L = (1/(4n)) sum (y - Y/y_sd)^2 with respect to the 5252
 * parameters into grad (device, float, parameter layout) and L into *loss
 * (device float, may be NULL).  Per-wavefront partial sums are reduced in a
 * fixed order: results are deterministic. */
int fr_mlp_grad(fr_plan *plan, const float *state, const float *X, const float *Y, int64_t n,
                float *grad, float *loss, fr_stream_t s);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1)
 * of the parameters in `state` on the rows (X, Y); *loss (device, may be NULL)
 * receives the loss before the update. */
int fr_mlp_train_step(fr_plan *plan, float *state, const float *X, const float *Y, int64_t n,
                      float lr, int step, float *loss, fr_stream_t s);

/* G (double state array) = network guess for P, u, v, w and the same
 * extrapolation E for the auxiliary variables. */
int fr_mlp_guess(fr_plan *plan, const float *state, const double *Un, const double *Unm1,
                 const double *Unm2, double *G, fr_stream_t s);

/*
 * fr_mlp_guess_checked -- the learned guess with plain extrapolation as its
 * fallback.  G receives the network's guess (as fr_mlp_guess) when its initial
 * pseudo-residual is not larger than accept_ratio times that of the
 * extrapolation the network corrects (FR_OPT_GUESS_BASE), and that
 * extrapolation otherwise (also when the network's guess is not finite).  The
 * initial pseudo-residual is the root mean square over all points of the
 * velocity part of R* = R(U) - M_V (3U - 4Un + Unm1) / (2 dt), the norm
 * fr_dual_step tests (BDF2 with the physical step dt > 0).  The pseudo-time
 * iteration that follows still decides the converged state, so the rule only
 * chooses where it starts.  norms (host, 2 doubles) receives the network's and
 * the extrapolation's initial norms, *used_network 1 or 0.  accept_ratio >= 0
 * (1: not worse).  G may alias none of the inputs.  Allocates one state array
 * of scratch on first use; synchronises the stream twice (norm read-backs).
 */
int fr_mlp_guess_checked(fr_plan *plan, const float *state, const double *Un, const double *Unm1,
                         const double *Unm2, double dt, double accept_ratio, double *G,
                         int *used_network, double norms[2], fr_stream_t s);

/*
 * fr_plan_kernel_stats -- with FR_OPT_PROFILE set, every kernel launch of the
 * plan is bracketed by two HIP events recorded on the launch stream.  This call
 * waits for the recorded events, adds their elapsed times to per-kernel totals
 * and returns the totals since the last reset: total_ms (milliseconds) and
 * launches for the kernel id `kernel` (fr_kernel).  reset != 0 clears the
 * totals after reading.  Not a compute call: it only reads back timings.
 */
int fr_plan_kernel_stats(fr_plan *plan, int kernel, double *total_ms, int64_t *launches,
                         int reset);

/* Status text, and the description of the last failure on this thread. */
const char *fr_strerror(int code);
const char *fr_last_error(void);

/*
 * fr_plan_operators -- host-only copy of the plan's double-precision 1D
 * operators for inspection (no device work).  out receives, in order:
 *   x[m], w[m]            Gauss-Legendre points and weights
 *   D[m][m]               D[i][k] = l_k'(x_i)
 *   lm[m], lp[m]          l_k(-1), l_k(+1)
 *   gl[m], gr[m]          derivatives of the left / right DG correction
 *                         functions at the points (Sec. 2.1)
 *   Dt[m][m]              partially corrected divergence operator
 *                         D - gl lm^T - gr lp^T (Table 1, stage 3)
 * i.e. m*(6 + 2m) doubles.  Returns FR_EINVAL for p outside 1..6.
 */
int fr_plan_operators(int p, double *out);

/*
 * fr_launch_shape -- host-only description of how the fused residual launches
 * its kernels for order p (1..6) and precision (FR_F64 / FR_F32); no device
 * work.  kernel = FR_K_TRACE (face-trace projection) or FR_K_FUSED (stages
 * 2-6).  out receives {elements per batch (the largest FR_OPT_BLOCK value the
 * kernel accepts), threads per workgroup, dynamic LDS bytes per workgroup}.
 * Returns FR_EINVAL for other arguments.
 */
int fr_launch_shape(int p, int precision, int kernel, int out[3]);

#ifdef __cplusplus
}
#endif

#endif /* FR_H */
