// Internal declarations shared by the host plan code and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/fr.h"

namespace fr {

constexpr int NV = 13;   // P, V(3), grad V (9)
constexpr int NTR = 7;   // face trace values: P, V(3), (S n_hat)(3)
constexpr int PMAX = 6;

// Geometry and physics constants handed to every kernel by value.
template <typename T>
struct Consts {
    T nvec[3][3];  // n_d = det(J) J^{-T} e_d  (row d)
    T nmag[3];     // |n_d|
    T nhat[3][3];  // n_d / |n_d|
    T inv_det;     // 1 / det(J)
    T zeta, nu, invT;
    int diag;      // 1 when J is diagonal: n_hat_d = e_d exactly
};

// Operator block in device memory, precision T, for order p (m = p + 1):
//   Dt[m][m]  partially corrected divergence operator
//   gl[m], gr[m]  correction function derivatives at the points
//   lm[m], lp[m]  Lagrange basis at xi = -1, +1
template <int M>
struct OpsLayout {
    static constexpr int Dt = 0, gl = M * M, gr = M * M + M, lm = M * M + 2 * M,
                         lp = M * M + 3 * M, size = M * M + 4 * M;
};

struct Scratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// One captured HIP graph and the launch parameters it was captured with.
struct GraphCache {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t key[20] = {};
};

// One classical RK4 stage of dU/dtau = k* applied to a residual k as it is
// produced (the fused kernel's epilogue), with k* = k - [v in V] (a s + B)
// when B is set (dual time stepping, velocity only), s the state that produced
// k in double:
//   first stage: acc = U + b k*,  else acc += b k*;  s' = U + cnext k*
//   last stage:  U = acc + b k*
// s' goes to s_out (plan precision) and, when set, s_out64 (double); on the
// last stage s_out (when set) receives (T) U.  partial (when set) receives one
// sum of (k*_V)^2 per workgroup.  Every index is read and written by one
// thread only, so s_in may equal s_out64; s_out must not be the residual
// kernel's input.
struct StageSpec {
    double *U;
    double *acc;
    const double *s_in;   // state that produced k (null: U)
    double *s_out64;
    void *s_out;
    const double *B;      // BDF constant [ne][3][m^3], or null
    double *partial;
    double a, b, cnext;
    int first, last;
    // face traces: tr_in non-null holds those of the input state (written by
    // the previous stage's epilogue), so the trace kernel is skipped; tr_out
    // non-null receives those of the state this stage produces (s', or U on
    // the last stage), in the working precision, as the trace kernel would
    // compute them from that state.  nx, ny, nz: the lattice (for tr_out).
    const void *tr_in;
    void *tr_out;
    int nx, ny, nz;
};

// capacity of the per-workgroup partial sums of a fused stage launch
constexpr int MAX_PARTIALS = 8192;

struct ProfRec {
    int kid;
    hipEvent_t a, b;
};

}  // namespace fr

struct fr_plan {
    int p, m, nx, ny, nz;
    int64_t ne;
    double zeta, nu, T;
    double J[9], Jinv[9], detJ;
    int precision;  // FR_F64 / FR_F32
    int variant;    // FR_FUSED / FR_UNFUSED
    int block;      // elements per workgroup override (0 = default)
    int form = 0;   // FR_OPT_FORM: FR_FORM_AUTO / _POINT / _LINES / _HALO (fused path)
    int guess_base = 2;  // extrapolation order the learned guess corrects
    // captured time-integration graphs ([0] pseudo-step with norm read-back,
    // [1] pseudo-step without, [2] RK4 step) and their capture stream
    int use_graphs = 0;
    // fused path: apply the RK stage updates in the fused kernel's epilogue
    int fuse_stage = 1;
    // pseudo-time scheme of the dual step: 0 RK4 with a fixed step, 1 RK34 with
    // locally adaptive steps (field and error estimate in rk34, initial step
    // rk34_h0 of the field held there)
    int pseudo = 0;
    double rk34_h0 = 0.0;
    fr::Scratch rk34;
    hipStream_t cap_stream = nullptr;
    fr::GraphCache graphs[3];
    // persistent grid sizes of the fused path on this plan's device, per
    // (order, precision, diagonal Jacobian): [0] trace kernel, [1] fused kernel,
    // [2] fused kernel with the stage epilogue, [3] its matrix-core form
    int fused_grid[4][fr::PMAX + 1][2][2] = {};
    // 1 once the LDS limit of the line-form kernels is set on this plan's
    // device, per (kernel: 0 residual, 1 traces; order; precision)
    int lines_attr[2][fr::PMAX + 1][2] = {};
    // 1 once the LDS limit of the unfused stage-1 kernel is set (order, precision)
    int unfused_attr[fr::PMAX + 1][2] = {};
    int device;
    // host copies of the operators (double)
    double x[8], w[8], D[64], lm[8], lp[8], gl[8], gr[8], Dt[64];
    // device operator blocks
    void *ops64 = nullptr, *ops32 = nullptr;
    fr::Consts<double> c64;
    fr::Consts<float> c32;
    // scratch
    fr::Scratch traces;     // [6][ne][7][m^2] of the working precision
    fr::Scratch traces2;    // second trace array: the stage epilogue's ping-pong
    fr::Scratch unfused;    // stage buffers of the unfused pipeline
    fr::Scratch rk;         // acc (double), stage (T), k (T)
    fr::Scratch dual;       // BDF constant part (double, velocity only)
    fr::Scratch norm;       // partial sums (double)
    fr::Scratch mlp;        // MLP gradient partials / moments
    fr::Scratch diag;       // partial sums of the flow diagnostics
    fr::Scratch guess;      // the fallback extrapolation of the checked learned guess (double)
    double *norm_host = nullptr;  // pinned host word for the norm read-back
    // optional per-kernel event timing
    int profile = 0;
    std::vector<fr::ProfRec> prof;
    double prof_ms[FR_K_COUNT] = {};
    int64_t prof_n[FR_K_COUNT] = {};
};

namespace fr {

// error helpers (host)
int set_error(int code, const char *fmt, ...);
int check_hip(hipError_t e, const char *what);
int ensure_scratch(Scratch &s, size_t bytes);
void free_scratch(Scratch &s);

// Brackets one kernel launch with HIP events when the plan profiles.
struct ProfScope {
    fr_plan *pl;
    int kid;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(fr_plan *p, int k, hipStream_t st);
    ~ProfScope();
};
void prof_harvest(fr_plan *pl);
void graphs_reset(fr_plan *pl);

// launchers (return FR_OK or an error code)
int launch_residual_fused(fr_plan *pl, const void *U, void *R, hipStream_t s);
int launch_residual_unfused(fr_plan *pl, const void *U, void *R, hipStream_t s);
int launch_residual_mfma(fr_plan *pl, const void *U, void *R, hipStream_t s);
// the fused (or matrix-core) residual with its face traces in the library's
// fixed per-device array; no allocation.  scratch_setup looks that array's
// address up on device dev (once per device, with dev current).
int launch_residual_noalloc(fr_plan *pl, const void *U, void *R, hipStream_t s);
int scratch_setup(int dev);
// the residual of the plan's variant (fused, unfused or matrix-core)
int launch_residual(fr_plan *pl, const void *U, void *R, hipStream_t s);
// fused residual of U followed by the stage update sp (no residual array);
// *nparts receives the number of partial sums written when sp.partial is set
int launch_residual_stage(fr_plan *pl, const void *U, const StageSpec &sp, int *nparts,
                          hipStream_t s);
// How fr_rk_step / fr_dual_step apply the RK stage update for this plan's
// current settings (FR_STAGE_SEPARATE, FR_STAGE_POINT or FR_STAGE_HALO).
int stage_path(const fr_plan *pl);
// Partial norm sums the stage-epilogue launch of this plan writes at most (the
// halo form's: one per batch; 0 for the other paths).
int stage_partials(const fr_plan *pl);
// kernel form fr_residual runs on this plan (FR_FORM_POINT or FR_FORM_LINES;
// 0 for the unfused and matrix-core variants)
int residual_form(const fr_plan *pl);
// the two trace arrays of the stage epilogue's ping-pong (allocated on first use)
int stage_trace_buffers(fr_plan *pl, void *&a, void *&b);


// Up to max_iters classical RK4 pseudo-steps of dU/dtau = R(U) - M_V (a U + B)
// + D (D may be null) on plan pl, from U (double, in place).  The RMS of the
// velocity part of the first-stage residual is read back (one host wait) for
// iterates 0, check_every, 2 check_every, ... and max_iters (check_every > 0),
// or only for iterate max_iters when check_every == 0 and norm_last; the loop
// stops early once a read norm is below tol (*converged = 1).  *iters counts
// completed pseudo-steps, *resid is the last norm read (NaN if none).
int pseudo_iterate(fr_plan *pl, double *U, const double *B, double a, const double *D,
                   double dtau, double tol, int max_iters, int check_every, bool norm_last,
                   int *iters, double *resid, int *converged, hipStream_t s);

// time integration kernels (timeint.hip)
int stage_blocks(int64_t n);
int launch_stage(fr_plan *pl, bool bdf, bool norm, double *U, double *acc, double *st64,
                 void *stT, const void *k, const double *B, double a, double b, double cnext,
                 int first, int last, double *partial, hipStream_t s, const double *D = nullptr);
int launch_stage34(fr_plan *pl, int stage, double *U, double *acc, double *err, double *h,
                   double *st64, void *stT, const void *k, const double *B, const double *D,
                   double a, double atol, double h0, double *partial, hipStream_t s);
int launch_fill(double *x, double v, int64_t n, hipStream_t s);
int launch_to_precision(fr_plan *pl, const double *U, void *out, int64_t n, hipStream_t s);
int launch_bdf_const(fr_plan *pl, const double *Un, const double *Unm1, double dt, double *B,
                     hipStream_t s);
int launch_final_sum(const double *partial, int nblocks, double *out, hipStream_t s);
int launch_extrap(const double *Un, const double *Unm1, const double *Unm2, int order,
                  int keep_ns, double *G, int64_t n, hipStream_t s);

}  // namespace fr
