// C ABI entry points that run work on the GPU: residual, RK4 steps, dual time
// steps and the extrapolated initial guess.  Argument checking happens here;
// the kernels assume validated, in-bounds launches.
#include <cmath>
#include <cstring>

#include "fr_internal.h"

using namespace fr;

namespace {

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

inline size_t esize(const fr_plan *pl) { return pl->precision == FR_F64 ? 8 : 4; }

int check_array(const void *p, const char *name)
{
    if (!p) return set_error(FR_EINVAL, "%s is NULL", name);
    if (!aligned16(p)) return set_error(FR_EINVAL, "%s is not 16-byte aligned", name);
    return FR_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

int residual(fr_plan *pl, const void *U, void *R, hipStream_t s)
{
    return pl->variant == FR_FUSED ? launch_residual_fused(pl, U, R, s)
                                   : launch_residual_unfused(pl, U, R, s);
}

struct RkBufs {
    double *acc;
    void *stT;
    void *k;
};

int rk_buffers(fr_plan *pl, RkBufs &b)
{
    const size_t n = fr_state_len(pl);
    const size_t bytes = n * 8 + 2 * n * esize(pl);
    if (int rc = ensure_scratch(pl->rk, bytes)) return rc;
    b.acc = (double *)pl->rk.ptr;
    b.stT = (char *)pl->rk.ptr + n * 8;
    b.k = (char *)b.stT + n * esize(pl);
    return FR_OK;
}

}  // namespace

extern "C" {

int fr_residual(fr_plan *pl, const void *U, void *R, fr_stream_t s)
{
    if (!pl) return set_error(FR_EINVAL, "fr_residual: NULL plan");
    if (int rc = check_array(U, "U")) return rc;
    if (int rc = check_array(R, "R")) return rc;
    const size_t bytes = fr_state_len(pl) * esize(pl);
    if (overlap(U, bytes, R, bytes)) return set_error(FR_EINVAL, "fr_residual: U and R overlap");
    return residual(pl, U, R, (hipStream_t)s);
}

int fr_rk_step(fr_plan *pl, double *U, double dt, int nsteps, fr_stream_t sv)
{
    if (!pl) return set_error(FR_EINVAL, "fr_rk_step: NULL plan");
    if (int rc = check_array(U, "U")) return rc;
    if (nsteps < 0 || !std::isfinite(dt))
        return set_error(FR_EINVAL, "fr_rk_step: nsteps=%d dt=%g", nsteps, dt);
    if (nsteps == 0) return FR_OK;
    hipStream_t s = (hipStream_t)sv;
    RkBufs b;
    if (int rc = rk_buffers(pl, b)) return rc;
    const bool f64 = pl->precision == FR_F64;
    const int64_t n = (int64_t)fr_state_len(pl);
    double *st64 = f64 ? (double *)b.stT : nullptr;
    int rc = FR_OK;
    if (!f64) rc = launch_to_precision(pl, U, b.stT, n, s);
    const double c[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
    const double w[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
    for (int step = 0; step < nsteps && !rc; ++step) {
        for (int st = 0; st < 4 && !rc; ++st) {
            const void *in = (st == 0 && f64) ? (const void *)U : b.stT;
            rc = residual(pl, in, b.k, s);
            if (rc) break;
            const bool last = st == 3;
            rc = launch_stage(pl, false, false, U, b.acc, st64, last && f64 ? nullptr : b.stT, b.k,
                              nullptr, 0.0, w[st], last ? 0.0 : c[st + 1], st == 0, last, nullptr,
                              s);
        }
    }
    return rc;
}

int fr_dual_step(fr_plan *pl, double *U, const double *Un, const double *Unm1, double dt,
                 double dtau, double tol, int max_iters, int check_every, int *iters,
                 double *resid, fr_stream_t sv)
{
    if (!pl) return set_error(FR_EINVAL, "fr_dual_step: NULL plan");
    if (int rc = check_array(U, "U")) return rc;
    if (int rc = check_array(Un, "Un")) return rc;
    if (Unm1 && !aligned16(Unm1)) return set_error(FR_EINVAL, "Unm1 is not 16-byte aligned");
    if (!iters || !resid) return set_error(FR_EINVAL, "fr_dual_step: NULL iters/resid");
    if (!(dt > 0.0) || !(dtau > 0.0) || !(tol > 0.0) || max_iters < 0 || check_every < 1)
        return set_error(FR_EINVAL, "fr_dual_step: dt=%g dtau=%g tol=%g max_iters=%d every=%d", dt,
                         dtau, tol, max_iters, check_every);
    hipStream_t s = (hipStream_t)sv;
    const bool f64 = pl->precision == FR_F64;
    const int64_t n = (int64_t)fr_state_len(pl);
    const int ns = pl->m * pl->m * pl->m;
    RkBufs b;
    if (int rc = rk_buffers(pl, b)) return rc;
    const size_t nB = (size_t)pl->ne * 3 * ns;
    if (int rc = ensure_scratch(pl->dual, (nB + (f64 ? 0 : (size_t)n)) * sizeof(double))) return rc;
    const int nblk = stage_blocks(n);
    if (int rc = ensure_scratch(pl->norm, (size_t)(nblk + 1) * sizeof(double))) return rc;
    if (!pl->norm_host &&
        check_hip(hipHostMalloc((void **)&pl->norm_host, sizeof(double), hipHostMallocDefault),
                  "hipHostMalloc"))
        return FR_ENOMEM;
    double *B = (double *)pl->dual.ptr;
    double *st64 = f64 ? (double *)b.stT : B + nB;
    double *partial = (double *)pl->norm.ptr;
    double *sum = partial + nblk;

    int rc = launch_bdf_const(pl, Un, Unm1, dt, B, s);
    const double a = Unm1 ? 1.5 / dt : 1.0 / dt;
    if (!rc && !f64) rc = launch_to_precision(pl, U, b.stT, n, s);
    const double c[4] = {0.0, 0.5 * dtau, 0.5 * dtau, dtau};
    const double w[4] = {dtau / 6.0, dtau / 3.0, dtau / 3.0, dtau / 6.0};
    const double count = 3.0 * (double)pl->ne * ns;
    int it = 0;
    double res = NAN;
    while (!rc) {
        rc = residual(pl, f64 ? (const void *)U : b.stT, b.k, s);
        if (rc) break;
        rc = launch_stage(pl, true, true, U, b.acc, st64, b.stT, b.k, B, a, w[0], c[1], 1, 0,
                          partial, s);
        if (rc) break;
        if (it % check_every == 0 || it >= max_iters) {
            rc = launch_final_sum(partial, nblk, sum, s);
            if (!rc) rc = check_hip(hipMemcpyAsync(pl->norm_host, sum, sizeof(double),
                                                   hipMemcpyDeviceToHost, s),
                                    "hipMemcpyAsync(norm)");
            if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
            if (rc) break;
            res = std::sqrt(*pl->norm_host / count);
            if (!std::isfinite(res)) {
                rc = set_error(FR_ENONFINITE, "pseudo-residual norm is %g after %d steps", res, it);
                break;
            }
            if (res < tol) break;
        }
        if (it >= max_iters) {
            rc = set_error(FR_ENOCONV, "no convergence in %d pseudo-steps (residual %g)", it, res);
            break;
        }
        for (int st = 1; st < 4 && !rc; ++st) {
            rc = residual(pl, b.stT, b.k, s);
            if (rc) break;
            const bool last = st == 3;
            rc = launch_stage(pl, true, false, U, b.acc, st64, (last && f64) ? nullptr : b.stT,
                              b.k, B, a, w[st], last ? 0.0 : c[st + 1], 0, last, nullptr, s);
        }
        if (!rc) ++it;
    }
    *iters = it;
    *resid = res;
    return rc;
}

int fr_guess_extrap(fr_plan *pl, const double *Un, const double *Unm1, const double *Unm2,
                    int order, double *G, fr_stream_t s)
{
    if (!pl) return set_error(FR_EINVAL, "fr_guess_extrap: NULL plan");
    if (order != 1 && order != 2) return set_error(FR_EINVAL, "fr_guess_extrap: order %d", order);
    if (int rc = check_array(Un, "Un")) return rc;
    if (int rc = check_array(Unm1, "Unm1")) return rc;
    if (order == 2)
        if (int rc = check_array(Unm2, "Unm2")) return rc;
    if (int rc = check_array(G, "G")) return rc;
    const size_t bytes = fr_state_len(pl) * 8;
    if (overlap(G, bytes, Un, bytes) || overlap(G, bytes, Unm1, bytes) ||
        (order == 2 && overlap(G, bytes, Unm2, bytes)))
        return set_error(FR_EINVAL, "fr_guess_extrap: G overlaps an input");
    return launch_extrap(Un, Unm1, Unm2, order, G, (int64_t)fr_state_len(pl), (hipStream_t)s);
}

}  // extern "C"
