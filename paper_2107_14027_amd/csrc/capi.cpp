// C ABI entry points that run work on the GPU: residual, RK4 steps, dual time
// steps and the extrapolated initial guess.  Argument checking happens here;
// the kernels assume validated, in-bounds launches.
#include <algorithm>
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
    return launch_residual(pl, U, R, s);
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

bool stage_in_epilogue(const fr_plan *pl)
{
    return stage_path(pl) != FR_STAGE_SEPARATE;
}

// every plan setting that changes the launches of a step
uint64_t config_word(const fr_plan *pl)
{
    return (uint64_t)pl->precision | (uint64_t)pl->variant << 8 | (uint64_t)pl->fuse_stage << 16 |
           (uint64_t)pl->pseudo << 24 | (uint64_t)(uint32_t)pl->block << 32;
}

uint64_t bits(double x)
{
    uint64_t u;
    std::memcpy(&u, &x, sizeof u);
    return u;
}

// Launch the work that `enqueue(stream)` issues as one HIP graph on stream s.
// The graph is captured on the plan's own stream the first time and again
// whenever `key` (every pointer and scalar baked into the launches) changes;
// all scratch must already be allocated (the callers run one step without a
// graph first).
template <class F>
int graph_run(fr_plan *pl, GraphCache &gc, const uint64_t (&key)[20], hipStream_t s, F &&enqueue)
{
    if (!gc.exec || std::memcmp(gc.key, key, sizeof key) != 0) {
        for (auto &g : pl->graphs)
            if (&g == &gc) {
                if (g.exec) hipGraphExecDestroy(g.exec);
                if (g.graph) hipGraphDestroy(g.graph);
                g = GraphCache{};
            }
        if (!pl->cap_stream)
            if (int rc = check_hip(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking),
                                   "hipStreamCreateWithFlags"))
                return rc;
        if (int rc = check_hip(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal),
                               "hipStreamBeginCapture"))
            return rc;
        int rc = enqueue(pl->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(pl->cap_stream, &g);
        if (rc || e != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return rc ? rc : check_hip(e, "hipStreamEndCapture");
        }
        if (int rc2 = check_hip(hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0),
                                "hipGraphInstantiate")) {
            hipGraphDestroy(g);
            gc.exec = nullptr;
            return rc2;
        }
        gc.graph = g;
        std::memcpy(gc.key, key, sizeof key);
    }
    return check_hip(hipGraphLaunch(gc.exec, s), "hipGraphLaunch");
}

}  // namespace

namespace fr {

int launch_residual(fr_plan *pl, const void *U, void *R, hipStream_t s)
{
    switch (pl->variant) {
        case FR_FUSED: return launch_residual_fused(pl, U, R, s);
        case FR_UNFUSED: return launch_residual_unfused(pl, U, R, s);
        case FR_MFMA: return launch_residual_mfma(pl, U, R, s);
    }
    return set_error(FR_EINVAL, "variant %d", pl->variant);
}

int pseudo_iterate(fr_plan *pl, double *U, const double *B, double a, const double *D,
                   double dtau, double tol, int max_iters, int check_every, bool norm_last,
                   int *iters, double *resid, int *converged, hipStream_t s)
{
    const bool f64 = pl->precision == FR_F64;
    const int64_t n = (int64_t)fr_state_len(pl);
    const int ns = pl->m * pl->m * pl->m;
    RkBufs b;
    if (int rc = rk_buffers(pl, b)) return rc;
    const size_t nB = (size_t)pl->ne * 3 * ns;
    // the double copy of the stage state the BDF term needs (FP32) follows the
    // BDF constant's slot in the plan's dual scratch
    if (!f64)
        if (int rc = ensure_scratch(pl->dual, (nB + (size_t)n) * sizeof(double))) return rc;
    const int cap = std::max(std::max(stage_blocks(n), MAX_PARTIALS), stage_partials(pl));
    if (int rc = ensure_scratch(pl->norm, (size_t)(cap + 1) * sizeof(double))) return rc;
    if (!pl->norm_host &&
        check_hip(hipHostMalloc((void **)&pl->norm_host, sizeof(double), hipHostMallocDefault),
                  "hipHostMalloc"))
        return FR_ENOMEM;
    double *st64 = f64 ? (double *)b.stT : (double *)pl->dual.ptr + nB;
    double *partial = (double *)pl->norm.ptr;
    double *sum = partial + cap;
    int nparts = stage_blocks(n);  // partial sums the first stage writes

    int rc = FR_OK;
    if (!f64) rc = launch_to_precision(pl, U, b.stT, n, s);
    const double c[4] = {0.0, 0.5 * dtau, 0.5 * dtau, dtau};
    const double w[4] = {dtau / 6.0, dtau / 3.0, dtau / 3.0, dtau / 6.0};
    const double count = 3.0 * (double)pl->ne * ns;
    // first stage of a pseudo-step (residual of the current iterate, with the
    // per-block partial sums of its velocity norm), the other three stages,
    // and the reduction + read-back of the norm into pinned host memory.
    // With the stage updates in the fused kernel's epilogue the stage states
    // alternate between the two stage buffers, and the double copy of the stage
    // state that the BDF term needs (FP32) is updated in place.  A fixed source
    // D runs on the separate stage kernel.
    // RK34 with locally adaptive steps: the step field persists in the plan
    // while the initial step is unchanged
    const bool rk34 = pl->pseudo == 1;
    double *h34 = nullptr, *err34 = nullptr;
    if (rk34) {
        const void *before = pl->rk34.ptr;
        if (int r = ensure_scratch(pl->rk34, 2 * (size_t)n * sizeof(double))) return r;
        h34 = (double *)pl->rk34.ptr;
        err34 = h34 + n;
        if (pl->rk34.ptr != before || pl->rk34_h0 != dtau) {
            if (int r = launch_fill(h34, dtau, n, s)) return r;
            pl->rk34_h0 = dtau;
        }
    }
    const bool epi = stage_in_epilogue(pl) && !D && !rk34;
    void *const bufs[2] = {b.stT, b.k};
    const int o = f64 ? 0 : 1;
    // face traces ping-pong between two arrays: each stage's epilogue writes
    // those of the state it produces, so only the call's first stage runs the
    // trace kernel (stage 0 reads A and writes B, stages 1, 2, 3 alternate)
    // (the halo form needs none)
    void *trA = nullptr, *trB = nullptr;
    const bool epi_traces = epi && stage_path(pl) == FR_STAGE_POINT;
    if (epi_traces)
        if (int r = stage_trace_buffers(pl, trA, trB)) return r;
    auto with_traces = [&](StageSpec sp, const void *in, void *out) {
        sp.tr_in = epi_traces ? in : nullptr;
        sp.tr_out = epi_traces ? out : nullptr;
        sp.nx = pl->nx;
        sp.ny = pl->ny;
        sp.nz = pl->nz;
        return sp;
    };
    bool chained = false;  // stage 0's input traces come from the previous stage 3
    auto stage0 = [&](hipStream_t st) -> int {
        if (rk34) {
            if (int r = residual(pl, f64 ? (const void *)U : b.stT, b.k, st)) return r;
            return launch_stage34(pl, 0, U, b.acc, err34, h34, st64, b.stT, b.k, B, D, a, tol, dtau,
                                  partial, st);
        }
        if (epi) {
            const StageSpec sp = with_traces(StageSpec{U, b.acc, nullptr, f64 ? nullptr : st64,
                                                       bufs[o], B, partial, a, w[0], c[1], 1, 0},
                                             chained ? trA : nullptr, trB);
            return launch_residual_stage(pl, f64 ? (const void *)U : bufs[0], sp, &nparts, st);
        }
        if (int r = residual(pl, f64 ? (const void *)U : b.stT, b.k, st)) return r;
        return launch_stage(pl, true, true, U, b.acc, st64, b.stT, b.k, B, a, w[0], c[1], 1, 0,
                            partial, st, D);
    };
    auto stages123 = [&](hipStream_t st) -> int {
        if (rk34) {
            for (int k = 1; k < 4; ++k) {
                if (int r = residual(pl, b.stT, b.k, st)) return r;
                if (int r = launch_stage34(pl, k, U, b.acc, err34, h34, st64,
                                           (k == 3 && f64) ? nullptr : b.stT, b.k, B, D, a, tol,
                                           dtau, nullptr, st))
                    return r;
            }
            return FR_OK;
        }
        if (epi) {
            for (int k = 1; k < 4; ++k) {
                const bool last = k == 3;
                void *in = bufs[(k - 1 + o) % 2];
                void *out = last ? (f64 ? nullptr : bufs[0]) : bufs[(k + o) % 2];
                const StageSpec sp = with_traces(
                    StageSpec{U, b.acc, f64 ? (const double *)in : st64,
                              (f64 || last) ? nullptr : st64, out, B, nullptr, a, w[k],
                              last ? 0.0 : c[k + 1], 0, last},
                    k % 2 ? trB : trA, k % 2 ? trA : trB);
                if (int r = launch_residual_stage(pl, in, sp, nullptr, st)) return r;
            }
            return FR_OK;
        }
        for (int k = 1; k < 4; ++k) {
            if (int r = residual(pl, b.stT, b.k, st)) return r;
            const bool last = k == 3;
            if (int r = launch_stage(pl, true, false, U, b.acc, st64, (last && f64) ? nullptr : b.stT,
                                     b.k, B, a, w[k], last ? 0.0 : c[k + 1], 0, last, nullptr, st, D))
                return r;
        }
        return FR_OK;
    };
    auto readback = [&](hipStream_t st) -> int {
        if (int r = launch_final_sum(partial, nparts, sum, st)) return r;
        return check_hip(hipMemcpyAsync(pl->norm_host, sum, sizeof(double), hipMemcpyDeviceToHost, st),
                         "hipMemcpyAsync(norm)");
    };
    int it = 0;
    double res = NAN;
    auto wait_norm = [&]() -> int {
        if (int r = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize")) return r;
        res = std::sqrt(*pl->norm_host / count);
        if (!std::isfinite(res))
            return set_error(FR_ENONFINITE, "pseudo-residual norm is %g after %d steps", res, it);
        return FR_OK;
    };
    // is the norm of iterate j read back?
    auto checked = [&](int j) {
        return check_every > 0 ? (j % check_every == 0 || j >= max_iters)
                               : (norm_last && j >= max_iters);
    };
    // iterate `it` has had its first stage (unless it is the last and its norm
    // is not wanted); its norm is known when `have`
    bool have = checked(0);
    if (!rc && (max_iters > 0 || have)) rc = stage0(s);
    chained = true;
    if (!rc && have) rc = readback(s);
    if (!rc && have) rc = wait_norm();
    *converged = 0;
    const bool graphs = pl->use_graphs && !pl->profile;
    while (!rc) {
        if (have && res < tol) {
            *converged = 1;
            break;
        }
        if (it >= max_iters) break;
        const bool check = checked(it + 1);
        const bool next0 = it + 1 < max_iters || check;
        auto body = [&](hipStream_t st) -> int {
            if (int r = stages123(st)) return r;
            if (!next0) return FR_OK;
            if (int r = stage0(st)) return r;
            return check ? readback(st) : FR_OK;
        };
        if (graphs) {
            const uint64_t key[20] = {1, (uint64_t)U, (uint64_t)B, (uint64_t)D, bits(a), bits(dtau),
                                      (uint64_t)check | (uint64_t)next0 << 1, (uint64_t)pl->rk.ptr,
                                      (uint64_t)pl->dual.ptr, (uint64_t)pl->norm.ptr,
                                      (uint64_t)pl->traces.ptr, (uint64_t)pl->unfused.ptr,
                                      config_word(pl), (uint64_t)pl->norm_host,
                                      (uint64_t)nparts, (uint64_t)pl->rk34.ptr, bits(tol),
                                      (uint64_t)pl->traces2.ptr};
            rc = graph_run(pl, pl->graphs[check ? 0 : 1], key, s, body);
        } else {
            rc = body(s);
        }
        if (rc) break;
        ++it;
        have = check;
        if (check) rc = wait_norm();
    }
    *iters = it;
    *resid = res;
    return rc;
}

}  // namespace fr

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

int fr_residual_noalloc(fr_plan *pl, const void *U, void *R, fr_stream_t s)
{
    if (!pl) return set_error(FR_EINVAL, "fr_residual_noalloc: NULL plan");
    if (int rc = check_array(U, "U")) return rc;
    if (int rc = check_array(R, "R")) return rc;
    const size_t bytes = fr_state_len(pl) * esize(pl);
    if (overlap(U, bytes, R, bytes))
        return set_error(FR_EINVAL, "fr_residual_noalloc: U and R overlap");
    return launch_residual_noalloc(pl, U, R, (hipStream_t)s);
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
    // stage updates in the fused kernel's epilogue: the stage states alternate
    // between the two stage buffers (no residual array); the last stage leaves
    // the working-precision copy of U in the first one, as the separate path does
    const bool epi = stage_in_epilogue(pl);
    void *const bufs[2] = {b.stT, b.k};
    const int o = f64 ? 0 : 1;
    // face traces ping-pong between two arrays (stage 0 reads A, writes B;
    // stages 1, 2, 3 alternate): only the call's first stage runs the trace kernel
    // (the halo form needs none)
    void *trA = nullptr, *trB = nullptr;
    const bool epi_traces = epi && stage_path(pl) == FR_STAGE_POINT;
    if (epi_traces)
        if (int r = stage_trace_buffers(pl, trA, trB)) return r;
    bool chained = false;
    auto step = [&](hipStream_t st) -> int {
        if (epi) {
            const void *in = f64 ? (const void *)U : bufs[0];
            for (int k = 0; k < 4; ++k) {
                const bool last = k == 3;
                void *out = last ? (f64 ? nullptr : bufs[0]) : bufs[(k + o) % 2];
                StageSpec sp{U, b.acc, nullptr, nullptr, out, nullptr, nullptr,
                             0.0, w[k], last ? 0.0 : c[k + 1], k == 0, last};
                if (epi_traces) {
                    sp.tr_in = k == 0 ? (chained ? trA : nullptr) : (k % 2 ? trB : trA);
                    sp.tr_out = k % 2 ? trA : trB;
                }
                sp.nx = pl->nx;
                sp.ny = pl->ny;
                sp.nz = pl->nz;
                if (int r = launch_residual_stage(pl, in, sp, nullptr, st)) return r;
                in = out;
            }
            return FR_OK;
        }
        for (int k = 0; k < 4; ++k) {
            const void *in = (k == 0 && f64) ? (const void *)U : b.stT;
            if (int r = residual(pl, in, b.k, st)) return r;
            const bool last = k == 3;
            if (int r = launch_stage(pl, false, false, U, b.acc, st64, last && f64 ? nullptr : b.stT,
                                     b.k, nullptr, 0.0, w[k], last ? 0.0 : c[k + 1], k == 0, last,
                                     nullptr, st))
                return r;
        }
        return FR_OK;
    };
    const bool graphs = pl->use_graphs && !pl->profile;
    for (int it = 0; it < nsteps && !rc; ++it) {
        chained = it > 0;
        if (graphs && it > 0) {
            const uint64_t key[20] = {2, (uint64_t)U, bits(dt), (uint64_t)pl->rk.ptr,
                                      (uint64_t)pl->traces.ptr, (uint64_t)pl->unfused.ptr,
                                      config_word(pl), (uint64_t)pl->traces2.ptr};
            rc = graph_run(pl, pl->graphs[2], key, s, step);
        } else {
            rc = step(s);
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
    const size_t n = fr_state_len(pl);
    const size_t nB = (size_t)pl->ne * 3 * pl->m * pl->m * pl->m;
    if (int rc = ensure_scratch(pl->dual, (nB + (f64 ? 0 : n)) * sizeof(double))) return rc;
    double *B = (double *)pl->dual.ptr;
    if (int rc = launch_bdf_const(pl, Un, Unm1, dt, B, s)) return rc;
    int conv = 0;
    const int rc = pseudo_iterate(pl, U, B, Unm1 ? 1.5 / dt : 1.0 / dt, nullptr, dtau, tol,
                                  max_iters, check_every, true, iters, resid, &conv, s);
    if (rc) return rc;
    if (!conv)
        return set_error(FR_ENOCONV, "no convergence in %d pseudo-steps (residual %g)", *iters,
                         *resid);
    return FR_OK;
}

int fr_guess_extrap(fr_plan *pl, const double *Un, const double *Unm1, const double *Unm2,
                    int order, double *G, fr_stream_t s)
{
    if (!pl) return set_error(FR_EINVAL, "fr_guess_extrap: NULL plan");
    const bool keep_p = (order & FR_GUESS_KEEP_P) != 0;
    order &= ~FR_GUESS_KEEP_P;
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
    return launch_extrap(Un, Unm1, Unm2, order, keep_p ? pl->m * pl->m * pl->m : 0, G,
                         (int64_t)fr_state_len(pl), (hipStream_t)s);
}

int fr_mlp_guess_checked(fr_plan *pl, const float *state, const double *Un, const double *Unm1,
                         const double *Unm2, double dt, double accept_ratio, double *G,
                         int *used_network, double norms[2], fr_stream_t sv)
{
    if (!pl) return set_error(FR_EINVAL, "fr_mlp_guess_checked: NULL plan");
    if (int rc = check_array(Un, "Un")) return rc;
    if (int rc = check_array(Unm1, "Unm1")) return rc;
    if (int rc = check_array(Unm2, "Unm2")) return rc;
    if (int rc = check_array(G, "G")) return rc;
    if (!state || !used_network || !norms || !(dt > 0.0) || !(accept_ratio >= 0.0))
        return set_error(FR_EINVAL, "fr_mlp_guess_checked: state=%p dt=%g ratio=%g", (const void *)state,
                         dt, accept_ratio);
    const size_t n = fr_state_len(pl);
    const size_t bytes = n * 8;
    if (overlap(G, bytes, Un, bytes) || overlap(G, bytes, Unm1, bytes) ||
        overlap(G, bytes, Unm2, bytes))
        return set_error(FR_EINVAL, "fr_mlp_guess_checked: G overlaps an input");
    hipStream_t s = (hipStream_t)sv;
    const bool f64 = pl->precision == FR_F64;
    const size_t nB = (size_t)pl->ne * 3 * pl->m * pl->m * pl->m;
    if (int rc = ensure_scratch(pl->guess, bytes)) return rc;
    if (int rc = ensure_scratch(pl->dual, (nB + (f64 ? 0 : n)) * sizeof(double))) return rc;
    double *E = (double *)pl->guess.ptr;
    double *B = (double *)pl->dual.ptr;
    // the extrapolation the network corrects, and the network's guess
    if (int rc = launch_extrap(Un, Unm1, Unm2, pl->guess_base, 0, E, (int64_t)n, s)) return rc;
    if (int rc = fr_mlp_guess(pl, state, Un, Unm1, Unm2, G, sv)) return rc;
    // initial pseudo-residual RMS (velocity part of R*, BDF2) of each: the first
    // stage of a pseudo-step without completing it, so neither guess changes
    if (int rc = launch_bdf_const(pl, Un, Unm1, dt, B, s)) return rc;
    const double a = 1.5 / dt;
    int it = 0, conv = 0;
    double rn = NAN, re = NAN;
    int rc = pseudo_iterate(pl, G, B, a, nullptr, dt, 0.0, 0, 1, true, &it, &rn, &conv, s);
    if (rc && rc != FR_ENONFINITE) return rc;
    if (rc == FR_ENONFINITE) rn = INFINITY;
    rc = pseudo_iterate(pl, E, B, a, nullptr, dt, 0.0, 0, 1, true, &it, &re, &conv, s);
    if (rc) return rc;
    norms[0] = rn;
    norms[1] = re;
    *used_network = std::isfinite(rn) && rn <= accept_ratio * re;
    if (!*used_network)
        return check_hip(hipMemcpyAsync(G, E, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync(G)");
    return FR_OK;
}

}  // extern "C"
