// Host side of the library: plan construction (1D FR operators and constant
// geometry, in double precision), option handling, scratch management and
// error reporting.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "fr_internal.h"

namespace fr {

static thread_local char g_last_error[512] = "";

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return code;
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return FR_OK;
    return set_error(e == hipErrorOutOfMemory ? FR_ENOMEM : FR_EHIP, "%s: %s", what,
                     hipGetErrorString(e));
}

int ensure_scratch(Scratch &s, size_t bytes)
{
    if (s.bytes >= bytes && s.ptr) return FR_OK;
    if (s.ptr) {
        hipDeviceSynchronize();
        hipFree(s.ptr);
        s.ptr = nullptr;
        s.bytes = 0;
    }
    hipError_t e = hipMalloc(&s.ptr, bytes);
    if (e != hipSuccess) {
        s.ptr = nullptr;
        return check_hip(e, "hipMalloc(scratch)");
    }
    s.bytes = bytes;
    return FR_OK;
}

void free_scratch(Scratch &s)
{
    if (s.ptr) hipFree(s.ptr);
    s.ptr = nullptr;
    s.bytes = 0;
}

// --------------------------------------------------------------------------
// 1D operators (Sec. 2.1).  Built independently of any reference code:
//  - Gauss-Legendre points by Newton's method on P_m in long double,
//  - Lagrange derivatives and endpoint values from the barycentric forms,
//  - DG correction-function derivatives from the lifting identity on Gauss
//    points: g_R'(x_i) = l_i(1) / w_i, g_L'(x_i) = -l_i(-1) / w_i,
//  - partially corrected operator Dt = D - g_L l(-1)^T - g_R l(1)^T.
// --------------------------------------------------------------------------
struct Ops1D {
    int m;
    double x[8], w[8], D[64], lm[8], lp[8], gl[8], gr[8], Dt[64];
};

static void legendre_ld(int n, long double t, long double &P, long double &dP)
{
    long double a = 1.0L, b = t;
    for (int k = 2; k <= n; ++k) {
        long double c = ((2 * k - 1) * t * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    P = (n == 0) ? 1.0L : b;
    // P_n'(t) = n (t P_n - P_{n-1}) / (t^2 - 1); t is never +-1 for interior roots
    dP = (n == 0) ? 0.0L : n * (t * P - a) / (t * t - 1.0L);
}

static void build_ops(int p, Ops1D &o)
{
    const int m = p + 1;
    o.m = m;
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < m; ++i) {
        long double t = -cosl(pi * (4 * i + 3) / (4 * m + 2));
        long double P, dP;
        for (int it = 0; it < 60; ++it) {
            legendre_ld(m, t, P, dP);
            long double dt = P / dP;
            t -= dt;
            if (fabsl(dt) < 1e-19L) break;
        }
        legendre_ld(m, t, P, dP);
        o.x[i] = (double)t;
        o.w[i] = (double)(2.0L / ((1.0L - t * t) * dP * dP));
    }
    double lam[8];
    for (int k = 0; k < m; ++k) {
        long double s = 1.0L;
        for (int j = 0; j < m; ++j)
            if (j != k) s *= (long double)o.x[k] - o.x[j];
        lam[k] = (double)(1.0L / s);
    }
    for (int i = 0; i < m; ++i) {
        long double diag = 0.0L;
        for (int k = 0; k < m; ++k) {
            if (k == i) continue;
            long double v = ((long double)lam[k] / lam[i]) / ((long double)o.x[i] - o.x[k]);
            o.D[i * m + k] = (double)v;
            diag -= v;
        }
        o.D[i * m + i] = (double)diag;
    }
    for (int side = 0; side < 2; ++side) {
        long double t = side ? 1.0L : -1.0L, den = 0.0L;
        for (int k = 0; k < m; ++k) den += (long double)lam[k] / (t - o.x[k]);
        for (int k = 0; k < m; ++k) {
            double v = (double)(((long double)lam[k] / (t - o.x[k])) / den);
            (side ? o.lp : o.lm)[k] = v;
        }
    }
    for (int i = 0; i < m; ++i) {
        o.gr[i] = o.lp[i] / o.w[i];
        o.gl[i] = -o.lm[i] / o.w[i];
    }
    for (int i = 0; i < m; ++i)
        for (int k = 0; k < m; ++k)
            o.Dt[i * m + k] = o.D[i * m + k] - o.gl[i] * o.lm[k] - o.gr[i] * o.lp[k];
}

template <typename T>
static void fill_consts(const fr_plan *pl, Consts<T> &c)
{
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        double nv[3];
        for (int j = 0; j < 3; ++j) {
            nv[j] = pl->detJ * pl->Jinv[3 * d + j];
            s += nv[j] * nv[j];
        }
        double mag = std::sqrt(s);
        c.nmag[d] = (T)mag;
        for (int j = 0; j < 3; ++j) {
            c.nvec[d][j] = (T)nv[j];
            c.nhat[d][j] = (T)(nv[j] / mag);
        }
    }
    c.inv_det = (T)(1.0 / pl->detJ);
    const double *J = pl->J;
    c.diag = (J[1] == 0.0 && J[2] == 0.0 && J[3] == 0.0 && J[5] == 0.0 && J[6] == 0.0 &&
              J[7] == 0.0) ? 1 : 0;
    c.zeta = (T)pl->zeta;
    c.nu = (T)pl->nu;
    c.invT = (T)(1.0 / pl->T);
}

template <typename T>
static void pack_ops(const fr_plan *pl, T *buf)
{
    const int m = pl->m;
    int o = 0;
    for (int i = 0; i < m * m; ++i) buf[o++] = (T)pl->Dt[i];
    for (int i = 0; i < m; ++i) buf[o++] = (T)pl->gl[i];
    for (int i = 0; i < m; ++i) buf[o++] = (T)pl->gr[i];
    for (int i = 0; i < m; ++i) buf[o++] = (T)pl->lm[i];
    for (int i = 0; i < m; ++i) buf[o++] = (T)pl->lp[i];
}

ProfScope::ProfScope(fr_plan *p, int k, hipStream_t st) : pl(p), kid(k), s(st)
{
    if (pl && pl->profile && hipEventCreate(&a) == hipSuccess) hipEventRecord(a, s);
}

ProfScope::~ProfScope()
{
    if (!a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) {
        hipEventDestroy(a);
        return;
    }
    hipEventRecord(b, s);
    pl->prof.push_back({kid, a, b});
    if (pl->prof.size() > 8192) prof_harvest(pl);
}

void graphs_reset(fr_plan *pl)
{
    for (auto &g : pl->graphs) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        if (g.graph) hipGraphDestroy(g.graph);
        g = fr::GraphCache{};
    }
}

void prof_harvest(fr_plan *pl)
{
    for (auto &r : pl->prof) {
        float ms = 0.f;
        hipEventSynchronize(r.b);
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            pl->prof_ms[r.kid] += ms;
            pl->prof_n[r.kid] += 1;
        }
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    pl->prof.clear();
}

}  // namespace fr

using namespace fr;

extern "C" {

const char *fr_last_error(void) { return g_last_error; }

const char *fr_strerror(int code)
{
    switch (code) {
        case FR_OK: return "ok";
        case FR_EINVAL: return "invalid argument";
        case FR_ENOMEM: return "out of memory";
        case FR_EHIP: return "HIP runtime error";
        case FR_ENONFINITE: return "non-finite residual";
        case FR_ENOCONV: return "pseudo-time iteration did not converge";
        case FR_EUNSUPPORTED: return "unsupported option";
        default: return "unknown status";
    }
}

int fr_plan_operators(int p, double *out)
{
    if (p < 1 || p > PMAX || !out) return set_error(FR_EINVAL, "fr_plan_operators: p=%d", p);
    Ops1D o;
    build_ops(p, o);
    const int m = p + 1;
    double *q = out;
    for (int i = 0; i < m; ++i) *q++ = o.x[i];
    for (int i = 0; i < m; ++i) *q++ = o.w[i];
    for (int i = 0; i < m * m; ++i) *q++ = o.D[i];
    for (int i = 0; i < m; ++i) *q++ = o.lm[i];
    for (int i = 0; i < m; ++i) *q++ = o.lp[i];
    for (int i = 0; i < m; ++i) *q++ = o.gl[i];
    for (int i = 0; i < m; ++i) *q++ = o.gr[i];
    for (int i = 0; i < m * m; ++i) *q++ = o.Dt[i];
    return FR_OK;
}

fr_plan *fr_plan_create(int p, int nx, int ny, int nz, const double jac[9], double acm_zeta,
                        const double hd_relax[2])
{
    if (p < 1 || p > PMAX) {
        set_error(FR_EINVAL, "fr_plan_create: order p=%d outside 1..%d", p, PMAX);
        return nullptr;
    }
    if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz > (int64_t)1 << 31) {
        set_error(FR_EINVAL, "fr_plan_create: bad lattice %d x %d x %d", nx, ny, nz);
        return nullptr;
    }
    if (!hd_relax || !(acm_zeta > 0.0) || !(hd_relax[0] >= 0.0) || !(hd_relax[1] > 0.0) ||
        !std::isfinite(acm_zeta) || !std::isfinite(hd_relax[0]) || !std::isfinite(hd_relax[1])) {
        set_error(FR_EINVAL, "fr_plan_create: need zeta > 0, nu >= 0, T > 0");
        return nullptr;
    }
    fr_plan *pl = new (std::nothrow) fr_plan();
    if (!pl) {
        set_error(FR_ENOMEM, "fr_plan_create: host allocation");
        return nullptr;
    }
    pl->p = p;
    pl->m = p + 1;
    pl->nx = nx;
    pl->ny = ny;
    pl->nz = nz;
    pl->ne = (int64_t)nx * ny * nz;
    pl->zeta = acm_zeta;
    pl->nu = hd_relax[0];
    pl->T = hd_relax[1];
    pl->precision = FR_F64;
    pl->variant = FR_FUSED;
    pl->block = 0;
    if (jac) {
        std::memcpy(pl->J, jac, sizeof pl->J);
    } else {
        std::memset(pl->J, 0, sizeof pl->J);
        pl->J[0] = M_PI / nx;
        pl->J[4] = M_PI / ny;
        pl->J[8] = M_PI / nz;
    }
    const double *A = pl->J;
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(det > 0.0) || !std::isfinite(det)) {
        set_error(FR_EINVAL, "fr_plan_create: Jacobian determinant %g is not positive", det);
        delete pl;
        return nullptr;
    }
    pl->detJ = det;
    double *B = pl->Jinv;  // adjugate / det
    B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;

    Ops1D o;
    build_ops(p, o);
    std::memcpy(pl->x, o.x, sizeof o.x);
    std::memcpy(pl->w, o.w, sizeof o.w);
    std::memcpy(pl->D, o.D, sizeof o.D);
    std::memcpy(pl->lm, o.lm, sizeof o.lm);
    std::memcpy(pl->lp, o.lp, sizeof o.lp);
    std::memcpy(pl->gl, o.gl, sizeof o.gl);
    std::memcpy(pl->gr, o.gr, sizeof o.gr);
    std::memcpy(pl->Dt, o.Dt, sizeof o.Dt);
    fill_consts(pl, pl->c64);
    fill_consts(pl, pl->c32);

    if (check_hip(hipGetDevice(&pl->device), "hipGetDevice") || fr::scratch_setup(pl->device)) {
        delete pl;
        return nullptr;
    }
    const int nops = pl->m * pl->m + 4 * pl->m;
    double h64[128];
    float h32[128];
    pack_ops(pl, h64);
    pack_ops(pl, h32);
    if (check_hip(hipMalloc(&pl->ops64, nops * sizeof(double)), "hipMalloc(ops64)") ||
        check_hip(hipMalloc(&pl->ops32, nops * sizeof(float)), "hipMalloc(ops32)") ||
        check_hip(hipMemcpy(pl->ops64, h64, nops * sizeof(double), hipMemcpyHostToDevice),
                  "hipMemcpy(ops64)") ||
        check_hip(hipMemcpy(pl->ops32, h32, nops * sizeof(float), hipMemcpyHostToDevice),
                  "hipMemcpy(ops32)")) {
        if (pl->ops64) hipFree(pl->ops64);
        if (pl->ops32) hipFree(pl->ops32);
        delete pl;
        return nullptr;
    }
    return pl;
}

int fr_plan_set_int(fr_plan *pl, int key, int value)
{
    if (!pl) return set_error(FR_EINVAL, "fr_plan_set_int: NULL plan");
    switch (key) {
        case FR_OPT_PRECISION:
            if (value != FR_F64 && value != FR_F32)
                return set_error(FR_EINVAL, "precision %d", value);
            if (value != pl->precision) {
                hipDeviceSynchronize();
                free_scratch(pl->traces);
    free_scratch(pl->traces2);
                free_scratch(pl->traces2);
                free_scratch(pl->unfused);
                free_scratch(pl->rk);
            }
            pl->precision = value;
            return FR_OK;
        case FR_OPT_VARIANT:
            if (value != FR_FUSED && value != FR_UNFUSED && value != FR_MFMA)
                return set_error(FR_EINVAL, "variant %d", value);
            pl->variant = value;
            return FR_OK;
        case FR_OPT_BLOCK:
            if (value < 0 || value > 64) return set_error(FR_EINVAL, "block %d", value);
            pl->block = value;
            return FR_OK;
        case FR_OPT_PROFILE:
            if (value != 0 && value != 1) return set_error(FR_EINVAL, "profile %d", value);
            pl->profile = value;
            return FR_OK;
        case FR_OPT_GUESS_BASE:
            if (value != 1 && value != 2) return set_error(FR_EINVAL, "guess base %d", value);
            pl->guess_base = value;
            return FR_OK;
        case FR_OPT_GRAPH:
            if (value != 0 && value != 1) return set_error(FR_EINVAL, "graph %d", value);
            pl->use_graphs = value;
            return FR_OK;
        case FR_OPT_FUSE_STAGE:
            if (value != 0 && value != 1) return set_error(FR_EINVAL, "fuse stage %d", value);
            pl->fuse_stage = value;
            return FR_OK;
        case FR_OPT_PSEUDO:
            if (value != 0 && value != 1) return set_error(FR_EINVAL, "pseudo-time scheme %d", value);
            pl->pseudo = value;
            return FR_OK;
        case FR_OPT_FORM:
            if (value != FR_FORM_AUTO && value != FR_FORM_POINT && value != FR_FORM_LINES &&
                value != FR_FORM_HALO)
                return set_error(FR_EINVAL, "form %d", value);
            pl->form = value;
            return FR_OK;
        default:
            return set_error(FR_EINVAL, "unknown option %d", key);
    }
}

int fr_plan_get_int(const fr_plan *pl, int key, int *value)
{
    if (!pl || !value) return set_error(FR_EINVAL, "fr_plan_get_int: NULL argument");
    switch (key) {
        case FR_OPT_PRECISION: *value = pl->precision; return FR_OK;
        case FR_OPT_VARIANT: *value = pl->variant; return FR_OK;
        case FR_OPT_BLOCK: *value = pl->block; return FR_OK;
        case FR_OPT_PROFILE: *value = pl->profile; return FR_OK;
        case FR_OPT_GUESS_BASE: *value = pl->guess_base; return FR_OK;
        case FR_OPT_GRAPH: *value = pl->use_graphs; return FR_OK;
        case FR_OPT_FUSE_STAGE: *value = pl->fuse_stage; return FR_OK;
        case FR_OPT_PSEUDO: *value = pl->pseudo; return FR_OK;
        case FR_OPT_FORM: *value = pl->form; return FR_OK;
        case FR_INFO_RESIDUAL_FORM: *value = fr::residual_form(pl); return FR_OK;
        case FR_INFO_STAGE_PATH: *value = fr::stage_path(pl); return FR_OK;
        default: return set_error(FR_EINVAL, "unknown option %d", key);
    }
}

int fr_plan_kernel_stats(fr_plan *pl, int kernel, double *total_ms, int64_t *launches, int reset)
{
    if (!pl || !total_ms || !launches || kernel < 0 || kernel >= FR_K_COUNT)
        return set_error(FR_EINVAL, "fr_plan_kernel_stats: bad argument");
    prof_harvest(pl);
    *total_ms = pl->prof_ms[kernel];
    *launches = pl->prof_n[kernel];
    if (reset)
        for (int k = 0; k < FR_K_COUNT; ++k) {
            pl->prof_ms[k] = 0.0;
            pl->prof_n[k] = 0;
        }
    return FR_OK;
}

void fr_plan_destroy(fr_plan *pl)
{
    if (!pl) return;
    hipDeviceSynchronize();
    prof_harvest(pl);
    graphs_reset(pl);
    if (pl->cap_stream) hipStreamDestroy(pl->cap_stream);
    free_scratch(pl->traces);
    free_scratch(pl->unfused);
    free_scratch(pl->rk);
    free_scratch(pl->dual);
    free_scratch(pl->norm);
    free_scratch(pl->mlp);
    free_scratch(pl->diag);
    free_scratch(pl->rk34);
    free_scratch(pl->guess);
    if (pl->norm_host) hipHostFree(pl->norm_host);
    if (pl->ops64) hipFree(pl->ops64);
    if (pl->ops32) hipFree(pl->ops32);
    delete pl;
}

size_t fr_state_len(const fr_plan *pl)
{
    if (!pl) return 0;
    return (size_t)pl->ne * NV * pl->m * pl->m * pl->m;
}

}  // extern "C"
