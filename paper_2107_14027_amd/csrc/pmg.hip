// P-multigrid dual time stepping (the paper's Sec. 5 accelerates the
// pseudo-iterations with a P-multigrid cycle of (order, pseudo-steps) and a
// pseudo-step grown by a constant factor per level below the finest).  A
// full-approximation-scheme cycle:
//   level l solves dU/dtau = R*_l(U) + d_l, R*_l the BDF pseudo-residual of
//   order l with the BDF constant restricted from the finest level, d_l the
//   defect (zero on the finest level);
//   down h -> l = h - 1:  r_h = R*_h(U_h) + d_h,  U_l = I U_h (kept as U_l^0),
//                         d_l = I r_h - R*_l(U_l);
//   up l -> h:            U_h += P (U_l - U_l^0);
// I is the L2 projection onto degree l per direction (Gauss quadrature of the
// fine points, exact), P the interpolation of the coarse nodal polynomial at
// the fine points; both are applied per element as tensor products.  Every
// level takes classical RK4 pseudo-steps of dtau * factor^(P - l).
//
// The transfers and the defect are small next to a residual (one read of each
// array), so their kernels are plain: one thread per output value.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fr_internal.h"

struct fr_pmg {
    fr_plan *fine = nullptr;
    int P = 0;
    std::vector<int> ord, nst;
    double factor = 1.75;
    fr_plan *lv[fr::PMAX + 1] = {};        // lv[P] = fine (borrowed), coarser ones owned
    double *U[fr::PMAX + 1] = {};          // coarse states (double)
    double *U0[fr::PMAX + 1] = {};         // coarse states at descent
    double *D[fr::PMAX + 1] = {};          // coarse defects
    double *B[fr::PMAX + 1] = {};          // BDF constants [ne][3][m^3] (finest included)
    double *ops = nullptr;                 // per level l below P: I (m_l x m_{l+1}), P (m_{l+1} x m_l)
    size_t offI[fr::PMAX + 1] = {}, offP[fr::PMAX + 1] = {};
    double *r = nullptr;                   // R*_h + d_h of the level being left (finest size)
};

namespace fr {
namespace {

constexpr int TBP = 256;

unsigned grid_of(int64_t n)
{
    int64_t g = (n + TBP - 1) / TBP;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

// out[blk][c][b][a] (+)= sum_{k,j,i} A[c][k] A[b][j] A[a][i] (X - X0)[blk][k][j][i]
// for every block of m_in^3 values (X0 may be null); A is m_out x m_in.
__global__ void __launch_bounds__(TBP)
    k_transfer(const double *__restrict__ X, const double *__restrict__ X0,
               double *__restrict__ out, const double *__restrict__ A, int m_in, int m_out,
               int64_t nblk, int add)
{
    __shared__ double sA[(PMAX + 1) * (PMAX + 1)];
    for (int t = threadIdx.x; t < m_out * m_in; t += TBP) sA[t] = A[t];
    __syncthreads();
    const int so = m_out * m_out * m_out, si = m_in * m_in * m_in;
    const int64_t total = nblk * so;
    for (int64_t g = (int64_t)blockIdx.x * TBP + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * TBP) {
        const int64_t blk = g / so;
        const int q = (int)(g - blk * so);
        const int a = q % m_out, b = (q / m_out) % m_out, c = q / (m_out * m_out);
        const double *x = X + blk * si;
        const double *x0 = X0 ? X0 + blk * si : nullptr;
        double acc = 0.0;
        for (int k = 0; k < m_in; ++k) {
            double sk = 0.0;
            for (int j = 0; j < m_in; ++j) {
                double sj = 0.0;
                for (int i = 0; i < m_in; ++i) {
                    const int idx = (k * m_in + j) * m_in + i;
                    const double v = x0 ? x[idx] - x0[idx] : x[idx];
                    sj = fma(sA[a * m_in + i], v, sj);
                }
                sk = fma(sA[b * m_in + j], sj, sk);
            }
            acc = fma(sA[c * m_in + k], sk, acc);
        }
        out[g] = add ? out[g] + acc : acc;
    }
}

// R* = k - [v in V] (a U + B) for a residual k of the plan precision;
//   mode 0: out = R* + D (D may be null);   mode 1: out -= R*.
template <typename T>
__global__ void __launch_bounds__(TBP)
    k_pseudo(const T *__restrict__ k, const double *__restrict__ U, const double *__restrict__ B,
             const double *__restrict__ D, double a, double *__restrict__ out, int64_t n, int ns,
             int mode)
{
    for (int64_t i = (int64_t)blockIdx.x * TBP + threadIdx.x; i < n; i += (int64_t)gridDim.x * TBP) {
        double kv = (double)k[i];
        const int64_t r = i / ns;
        const int v = (int)(r % NV);
        if (v >= 1 && v <= 3) {
            const int64_t e = r / NV;
            kv -= fma(a, U[i], B[(e * 3 + (v - 1)) * ns + (i - r * ns)]);
        }
        if (mode == 0) out[i] = D ? kv + D[i] : kv;
        else out[i] -= kv;
    }
}

int launch_transfer(const double *X, const double *X0, double *out, const double *A, int m_in,
                    int m_out, int64_t nblk, bool add, hipStream_t s)
{
    hipLaunchKernelGGL(k_transfer, dim3(grid_of(nblk * m_out * m_out * m_out)), dim3(TBP), 0, s,
                       X, X0, out, A, m_in, m_out, nblk, add ? 1 : 0);
    return check_hip(hipGetLastError(), "k_transfer launch");
}

// out = R*_l(U) + D (mode 0) or out -= R*_l(U) (mode 1) on plan pl
int pseudo_residual(fr_plan *pl, const double *U, const double *B, const double *D, double a,
                    double *out, int mode, hipStream_t s)
{
    const int64_t n = (int64_t)fr_state_len(pl);
    const int ns = pl->m * pl->m * pl->m;
    const bool f64 = pl->precision == FR_F64;
    const size_t esz = f64 ? 8 : 4;
    // the plan's RK scratch: [acc (double)][stage (T)][k (T)]
    if (int rc = ensure_scratch(pl->rk, (size_t)n * 8 + 2 * (size_t)n * esz)) return rc;
    void *st = (char *)pl->rk.ptr + n * 8;
    void *k = (char *)st + n * esz;
    if (!f64)
        if (int rc = launch_to_precision(pl, U, st, n, s)) return rc;
    const int rc = launch_residual(pl, f64 ? (const void *)U : st, k, s);
    if (rc) return rc;
    if (f64)
        hipLaunchKernelGGL(k_pseudo<double>, dim3(grid_of(n)), dim3(TBP), 0, s, (const double *)k, U,
                           B, D, a, out, n, ns, mode);
    else
        hipLaunchKernelGGL(k_pseudo<float>, dim3(grid_of(n)), dim3(TBP), 0, s, (const float *)k, U,
                           B, D, a, out, n, ns, mode);
    return check_hip(hipGetLastError(), "k_pseudo launch");
}

void legendre_all(int nmax, double x, double *P)
{
    P[0] = 1.0;
    if (nmax >= 1) P[1] = x;
    for (int k = 1; k < nmax; ++k) P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
}

// I (ml x mh): fine nodal values -> coarse nodal values of the L2 projection;
// Pm (mh x ml): coarse nodal polynomial evaluated at the fine points.
void transfer_1d(const fr_plan *fine, const fr_plan *coarse, double *I, double *Pm)
{
    const int mh = fine->m, ml = coarse->m;
    double Ph[8][8], Pl[8][8];
    for (int j = 0; j < mh; ++j) legendre_all(ml - 1, fine->x[j], Ph[j]);
    for (int i = 0; i < ml; ++i) legendre_all(ml - 1, coarse->x[i], Pl[i]);
    for (int i = 0; i < ml; ++i)
        for (int j = 0; j < mh; ++j) {
            double s = 0.0;
            for (int k = 0; k < ml; ++k) s += 0.5 * (2 * k + 1) * Pl[i][k] * Ph[j][k];
            I[i * mh + j] = s * fine->w[j];
        }
    for (int i = 0; i < mh; ++i)
        for (int a = 0; a < ml; ++a) {
            double l = 1.0;
            for (int b = 0; b < ml; ++b)
                if (b != a) l *= (fine->x[i] - coarse->x[b]) / (coarse->x[a] - coarse->x[b]);
            Pm[i * ml + a] = l;
        }
}

void pmg_free(fr_pmg *mg)
{
    for (int l = 0; l <= PMAX; ++l) {
        if (l != mg->P && mg->lv[l]) fr_plan_destroy(mg->lv[l]);
        for (double *p : {mg->U[l], mg->U0[l], mg->D[l], mg->B[l]})
            if (p) hipFree(p);
    }
    if (mg->ops) hipFree(mg->ops);
    if (mg->r) hipFree(mg->r);
    delete mg;
}

}  // namespace
}  // namespace fr

using namespace fr;

extern "C" {

fr_pmg *fr_pmg_create(fr_plan *fine, int nlevels, const int *orders, const int *steps,
                      double factor)
{
    if (!fine) {
        set_error(FR_EINVAL, "fr_pmg_create: NULL plan");
        return nullptr;
    }
    if (!(factor > 0.0) || !std::isfinite(factor)) {
        set_error(FR_EINVAL, "fr_pmg_create: factor %g", factor);
        return nullptr;
    }
    const int P = fine->p;
    std::vector<int> ord, nst;
    if (nlevels == 0 && !orders && !steps) {
        // the paper's cycle shape: one step per level down, four on order 1,
        // one per level up, seven on the finest order
        if (P == 1) {
            ord = {1};
            nst = {1};
        } else {
            for (int p = P; p > 1; --p) ord.push_back(p), nst.push_back(1);
            ord.push_back(1), nst.push_back(4);
            for (int p = 2; p < P; ++p) ord.push_back(p), nst.push_back(1);
            ord.push_back(P), nst.push_back(7);
        }
    } else {
        if (nlevels < 1 || !orders || !steps) {
            set_error(FR_EINVAL, "fr_pmg_create: %d levels", nlevels);
            return nullptr;
        }
        ord.assign(orders, orders + nlevels);
        nst.assign(steps, steps + nlevels);
    }
    const int nl = (int)ord.size();
    if (ord[0] != P || ord[nl - 1] != P) {
        set_error(FR_EINVAL, "fr_pmg_create: the cycle must start and end on order %d", P);
        return nullptr;
    }
    for (int i = 0; i < nl; ++i) {
        if (nst[i] < 0 || ord[i] < 1 || ord[i] > P ||
            (i > 0 && std::abs(ord[i] - ord[i - 1]) != 1)) {
            set_error(FR_EINVAL, "fr_pmg_create: bad cycle entry %d (order %d, %d steps)", i,
                      ord[i], nst[i]);
            return nullptr;
        }
    }
    fr_pmg *mg = new fr_pmg;
    mg->fine = fine;
    mg->P = P;
    mg->ord = ord;
    mg->nst = nst;
    mg->factor = factor;
    mg->lv[P] = fine;
    const int pmin = *std::min_element(ord.begin(), ord.end());
    const double hd[2] = {fine->nu, fine->T};
    const int64_t ne = fine->ne;
    bool ok = true;
    for (int l = pmin; l < P && ok; ++l) {
        mg->lv[l] = fr_plan_create(l, fine->nx, fine->ny, fine->nz, fine->J, fine->zeta, hd);
        ok = mg->lv[l] != nullptr;
    }
    size_t nops = 0;
    for (int l = pmin; l < P; ++l) {
        mg->offI[l] = nops;
        nops += (size_t)(l + 1) * (l + 2);
        mg->offP[l] = nops;
        nops += (size_t)(l + 1) * (l + 2);
    }
    for (int l = pmin; l <= P && ok; ++l) {
        const size_t ns = (size_t)(l + 1) * (l + 1) * (l + 1), n = (size_t)ne * NV * ns;
        ok = check_hip(hipMalloc((void **)&mg->B[l], (size_t)ne * 3 * ns * sizeof(double)),
                       "hipMalloc(pmg)") == FR_OK;
        if (ok && l < P)
            ok = check_hip(hipMalloc((void **)&mg->U[l], n * sizeof(double)), "hipMalloc(pmg)") == FR_OK &&
                 check_hip(hipMalloc((void **)&mg->U0[l], n * sizeof(double)), "hipMalloc(pmg)") == FR_OK &&
                 check_hip(hipMalloc((void **)&mg->D[l], n * sizeof(double)), "hipMalloc(pmg)") == FR_OK;
    }
    if (ok)
        ok = check_hip(hipMalloc((void **)&mg->r, fr_state_len(fine) * sizeof(double)),
                       "hipMalloc(pmg)") == FR_OK;
    if (ok && nops) {
        std::vector<double> h(nops);
        for (int l = pmin; l < P; ++l)
            transfer_1d(mg->lv[l + 1], mg->lv[l], h.data() + mg->offI[l], h.data() + mg->offP[l]);
        ok = check_hip(hipMalloc((void **)&mg->ops, nops * sizeof(double)), "hipMalloc(pmg)") == FR_OK &&
             check_hip(hipMemcpy(mg->ops, h.data(), nops * sizeof(double), hipMemcpyHostToDevice),
                       "hipMemcpy(pmg)") == FR_OK;
    }
    if (!ok) {
        pmg_free(mg);
        return nullptr;
    }
    return mg;
}

void fr_pmg_destroy(fr_pmg *mg)
{
    if (!mg) return;
    hipDeviceSynchronize();
    pmg_free(mg);
}

int fr_pmg_dual_step(fr_pmg *mg, double *U, const double *Un, const double *Unm1, double dt,
                     double dtau, double tol, int max_cycles, int *cycles, double *resid,
                     fr_stream_t sv)
{
    if (!mg) return set_error(FR_EINVAL, "fr_pmg_dual_step: NULL multigrid");
    if (!U || !Un || !cycles || !resid)
        return set_error(FR_EINVAL, "fr_pmg_dual_step: NULL argument");
    if (!(dt > 0.0) || !(dtau > 0.0) || !(tol > 0.0) || max_cycles < 0)
        return set_error(FR_EINVAL, "fr_pmg_dual_step: dt=%g dtau=%g tol=%g max_cycles=%d", dt,
                         dtau, tol, max_cycles);
    *cycles = 0;
    *resid = NAN;
    hipStream_t s = (hipStream_t)sv;
    const int P = mg->P;
    fr_plan *fine = mg->fine;
    const int64_t ne = fine->ne;
    // coarse plans follow the fine plan's settings
    for (int l = 1; l < P; ++l)
        if (fr_plan *c = mg->lv[l]) {
            if (int rc = fr_plan_set_int(c, FR_OPT_PRECISION, fine->precision)) return rc;
            if (int rc = fr_plan_set_int(c, FR_OPT_VARIANT, fine->variant)) return rc;
            if (int rc = fr_plan_set_int(c, FR_OPT_FUSE_STAGE, fine->fuse_stage)) return rc;
            if (int rc = fr_plan_set_int(c, FR_OPT_PSEUDO, fine->pseudo)) return rc;
            if (int rc = fr_plan_set_int(c, FR_OPT_GRAPH, fine->use_graphs)) return rc;
        }
    const double a = Unm1 ? 1.5 / dt : 1.0 / dt;
    if (int rc = launch_bdf_const(fine, Un, Unm1, dt, mg->B[P], s)) return rc;
    for (int l = P - 1; l >= 1 && mg->lv[l]; --l)
        if (int rc = launch_transfer(mg->B[l + 1], nullptr, mg->B[l], mg->ops + mg->offI[l], l + 2,
                                     l + 1, ne * 3, false, s))
            return rc;
    // the finest level's norm (no steps)
    int it = 0, conv = 0, done = 0;
    double res = NAN;
    auto fail = [&](int rc) {
        *cycles = done;
        *resid = res;
        return rc;
    };
    if (int rc = pseudo_iterate(fine, U, mg->B[P], a, nullptr, dtau, tol, 0, 1, true, &it, &res,
                                &conv, s))
        return fail(rc);
    const int nl = (int)mg->ord.size();
    while (!conv && done < max_cycles) {
        double *Us[PMAX + 1] = {};
        Us[P] = U;
        for (int l = 1; l < P; ++l) Us[l] = mg->U[l];
        int prev = 0;
        for (int i = 0; i < nl; ++i) {
            const int p = mg->ord[i];
            if (prev && p < prev) {
                const int h = prev;
                if (int rc = pseudo_residual(mg->lv[h], Us[h], mg->B[h], h < P ? mg->D[h] : nullptr,
                                             a, mg->r, 0, s))
                    return fail(rc);
                const double *I = mg->ops + mg->offI[p];
                const size_t n = fr_state_len(mg->lv[p]);
                if (int rc = launch_transfer(Us[h], nullptr, Us[p], I, h + 1, p + 1, ne * NV, false, s))
                    return fail(rc);
                if (int rc = check_hip(hipMemcpyAsync(mg->U0[p], Us[p], n * sizeof(double),
                                                      hipMemcpyDeviceToDevice, s),
                                       "hipMemcpyAsync(pmg)"))
                    return fail(rc);
                if (int rc = launch_transfer(mg->r, nullptr, mg->D[p], I, h + 1, p + 1, ne * NV, false, s))
                    return fail(rc);
                if (int rc = pseudo_residual(mg->lv[p], Us[p], mg->B[p], nullptr, a, mg->D[p], 1, s))
                    return fail(rc);
            } else if (prev && p > prev) {
                const int l = prev;
                if (int rc = launch_transfer(Us[l], mg->U0[l], Us[p], mg->ops + mg->offP[l], l + 1,
                                             p + 1, ne * NV, true, s))
                    return fail(rc);
            }
            const bool last = i == nl - 1;
            const double dt_l = dtau * std::pow(mg->factor, P - p);
            int li = 0, lc = 0;
            double lr = NAN;
            if (int rc = pseudo_iterate(mg->lv[p], Us[p], mg->B[p], a, p < P ? mg->D[p] : nullptr,
                                        dt_l, tol, mg->nst[i], 0, last, &li, &lr, &lc, s))
                return fail(rc);
            if (last) res = lr;
            prev = p;
        }
        ++done;
        conv = res < tol;
    }
    *cycles = done;
    *resid = res;
    if (!std::isfinite(res))
        return set_error(FR_ENONFINITE, "pseudo-residual norm is %g after %d cycles", res, done);
    if (!conv)
        return set_error(FR_ENOCONV, "no convergence in %d cycles (residual %g)", done, res);
    return FR_OK;
}

}  // extern "C"
