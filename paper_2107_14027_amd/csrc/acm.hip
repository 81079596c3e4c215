// Standard ACM with LDG viscous fluxes: the comparison system of the paper's
// Sec. 5 (eq. acm_2d taken to three dimensions), unknowns (P, u, v, w) in
// double precision,
//   dU/dtau + div F = 0,  F_j = [zeta u_j ; u_i u_j + P delta_ij - nu du_i/dx_j].
// The viscous term needs the FR route for second-order systems (Sec. 2.1):
// a corrected velocity gradient with a common solution at the interfaces,
// then the FR divergence of the flux built with it.  Interfaces (Sec. 5):
// Rusanov on the inviscid part (the ACM-HD wave speed), LDG on the viscous
// part.  Between L (element on the minus side of a face) and R (plus side),
// unit normal n along +xi_d:
//   u^I   = (u_L + u_R)/2 + beta (u_L - u_R)
//   F_v^I = (F_vL + F_vR).n/2 - beta (F_vL - F_vR).n + tau (u_L - u_R)   (velocity)
//
// Four kernels compiled per order, every intermediate through HBM (this is
// the unfused multi-step pipeline that hyperbolised diffusion removes); the
// trace, gradient and residual kernels stage their elements' data in LDS:
//   k_acm_trace   U -> face traces of P, V         utr[e][6][4][m^2]
//   k_acm_grad    U, utr -> corrected gradient     Q[e][9][m^3]   (du_i/dx_j at 3 i + j)
//   k_acm_common  utr, Q -> common normal flux     FI[e][3][4][m^2] (plus face of e)
//   k_acm_resid   U, Q, FI -> R = -div F           R[e][4][m^3]
// Faces are numbered f = 2 d + side (side 0: xi_d = -1); a face point (a, b)
// holds the two tangential point indices in increasing direction order.
#include <algorithm>
#include <cmath>

#include "fr_internal.h"

namespace fr {
namespace {

constexpr int NA = 4;
constexpr int TB = 256;
constexpr int MM = PMAX + 1;

struct AcmArgs {
    double D[MM * MM], Dt[MM * MM];  // l_k'(x_i); D minus the two boundary corrections
    double gl[MM], gr[MM];            // correction derivatives h_l'(x_i), h_r'(x_i)
    double lm[MM], lp[MM];            // l_k(-1), l_k(+1)
    double Jinv[9];                   // (J^{-1})_{d j} at 3 d + j
    double nvec[9], nhat[9], nmag[3]; // n_d = det J J^{-T} e_d, n_d / |n_d|, |n_d|
    double inv_det, zeta, nu, beta, tau;
    int m, nx, ny, nz;
};

__device__ __forceinline__ int line_pt(int m, int d, int a, int b, int l)
{
    return d == 0 ? l + m * (a + m * b) : (d == 1 ? a + m * (l + m * b) : a + m * (b + m * l));
}

// neighbour of element e one step along direction d (dir = +-1), periodic
__device__ __forceinline__ int64_t nbr(const AcmArgs &A, int64_t e, int d, int dir)
{
    int64_t ex = e % A.nx, t = e / A.nx;
    int64_t ey = t % A.ny, ez = t / A.ny;
    if (d == 0) ex = (ex + dir + A.nx) % A.nx;
    else if (d == 1) ey = (ey + dir + A.ny) % A.ny;
    else ez = (ez + dir + A.nz) % A.nz;
    return ex + (int64_t)A.nx * (ey + (int64_t)A.ny * ez);
}

// the line through point (i, j, k) along d: its position l0 and face point (a, b)
__device__ __forceinline__ void line_of(int d, int i, int j, int k, int &l0, int &a, int &b)
{
    if (d == 0) l0 = i, a = j, b = k;
    else if (d == 1) l0 = j, a = i, b = k;
    else l0 = k, a = i, b = j;
}

// Face traces of (P, V): a workgroup loads the states of `epb` elements into
// LDS with coalesced reads, then writes their traces in output order
// (utr[e][6][4][m^2], consecutive threads write consecutive values).
template <int M>
__global__ void __launch_bounds__(TB) k_acm_trace(const double *__restrict__ U,
                                                  double *__restrict__ utr, AcmArgs A, int64_t ne,
                                                  int epb)
{
    extern __shared__ double lds[];   // [epb][4][m^3]
    constexpr int m = M, nfp = m * m, ns = nfp * m;
    const int64_t e0 = (int64_t)blockIdx.x * epb;
    const int nel = (int)(ne - e0 < epb ? ne - e0 : epb);
    const double *Ub = U + e0 * NA * ns;
    for (int i = threadIdx.x; i < nel * NA * ns; i += TB) lds[i] = Ub[i];
    __syncthreads();
    constexpr int per = 6 * NA * nfp;
    double *ob = utr + e0 * per;
    for (int o = threadIdx.x; o < nel * per; o += TB) {
        const int el = o / per, r = o % per;
        const int f = r / (NA * nfp), v = (r / nfp) % NA, ab = r % nfp;
        const int d = f >> 1, a = ab % m, b = ab / m;
        const double *L = (f & 1) ? A.lp : A.lm;
        const double *X = lds + (el * NA + v) * ns;
        double acc = 0.0;
        for (int l = 0; l < m; ++l) acc += L[l] * X[line_pt(m, d, a, b, l)];
        ob[o] = acc;
    }
}

// Workgroups of the gradient and residual kernels hold `epb` whole elements,
// one thread per solution point (block rounded up to whole waves, at most
// RES_TB threads); the element data they contract along lines sit in LDS.
constexpr int RES_TB = 384;

template <int M>
__global__ void __launch_bounds__(RES_TB) k_acm_grad(const double *__restrict__ U,
                                                     const double *__restrict__ utr,
                                                     double *__restrict__ Q, AcmArgs A, int64_t ne,
                                                     int epb)
{
    extern __shared__ double lds[];   // [epb][3][m^3] velocity
    constexpr int m = M, nfp = m * m, ns = nfp * m;
    const int el = threadIdx.x / ns, q = threadIdx.x % ns;
    const int64_t e = (int64_t)blockIdx.x * epb + el;
    const bool on = el < epb && e < ne;
    double *Vl = lds + (size_t)el * 3 * ns;
    if (on)
        for (int c = 0; c < 3; ++c) Vl[c * ns + q] = U[(e * NA + 1 + c) * ns + q];
    __syncthreads();
    if (!on) return;
    const int i = q % m, j = (q / m) % m, k = q / nfp;
    double g[3][3];  // g[c][d]: d/dxi_d of velocity component c
    for (int d = 0; d < 3; ++d) {
        int l0, a, b;
        line_of(d, i, j, k, l0, a, b);
        const int ab = a + m * b;
        const int64_t em = nbr(A, e, d, -1), ep = nbr(A, e, d, +1);
        for (int c = 0; c < 3; ++c) {
            const int v = 1 + c;
            double s = 0.0;
#pragma unroll 1
            for (int l = 0; l < m; ++l) s += A.D[l0 * m + l] * Vl[c * ns + line_pt(m, d, a, b, l)];
            const double om = utr[((e * 6 + 2 * d) * NA + v) * nfp + ab];
            const double op = utr[((e * 6 + 2 * d + 1) * NA + v) * nfp + ab];
            const double nm = utr[((em * 6 + 2 * d + 1) * NA + v) * nfp + ab];  // e-1's plus face
            const double np = utr[((ep * 6 + 2 * d) * NA + v) * nfp + ab];      // e+1's minus face
            const double uim = 0.5 * (nm + om) + A.beta * (nm - om);
            const double uip = 0.5 * (op + np) + A.beta * (op - np);
            g[c][d] = s + A.gl[l0] * (uim - om) + A.gr[l0] * (uip - op);
        }
    }
    double *Qe = Q + e * 9 * ns + q;
    for (int c = 0; c < 3; ++c)
        for (int jx = 0; jx < 3; ++jx)
            Qe[(3 * c + jx) * ns] =
                A.Jinv[jx] * g[c][0] + A.Jinv[3 + jx] * g[c][1] + A.Jinv[6 + jx] * g[c][2];
}

template <int M>
__global__ void __launch_bounds__(TB) k_acm_common(const double *__restrict__ utr,
                                                   const double *__restrict__ Q,
                                                   double *__restrict__ FI, AcmArgs A, int64_t ne)
{
    constexpr int m = M, nfp = m * m, ns = nfp * m;
    const int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (t >= ne * 3 * nfp) return;
    const int ab = (int)(t % nfp);
    const int d = (int)((t / nfp) % 3);
    const int64_t e = t / (3 * nfp);
    const int a = ab % m, b = ab / m;
    const int64_t er = nbr(A, e, d, +1);
    const double *nh = A.nhat + 3 * d;
    double uL[NA], uR[NA];
    for (int v = 0; v < NA; ++v) {
        uL[v] = utr[((e * 6 + 2 * d + 1) * NA + v) * nfp + ab];
        uR[v] = utr[((er * 6 + 2 * d) * NA + v) * nfp + ab];
    }
    // viscous normal flux -nu (grad u_c) . n of both sides, from Q traced to the face
    double fvL[3], fvR[3];
    for (int c = 0; c < 3; ++c) {
        double sl = 0.0, sr = 0.0;
        for (int jx = 0; jx < 3; ++jx) {
            double ql = 0.0, qr = 0.0;
            for (int l = 0; l < m; ++l) {
                const int pt = line_pt(m, d, a, b, l);
                ql += A.lp[l] * Q[(e * 9 + 3 * c + jx) * ns + pt];
                qr += A.lm[l] * Q[(er * 9 + 3 * c + jx) * ns + pt];
            }
            sl += ql * nh[jx];
            sr += qr * nh[jx];
        }
        fvL[c] = -A.nu * sl;
        fvR[c] = -A.nu * sr;
    }
    const double vnL = uL[1] * nh[0] + uL[2] * nh[1] + uL[3] * nh[2];
    const double vnR = uR[1] * nh[0] + uR[2] * nh[1] + uR[3] * nh[2];
    const double lam = fmax(fabs(vnL) + sqrt(vnL * vnL + A.zeta), fabs(vnR) + sqrt(vnR * vnR + A.zeta));
    double *out = FI + (e * 3 + d) * NA * nfp + ab;
    out[0] = 0.5 * A.zeta * (vnL + vnR) - 0.5 * lam * (uR[0] - uL[0]);
    for (int c = 0; c < 3; ++c) {
        const double mL = uL[1 + c] * vnL + uL[0] * nh[c];
        const double mR = uR[1 + c] * vnR + uR[0] * nh[c];
        out[(1 + c) * nfp] = 0.5 * (mL + mR) - 0.5 * lam * (uR[1 + c] - uL[1 + c]) +
                             0.5 * (fvL[c] + fvR[c]) - A.beta * (fvL[c] - fvR[c]) +
                             A.tau * (uL[1 + c] - uR[1 + c]);
    }
}

// Residual: each thread forms the transformed flux (F . n_d, four values) at
// its own point for one direction at a time, in LDS; after a barrier it
// contracts the partially corrected operator along its d-line.
template <int M>
__global__ void __launch_bounds__(RES_TB) k_acm_resid(const double *__restrict__ U,
                                                      const double *__restrict__ Q,
                                                      const double *__restrict__ FI,
                                                      double *__restrict__ R, AcmArgs A, int64_t ne,
                                                      int epb)
{
    extern __shared__ double lds[];   // [epb][4][m^3]
    constexpr int m = M, nfp = m * m, ns = nfp * m;
    const int el = threadIdx.x / ns, q = threadIdx.x % ns;
    const int64_t e = (int64_t)blockIdx.x * epb + el;
    const bool on = el < epb && e < ne;
    const int i = q % m, j = (q / m) % m, k = q / nfp;
    double P = 0.0, V[3] = {0.0, 0.0, 0.0}, G[9];
    if (on) {
        P = U[e * NA * ns + q];
        for (int c = 0; c < 3; ++c) V[c] = U[(e * NA + 1 + c) * ns + q];
        for (int t = 0; t < 9; ++t) G[t] = Q[(e * 9 + t) * ns + q];
    }
    double *F = lds + (size_t)el * NA * ns;
    double div[NA] = {0.0, 0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        if (on) {
            const double *nv = A.nvec + 3 * d;
            const double vn = V[0] * nv[0] + V[1] * nv[1] + V[2] * nv[2];
            F[q] = A.zeta * vn;
            for (int c = 0; c < 3; ++c) {
                // (V_c V + P e_c - nu grad u_c) . n_d
                const double gn = G[3 * c] * nv[0] + G[3 * c + 1] * nv[1] + G[3 * c + 2] * nv[2];
                F[(1 + c) * ns + q] = V[c] * vn + P * nv[c] - A.nu * gn;
            }
        }
        __syncthreads();
        if (on) {
            int l0, a, b;
            line_of(d, i, j, k, l0, a, b);
#pragma unroll 1
            for (int l = 0; l < m; ++l) {
                const int pt = line_pt(m, d, a, b, l);
                const double w = A.Dt[l0 * m + l];
                for (int v = 0; v < NA; ++v) div[v] += w * F[v * ns + pt];
            }
            const int ab = a + m * b;
            const int64_t em = nbr(A, e, d, -1);
            const double *Fp = FI + (e * 3 + d) * NA * nfp + ab;
            const double *Fm = FI + (em * 3 + d) * NA * nfp + ab;
            for (int v = 0; v < NA; ++v)
                div[v] += A.nmag[d] * (A.gl[l0] * Fm[v * nfp] + A.gr[l0] * Fp[v * nfp]);
        }
        __syncthreads();
    }
    if (!on) return;
    double *Re = R + e * NA * ns + q;
    for (int v = 0; v < NA; ++v) Re[v * ns] = -div[v] * A.inv_det;
}

// Dual time stepping of this system (Sec. 5): dU/dtau = R*(U) with the BDF
// source on the velocity only, dU/dt = a U + B (BDF2: a = 3/(2 dt),
// B = (-4 Un + Unm1)/(2 dt); BDF1: a = 1/dt, B = -Un/dt), classical RK4
// pseudo-steps of a fixed size.
__global__ void __launch_bounds__(TB) k_acm_bdf(const double *__restrict__ Un,
                                                const double *__restrict__ Unm1,
                                                double *__restrict__ B, double dt, int64_t n, int ns)
{
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    const int v = (int)((i / ns) % NA);
    B[i] = v == 0 ? 0.0 : (Unm1 ? (-4.0 * Un[i] + Unm1[i]) / (2.0 * dt) : -Un[i] / dt);
}

__device__ __forceinline__ double pseudo_k(const double *R, const double *S, const double *B,
                                           double a, int64_t i, int ns)
{
    const int v = (int)((i / ns) % NA);
    return v == 0 ? R[i] : R[i] - (a * S[i] + B[i]);
}

// RK4 stage s of dU/dtau = k*, k* the pseudo-residual of the state S that
// produced R:  s = 0: acc = k/6, S' = U + dtau/2 k;  s = 1, 2: acc += k/3,
// S' = U + c dtau k;  s = 3: U += dtau (acc + k/6).  S may be S' (one thread
// per index).
__global__ void __launch_bounds__(TB) k_acm_stage(double *__restrict__ U, const double *S,
                                                  const double *__restrict__ R,
                                                  const double *__restrict__ B,
                                                  double *__restrict__ acc, double *Sn, double a,
                                                  double dtau, int s, int64_t n, int ns)
{
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    const double k = pseudo_k(R, S, B, a, i, ns);
    if (s == 0) {
        acc[i] = k / 6.0;
        Sn[i] = U[i] + (0.5 * dtau) * k;
    } else if (s < 3) {
        acc[i] += k / 3.0;
        Sn[i] = U[i] + ((s == 1 ? 0.5 : 1.0) * dtau) * k;
    } else {
        U[i] += dtau * (acc[i] + k / 6.0);
    }
}

constexpr int NORM_BLOCKS = 1024;

// sum over the velocity values of k*^2: per-block partials in a fixed order
__global__ void __launch_bounds__(TB) k_acm_norm(const double *__restrict__ U,
                                                 const double *__restrict__ R,
                                                 const double *__restrict__ B, double a, int64_t n,
                                                 int ns, double *__restrict__ part)
{
    __shared__ double sh[TB];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)NORM_BLOCKS * TB)
        if ((i / ns) % NA) {
            const double k = pseudo_k(R, U, B, a, i, ns);
            acc += k * k;
        }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(TB) k_acm_norm_final(const double *__restrict__ part,
                                                       double *__restrict__ out)
{
    __shared__ double sh[TB];
    double acc = 0.0;
    for (int i = threadIdx.x; i < NORM_BLOCKS; i += TB) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + TB - 1) / TB); }

}  // namespace
}  // namespace fr

struct fr_acm {
    fr_plan *plan = nullptr;
    fr::AcmArgs args;
    double *utr = nullptr, *Q = nullptr, *FI = nullptr;
    // dual time stepping (allocated on its first call): residual, stage state,
    // RK accumulator, BDF constant, norm partials and result, pinned read-back
    double *R = nullptr, *S = nullptr, *acc = nullptr, *B = nullptr, *part = nullptr;
    double *host = nullptr;
};

using namespace fr;

namespace {

int acm_check(fr_acm *a, const void *U, const void *out, const char *what)
{
    if (!a || !U || !out) return set_error(FR_EINVAL, "%s: NULL argument", what);
    if (((uintptr_t)U | (uintptr_t)out) & 7) return set_error(FR_EINVAL, "%s: unaligned state", what);
    if (U == out) return set_error(FR_EINVAL, "%s: the output may not alias the input", what);
    return FR_OK;
}

// Trace and gradient kernels for order M - 1; the workgroups of both hold
// `epb` whole elements.
template <int M>
int launch_grad(fr_acm *a, const double *U, int64_t ne, int epb, hipStream_t s)
{
    constexpr int ns = M * M * M;
    hipLaunchKernelGGL(k_acm_trace<M>, dim3((unsigned)((ne + epb - 1) / epb)), dim3(TB),
                       (size_t)epb * NA * ns * sizeof(double), s, U, a->utr, a->args, ne, epb);
    if (int rc = check_hip(hipGetLastError(), "k_acm_trace launch")) return rc;
    hipLaunchKernelGGL(k_acm_grad<M>, dim3((unsigned)((ne + epb - 1) / epb)), dim3((epb * ns + 63) / 64 * 64),
                       (size_t)epb * 3 * ns * sizeof(double), s, U, a->utr, a->Q, a->args, ne, epb);
    return check_hip(hipGetLastError(), "k_acm_grad launch");
}

template <int M>
int launch_back(fr_acm *a, const double *U, double *R, int64_t ne, int epb, hipStream_t s)
{
    constexpr int nfp = M * M, ns = nfp * M;
    hipLaunchKernelGGL(k_acm_common<M>, dim3(blocks_for(ne * 3 * nfp)), dim3(TB), 0, s, a->utr, a->Q, a->FI,
                       a->args, ne);
    if (int rc = check_hip(hipGetLastError(), "k_acm_common launch")) return rc;
    hipLaunchKernelGGL(k_acm_resid<M>, dim3((unsigned)((ne + epb - 1) / epb)), dim3((epb * ns + 63) / 64 * 64),
                       (size_t)epb * NA * ns * sizeof(double), s, U, a->Q, a->FI, R, a->args, ne, epb);
    return check_hip(hipGetLastError(), "k_acm_resid launch");
}

#define FR_ACM_ORDERS(CALL)                                                                       \
    switch (a->args.m) {                                                                         \
    case 2: return CALL(2);                                                                      \
    case 3: return CALL(3);                                                                      \
    case 4: return CALL(4);                                                                      \
    case 5: return CALL(5);                                                                      \
    case 6: return CALL(6);                                                                      \
    case 7: return CALL(7);                                                                      \
    default: return set_error(FR_EUNSUPPORTED, "standard ACM: order %d", a->args.m - 1);         \
    }

int launch_front(fr_acm *a, const double *U, hipStream_t s)
{
    const int64_t ne = a->plan->ne;
    const int ns = a->args.m * a->args.m * a->args.m;
    const int epb = ns >= 256 ? 1 : 256 / ns;
#define FR_ACM_GRAD(M) launch_grad<M>(a, U, ne, epb, s)
    FR_ACM_ORDERS(FR_ACM_GRAD)
#undef FR_ACM_GRAD
}

int launch_residual(fr_acm *a, const double *U, double *R, hipStream_t s)
{
    const int64_t ne = a->plan->ne;
    const int ns = a->args.m * a->args.m * a->args.m;
    if (int rc = launch_front(a, U, s)) return rc;
    const int epb = ns >= 256 ? 1 : 256 / ns;
#define FR_ACM_BACK(M) launch_back<M>(a, U, R, ne, epb, s)
    FR_ACM_ORDERS(FR_ACM_BACK)
#undef FR_ACM_BACK
}

// Allocates the dual-stepping arrays all together: after a failure nothing is
// kept, so a later call tries again from scratch.
int ensure_dual(fr_acm *a)
{
    if (a->host) return FR_OK;
    const size_t n = (size_t)a->plan->ne * NA * a->args.m * a->args.m * a->args.m;
    double *dev[5] = {};
    double *host = nullptr;
    const size_t sizes[5] = {n, n, n, n, NORM_BLOCKS + 1};
    int rc = FR_OK;
    for (int i = 0; i < 5 && rc == FR_OK; ++i)
        rc = check_hip(hipMalloc((void **)&dev[i], sizes[i] * sizeof(double)), "hipMalloc(acm dual)");
    if (rc == FR_OK)
        rc = check_hip(hipHostMalloc((void **)&host, sizeof(double), hipHostMallocDefault),
                       "hipHostMalloc(acm norm)");
    if (rc != FR_OK) {
        for (double *p : dev)
            if (p) (void)hipFree(p);
        return rc;
    }
    a->R = dev[0], a->S = dev[1], a->acc = dev[2], a->B = dev[3], a->part = dev[4];
    a->host = host;
    return FR_OK;
}

// RMS of the velocity part of k* = R - M_V (a U + B), read back (synchronises s)
int velocity_rms(fr_acm *a, const double *U, double a_bdf, double *out, hipStream_t s)
{
    const int64_t n = a->plan->ne * NA * a->args.m * a->args.m * a->args.m;
    const int ns = a->args.m * a->args.m * a->args.m;
    hipLaunchKernelGGL(k_acm_norm, dim3(NORM_BLOCKS), dim3(TB), 0, s, U, a->R, a->B, a_bdf, n, ns,
                       a->part);
    if (int rc = check_hip(hipGetLastError(), "k_acm_norm launch")) return rc;
    hipLaunchKernelGGL(k_acm_norm_final, dim3(1), dim3(TB), 0, s, a->part, a->part + NORM_BLOCKS);
    if (int rc = check_hip(hipGetLastError(), "k_acm_norm_final launch")) return rc;
    if (int rc = check_hip(hipMemcpyAsync(a->host, a->part + NORM_BLOCKS, sizeof(double),
                                          hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync(acm norm)"))
        return rc;
    if (int rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize(acm norm)")) return rc;
    *out = std::sqrt(*a->host / (3.0 * (double)a->plan->ne * ns));
    return FR_OK;
}

}  // namespace

extern "C" {

fr_acm *fr_acm_create(fr_plan *plan, double ldg_beta, double ldg_tau)
{
    if (!plan) {
        set_error(FR_EINVAL, "fr_acm_create: NULL plan");
        return nullptr;
    }
    if (!std::isfinite(ldg_beta) || !std::isfinite(ldg_tau) || ldg_tau < 0.0) {
        set_error(FR_EINVAL, "fr_acm_create: beta=%g tau=%g", ldg_beta, ldg_tau);
        return nullptr;
    }
    fr_acm *a = new fr_acm();
    a->plan = plan;
    AcmArgs &A = a->args;
    const int m = plan->m;
    A.m = m;
    A.nx = plan->nx, A.ny = plan->ny, A.nz = plan->nz;
    for (int i = 0; i < m * m; ++i) A.D[i] = plan->D[i], A.Dt[i] = plan->Dt[i];
    for (int i = 0; i < m; ++i)
        A.gl[i] = plan->gl[i], A.gr[i] = plan->gr[i], A.lm[i] = plan->lm[i], A.lp[i] = plan->lp[i];
    for (int d = 0; d < 3; ++d) {
        A.nmag[d] = plan->c64.nmag[d];
        for (int j = 0; j < 3; ++j) {
            A.Jinv[3 * d + j] = plan->Jinv[3 * d + j];
            A.nvec[3 * d + j] = plan->c64.nvec[d][j];
            A.nhat[3 * d + j] = plan->c64.nhat[d][j];
        }
    }
    A.inv_det = 1.0 / plan->detJ;
    A.zeta = plan->zeta;
    A.nu = plan->nu;
    A.beta = ldg_beta;
    A.tau = ldg_tau;
    const int64_t ne = plan->ne;
    const size_t nfp = (size_t)m * m, ns = nfp * m;
    if (check_hip(hipMalloc((void **)&a->utr, (size_t)ne * 6 * NA * nfp * sizeof(double)), "hipMalloc(acm traces)") ||
        check_hip(hipMalloc((void **)&a->Q, (size_t)ne * 9 * ns * sizeof(double)), "hipMalloc(acm gradient)") ||
        check_hip(hipMalloc((void **)&a->FI, (size_t)ne * 3 * NA * nfp * sizeof(double)), "hipMalloc(acm fluxes)")) {
        fr_acm_destroy(a);
        return nullptr;
    }
    return a;
}

int fr_acm_gradient(fr_acm *a, const double *U, double *Q, fr_stream_t sv)
{
    if (int rc = acm_check(a, U, Q, "fr_acm_gradient")) return rc;
    hipStream_t s = (hipStream_t)sv;
    if (int rc = launch_front(a, U, s)) return rc;
    const size_t bytes = (size_t)a->plan->ne * 9 * a->args.m * a->args.m * a->args.m * sizeof(double);
    return check_hip(hipMemcpyAsync(Q, a->Q, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync(acm gradient)");
}

int fr_acm_residual(fr_acm *a, const double *U, double *R, fr_stream_t sv)
{
    if (int rc = acm_check(a, U, R, "fr_acm_residual")) return rc;
    return launch_residual(a, U, R, (hipStream_t)sv);
}

int fr_acm_dual_step(fr_acm *a, double *U, const double *Un, const double *Unm1, double dt,
                     double dtau, double tol, int max_iters, int check_every, int *iters,
                     double *resid, fr_stream_t sv)
{
    if (!a || !U || !Un || !iters || !resid)
        return set_error(FR_EINVAL, "fr_acm_dual_step: NULL argument");
    if (U == Un || U == Unm1) return set_error(FR_EINVAL, "fr_acm_dual_step: U aliases a past state");
    if (!(dt > 0.0) || !(dtau > 0.0) || !(tol > 0.0) || max_iters < 0 || check_every < 1)
        return set_error(FR_EINVAL, "fr_acm_dual_step: dt=%g dtau=%g tol=%g max_iters=%d check_every=%d",
                         dt, dtau, tol, max_iters, check_every);
    if (((uintptr_t)U | (uintptr_t)Un | (uintptr_t)Unm1) & 7)
        return set_error(FR_EINVAL, "fr_acm_dual_step: unaligned state");
    *iters = 0;
    *resid = NAN;
    if (int rc = ensure_dual(a)) return rc;
    hipStream_t s = (hipStream_t)sv;
    const int ns = a->args.m * a->args.m * a->args.m;
    const int64_t n = a->plan->ne * NA * ns;
    const unsigned g = blocks_for(n);
    const double ab = Unm1 ? 1.5 / dt : 1.0 / dt;
    hipLaunchKernelGGL(k_acm_bdf, dim3(g), dim3(TB), 0, s, Un, Unm1, a->B, dt, n, ns);
    if (int rc = check_hip(hipGetLastError(), "k_acm_bdf launch")) return rc;
    int it = 0;
    double res = NAN;
    for (;;) {
        if (int rc = launch_residual(a, U, a->R, s)) return rc;
        if (it % check_every == 0 || it >= max_iters) {
            if (int rc = velocity_rms(a, U, ab, &res, s)) return rc;
            *iters = it;
            *resid = res;
            if (!std::isfinite(res))
                return set_error(FR_ENONFINITE, "pseudo-residual norm is %g after %d steps", res, it);
            if (res < tol) return FR_OK;
        }
        if (it >= max_iters) break;
        for (int st = 0; st < 4; ++st) {
            if (st > 0)
                if (int rc = launch_residual(a, a->S, a->R, s)) return rc;
            hipLaunchKernelGGL(k_acm_stage, dim3(g), dim3(TB), 0, s, U, st == 0 ? U : a->S, a->R,
                               a->B, a->acc, a->S, ab, dtau, st, n, ns);
            if (int rc = check_hip(hipGetLastError(), "k_acm_stage launch")) return rc;
        }
        ++it;
    }
    return set_error(FR_ENOCONV, "no convergence in %d pseudo-steps (residual %g)", it, res);
}

void fr_acm_destroy(fr_acm *a)
{
    if (!a) return;
    if (a->utr) (void)hipFree(a->utr);
    if (a->Q) (void)hipFree(a->Q);
    if (a->FI) (void)hipFree(a->FI);
    double *bufs[5] = {a->R, a->S, a->acc, a->B, a->part};
    for (double *b : bufs)
        if (b) (void)hipFree(b);
    if (a->host) (void)hipHostFree(a->host);
    delete a;
}

}  // extern "C"
