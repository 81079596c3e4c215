// ACM-HD residual on linear hexahedra: the Jacobian varies inside each
// element, which the paper leaves as future work, noting that linear elements
// need only their corners (Sec. 6).  Each element is the trilinear image of
// [-1, 1]^3 written in monomials,
//   x(xi) = b0 + b1 xi0 + b2 xi1 + b3 xi2 + b4 xi0 xi1 + b5 xi1 xi2 + b6 xi0 xi2
//           + b7 xi0 xi1 xi2,
// with b computed from the 8 corners; the tangents a_d = dx/dxi_d, the metric
// rows S_d = a_{d+1} x a_{d+2} (= det J J^{-T} e_d) and det J = a_0 . S_0 are
// evaluated wherever they are needed, so no metric array is stored.  The FR
// residual of Table 1 with these point-wise metrics:
//   F_hat_d = F(U) . S_d at every point, its derivative along xi_d with the
//   partially corrected operator, the common flux |S_d| F^I(n_hat = S_d/|S_d|)
//   at every face point (once per interface, from the minus-side element's
//   metric), R = -div / det J + S(U).
// Three kernels, double precision (the trace kernel stages its elements'
// states in LDS, the residual kernel their transformed fluxes):
//   k_lh_trace   corners, U -> face traces of P, V and (grad V) n_hat
//                                                      utr[e][6][7][m^2]
//   k_lh_common  corners, utr -> |S| F^I               FI[e][3][13][m^2]  (plus faces)
//   k_lh_resid   corners, U, FI -> R
#include <cmath>

#include "fr_device.h"

namespace fr {
namespace {

constexpr int TB = 256;
constexpr int MM = PMAX + 1;

struct LhArgs {
    double Dt[MM * MM];      // partially corrected derivative operator
    double gl[MM], gr[MM];   // correction derivatives at the points
    double lm[MM], lp[MM];   // l_k(-1), l_k(+1)
    double x[MM];            // solution points
    double zeta, nu, invT;
    int m, nx, ny, nz;
};

__device__ __forceinline__ int lpt(int m, int d, int a, int b, int l)
{
    return d == 0 ? l + m * (a + m * b) : (d == 1 ? a + m * (l + m * b) : a + m * (b + m * l));
}

__device__ __forceinline__ int64_t nbr_plus(const LhArgs &A, int64_t e, int d, int dir)
{
    int64_t ex = e % A.nx, t = e / A.nx;
    int64_t ey = t % A.ny, ez = t / A.ny;
    if (d == 0) ex = (ex + dir + A.nx) % A.nx;
    else if (d == 1) ey = (ey + dir + A.ny) % A.ny;
    else ez = (ez + dir + A.nz) % A.nz;
    return ex + (int64_t)A.nx * (ey + (int64_t)A.ny * ez);
}

// monomial coefficients b[k][j] of the trilinear map from corners Ce[8][3]
// (corner c = c0 + 2 c1 + 4 c2, c_d = 0 at xi_d = -1)
__device__ __forceinline__ void trilinear(const double *__restrict__ Ce, double b[8][3])
{
    for (int k = 0; k < 8; ++k)
        for (int j = 0; j < 3; ++j) b[k][j] = 0.0;
    for (int c = 0; c < 8; ++c) {
        const double s0 = (c & 1) ? 1.0 : -1.0, s1 = (c & 2) ? 1.0 : -1.0, s2 = (c & 4) ? 1.0 : -1.0;
        const double mono[8] = {1.0, s0, s1, s2, s0 * s1, s1 * s2, s0 * s2, s0 * s1 * s2};
        for (int j = 0; j < 3; ++j) {
            const double X = Ce[3 * c + j];
            for (int k = 0; k < 8; ++k) b[k][j] += 0.125 * mono[k] * X;
        }
    }
}

// metric row S_d = a_{d+1} x a_{d+2} at xi = (x0, x1, x2); det J when wanted
__device__ __forceinline__ void metric_row(const double b[8][3], double x0, double x1, double x2,
                                           int d, double S[3], double *det)
{
    double a[3][3];
    for (int j = 0; j < 3; ++j) {
        a[0][j] = b[1][j] + b[4][j] * x1 + b[6][j] * x2 + b[7][j] * x1 * x2;
        a[1][j] = b[2][j] + b[4][j] * x0 + b[5][j] * x2 + b[7][j] * x0 * x2;
        a[2][j] = b[3][j] + b[5][j] * x1 + b[6][j] * x0 + b[7][j] * x0 * x1;
    }
    const double *p = a[(d + 1) % 3], *q = a[(d + 2) % 3];
    S[0] = p[1] * q[2] - p[2] * q[1];
    S[1] = p[2] * q[0] - p[0] * q[2];
    S[2] = p[0] * q[1] - p[1] * q[0];
    if (det) {
        const double s0 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
        const double s1 = a[1][2] * a[2][0] - a[1][0] * a[2][2];
        const double s2 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
        *det = a[0][0] * s0 + a[0][1] * s1 + a[0][2] * s2;
    }
}

// unit normal n_hat = S_d / |S_d| and |S_d| at face point (a, b) of face f
// (xi_d = -1 or +1; the normal points along +xi_d on both faces)
__device__ __forceinline__ double face_normal(const double b[8][3], const LhArgs &A, int f, int a, int bb,
                                              double nh[3])
{
    const int d = f >> 1;
    const double xs = (f & 1) ? 1.0 : -1.0, xa = A.x[a], xb = A.x[bb];
    const double x0 = d == 0 ? xs : xa, x1 = d == 0 ? xa : (d == 1 ? xs : xb), x2 = d == 2 ? xs : xb;
    double S[3];
    metric_row(b, x0, x1, x2, d, S, nullptr);
    const double nmag = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    nh[0] = S[0] / nmag, nh[1] = S[1] / nmag, nh[2] = S[2] / nmag;
    return nmag;
}

// Face traces: a workgroup loads the states of `epb` elements into LDS with
// coalesced reads; one thread per (element, face, face point) then writes the
// 7 values the common flux needs, P, V and (grad V) n_hat, with n_hat from
// the element's own corners (utr[e][f][7][m^2]; consecutive threads write
// consecutive face points).
template <int M>
__global__ void __launch_bounds__(TB) k_lh_trace(const double *__restrict__ corners,
                                                 const double *__restrict__ U,
                                                 double *__restrict__ utr, LhArgs A, int64_t ne,
                                                 int epb)
{
    extern __shared__ double lds[];   // [epb][13][m^3]
    constexpr int m = M, nfp = m * m, ns = nfp * m;
    const int64_t e0 = (int64_t)blockIdx.x * epb;
    const int nel = (int)(ne - e0 < epb ? ne - e0 : epb);
    const int nin = nel * NV * ns;
    const double *Ub = U + e0 * NV * ns;
    for (int i = threadIdx.x; i < nin; i += TB) lds[i] = Ub[i];
    __syncthreads();
    for (int o = threadIdx.x; o < nel * 6 * nfp; o += TB) {
        const int el = o / (6 * nfp), f = (o / nfp) % 6, ab = o % nfp;
        const int d = f >> 1, a = ab % m, b = ab / m;
        double bc[8][3], nh[3];
        trilinear(corners + (e0 + el) * 24, bc);
        face_normal(bc, A, f, a, b, nh);
        const double *L = (f & 1) ? A.lp : A.lm;
        const double *X = lds + el * NV * ns;
        double t[NV];
        for (int v = 0; v < NV; ++v) {
            double acc = 0.0;
            for (int l = 0; l < m; ++l) acc += L[l] * X[v * ns + lpt(m, d, a, b, l)];
            t[v] = acc;
        }
        double *out = utr + ((e0 + el) * 6 + f) * NTR * nfp + ab;
        for (int c = 0; c < 4; ++c) out[c * nfp] = t[c];
        for (int i = 0; i < 3; ++i)
            out[(4 + i) * nfp] = t[4 + 3 * i] * nh[0] + t[5 + 3 * i] * nh[1] + t[6 + 3 * i] * nh[2];
    }
}

// Common flux at the plus faces: Rusanov on (P, V), mean of the two normal
// fluxes for the auxiliary equations, from the 7-value traces, along the
// minus-side element's normal, times |S_d|.
template <int M>
__global__ void __launch_bounds__(TB) k_lh_common(const double *__restrict__ corners,
                                                  const double *__restrict__ utr,
                                                  double *__restrict__ FI, LhArgs A, int64_t ne)
{
    constexpr int m = M, nfp = m * m;
    const int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (t >= ne * 3 * nfp) return;
    const int ab = (int)(t % nfp);
    const int d = (int)((t / nfp) % 3);
    const int64_t e = t / (3 * nfp);
    const int a = ab % m, b = ab / m;
    double bc[8][3], nh[3];
    trilinear(corners + e * 24, bc);
    const double nmag = face_normal(bc, A, 2 * d + 1, a, b, nh);
    const int64_t er = nbr_plus(A, e, d, +1);
    double L[NTR], R[NTR];
    for (int c = 0; c < NTR; ++c) {
        L[c] = utr[((e * 6 + 2 * d + 1) * NTR + c) * nfp + ab];
        R[c] = utr[((er * 6 + 2 * d) * NTR + c) * nfp + ab];
    }
    const double vnL = L[1] * nh[0] + L[2] * nh[1] + L[3] * nh[2];
    const double vnR = R[1] * nh[0] + R[2] * nh[1] + R[3] * nh[2];
    const double lam = fmax(fabs(vnL) + sqrt(vnL * vnL + A.zeta), fabs(vnR) + sqrt(vnR * vnR + A.zeta));
    double *out = FI + (e * 3 + d) * NV * nfp + ab;
    out[0] = nmag * (0.5 * A.zeta * (vnL + vnR) - 0.5 * lam * (R[0] - L[0]));
    for (int i = 0; i < 3; ++i) {
        const double fl = L[1 + i] * vnL + L[0] * nh[i] - A.nu * L[4 + i];
        const double fr = R[1 + i] * vnR + R[0] * nh[i] - A.nu * R[4 + i];
        out[(1 + i) * nfp] = nmag * (0.5 * (fl + fr) - 0.5 * lam * (R[1 + i] - L[1 + i]));
        const double vm = -0.5 * A.invT * (L[1 + i] + R[1 + i]);
        for (int k = 0; k < 3; ++k) out[(4 + 3 * i + k) * nfp] = nmag * (vm * nh[k]);
    }
}

// Residual: a workgroup holds `epb` elements, one thread per solution point.
// Each thread evaluates the metric at its own point once; per direction d it
// writes its transformed flux F . S_d to LDS, and after a barrier contracts
// the partially corrected operator along its d-line from LDS, so the flux is
// evaluated three times per point rather than on every point of three lines.
constexpr int RES_TB = 384;

// (Compiled per order with the line loop kept rolled: unrolling it for a
// fixed order costs registers, 230 or more from p = 4 up, and spills at p = 5, 6.)
template <int M>
__global__ void __launch_bounds__(RES_TB) k_lh_resid(const double *__restrict__ corners,
                                                     const double *__restrict__ U,
                                                     const double *__restrict__ FI,
                                                     double *__restrict__ R, LhArgs A, int64_t ne,
                                                     int epb)
{
    extern __shared__ double lds[];   // [epb][13][m^3]
    constexpr int m = M, nfp = m * m, ns = nfp * m;
    const int el = threadIdx.x / ns, q = threadIdx.x % ns;
    const int64_t e = (int64_t)blockIdx.x * epb + el;
    const bool on = el < epb && e < ne;
    const int pi[3] = {q % m, (q / m) % m, q / nfp};
    double S[3][3], det = 1.0, Up[NV], div[NV];
    for (int v = 0; v < NV; ++v) div[v] = 0.0;
    if (on) {
        double bc[8][3];
        trilinear(corners + e * 24, bc);
        for (int d = 0; d < 3; ++d)
            metric_row(bc, A.x[pi[0]], A.x[pi[1]], A.x[pi[2]], d, S[d], d == 0 ? &det : nullptr);
        for (int v = 0; v < NV; ++v) Up[v] = U[(e * NV + v) * ns + q];
    }
    double *F = lds + (size_t)el * NV * ns;
    for (int d = 0; d < 3; ++d) {
        if (on) {
            double Fh[NV];
            dev::flux_dot<double>(Up, S[d], A.zeta, A.nu, A.invT, Fh);
            for (int v = 0; v < NV; ++v) F[v * ns + q] = Fh[v];
        }
        __syncthreads();
        if (on) {
            const int l0 = pi[d];
            const int a = d == 0 ? pi[1] : pi[0], b = d == 2 ? pi[1] : pi[2];
#pragma unroll 1
            for (int l = 0; l < m; ++l) {
                const int pt = lpt(m, d, a, b, l);
                const double w = A.Dt[l0 * m + l];
                for (int v = 0; v < NV; ++v) div[v] += w * F[v * ns + pt];
            }
            const int ab = a + m * b;
            const int64_t em = nbr_plus(A, e, d, -1);
            const double *Fp = FI + (e * 3 + d) * NV * nfp + ab;
            const double *Fm = FI + (em * 3 + d) * NV * nfp + ab;
            for (int v = 0; v < NV; ++v) div[v] += A.gl[l0] * Fm[v * nfp] + A.gr[l0] * Fp[v * nfp];
        }
        __syncthreads();
    }
    if (!on) return;
    double *Re = R + e * NV * ns + q;
    for (int v = 0; v < NV; ++v) {
        double r = -div[v] / det;
        if (v >= 4) r -= Up[v] * A.invT;
        Re[v * ns] = r;
    }
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + TB - 1) / TB); }

}  // namespace
}  // namespace fr

struct fr_lhex {
    fr_plan *plan = nullptr;
    fr::LhArgs args;
    double *utr = nullptr, *FI = nullptr;
};

using namespace fr;

namespace {

// Launches for order M - 1: elements per workgroup of the trace and residual
// kernels are as many whole elements as fit 256 threads (one if an element has
// more points); the residual kernel takes one thread per point, rounded up to
// whole waves.
template <int M>
int launch_lhex(fr_lhex *h, const double *corners, const double *U, double *R, hipStream_t s)
{
    constexpr int nfp = M * M, ns = nfp * M;
    const int64_t ne = h->plan->ne;
    const int epb = ns >= 256 ? 1 : 256 / ns;
    const size_t lds = (size_t)epb * NV * ns * sizeof(double);
    const unsigned groups = (unsigned)((ne + epb - 1) / epb);
    hipLaunchKernelGGL(k_lh_trace<M>, dim3(groups), dim3(TB), lds, s, corners, U, h->utr, h->args, ne, epb);
    if (int rc = check_hip(hipGetLastError(), "k_lh_trace launch")) return rc;
    hipLaunchKernelGGL(k_lh_common<M>, dim3(blocks_of(ne * 3 * nfp)), dim3(TB), 0, s, corners, h->utr,
                       h->FI, h->args, ne);
    if (int rc = check_hip(hipGetLastError(), "k_lh_common launch")) return rc;
    const int threads = (epb * ns + 63) / 64 * 64;
    hipLaunchKernelGGL(k_lh_resid<M>, dim3(groups), dim3(threads), lds, s, corners, U, h->FI, R, h->args,
                       ne, epb);
    return check_hip(hipGetLastError(), "k_lh_resid launch");
}

}  // namespace

extern "C" {

fr_lhex *fr_lhex_create(fr_plan *plan)
{
    if (!plan) {
        set_error(FR_EINVAL, "fr_lhex_create: NULL plan");
        return nullptr;
    }
    fr_lhex *h = new fr_lhex();
    h->plan = plan;
    LhArgs &A = h->args;
    const int m = plan->m;
    A.m = m;
    A.nx = plan->nx, A.ny = plan->ny, A.nz = plan->nz;
    for (int i = 0; i < m * m; ++i) A.Dt[i] = plan->Dt[i];
    for (int i = 0; i < m; ++i)
        A.gl[i] = plan->gl[i], A.gr[i] = plan->gr[i], A.lm[i] = plan->lm[i], A.lp[i] = plan->lp[i],
        A.x[i] = plan->x[i];
    A.zeta = plan->zeta;
    A.nu = plan->nu;
    A.invT = 1.0 / plan->T;
    const size_t nfp = (size_t)m * m, ne = (size_t)plan->ne;
    if (check_hip(hipMalloc((void **)&h->utr, ne * 6 * NTR * nfp * sizeof(double)), "hipMalloc(lhex traces)") ||
        check_hip(hipMalloc((void **)&h->FI, ne * 3 * NV * nfp * sizeof(double)), "hipMalloc(lhex fluxes)")) {
        fr_lhex_destroy(h);
        return nullptr;
    }
    return h;
}

int fr_lhex_residual(fr_lhex *h, const double *corners, const double *U, double *R, fr_stream_t sv)
{
    if (!h || !corners || !U || !R) return set_error(FR_EINVAL, "fr_lhex_residual: NULL argument");
    if (((uintptr_t)corners | (uintptr_t)U | (uintptr_t)R) & 7)
        return set_error(FR_EINVAL, "fr_lhex_residual: unaligned array");
    if (U == R) return set_error(FR_EINVAL, "fr_lhex_residual: R may not alias U");
    hipStream_t s = (hipStream_t)sv;
    switch (h->args.m) {
    case 2: return launch_lhex<2>(h, corners, U, R, s);
    case 3: return launch_lhex<3>(h, corners, U, R, s);
    case 4: return launch_lhex<4>(h, corners, U, R, s);
    case 5: return launch_lhex<5>(h, corners, U, R, s);
    case 6: return launch_lhex<6>(h, corners, U, R, s);
    case 7: return launch_lhex<7>(h, corners, U, R, s);
    default: return set_error(FR_EUNSUPPORTED, "fr_lhex_residual: order %d", h->args.m - 1);
    }
}

void fr_lhex_destroy(fr_lhex *h)
{
    if (!h) return;
    if (h->utr) (void)hipFree(h->utr);
    if (h->FI) (void)hipFree(h->FI);
    delete h;
}

}  // extern "C"
