// Flow diagnostics of a state (Sec. 5 follows the Taylor-Green run through the
// enstrophy (nu / |Omega|) int omega . omega dx, omega = curl V, and the
// kinetic energy (1 / |Omega|) int |V|^2 / 2 dx).  The integrals are the Gauss
// quadrature of the solution points, exact for the squares of the nodal
// polynomials; omega is formed from the auxiliary variables (the velocity
// gradient that hyperbolised diffusion carries):
//   omega = (s_y - r_z, q_z - s_x, r_x - q_y).
// One pass over 6 of the 13 variables plus the velocity; per-block partial
// sums in a fixed order, then one block sums them (deterministic).
#include <cmath>

#include "fr_internal.h"

namespace fr {
namespace {

constexpr int TBD = 256;
constexpr int NBD = 1024;

struct Weights {
    double w[PMAX + 1];
};

__device__ double wave_block_sum(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < TBD / 64; ++i) s += sh[i];
    return s;
}

__global__ void __launch_bounds__(TBD)
    k_diag(const double *__restrict__ U, Weights wt, int m, int64_t ne, double *__restrict__ part)
{
    __shared__ double sh[TBD / 64];
    const int ns = m * m * m;
    const int64_t npts = ne * ns;
    double ke = 0.0, en = 0.0;
    for (int64_t g = (int64_t)blockIdx.x * TBD + threadIdx.x; g < npts; g += (int64_t)gridDim.x * TBD) {
        const int64_t e = g / ns;
        const int q = (int)(g - e * ns);
        const double W = wt.w[q % m] * wt.w[(q / m) % m] * wt.w[q / (m * m)];
        const double *Ue = U + e * NV * ns + q;
        const double u = Ue[1 * ns], v = Ue[2 * ns], w = Ue[3 * ns];
        const double qy = Ue[5 * ns], qz = Ue[6 * ns], rx = Ue[7 * ns], rz = Ue[9 * ns];
        const double sx = Ue[10 * ns], sy = Ue[11 * ns];
        const double o0 = sy - rz, o1 = qz - sx, o2 = rx - qy;
        ke = fma(W, 0.5 * (u * u + v * v + w * w), ke);
        en = fma(W, o0 * o0 + o1 * o1 + o2 * o2, en);
    }
    const double bk = wave_block_sum(ke, sh);
    const double be = wave_block_sum(en, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = bk;
        part[NBD + blockIdx.x] = be;
    }
}

__global__ void __launch_bounds__(TBD) k_diag_final(const double *__restrict__ part, int nb,
                                                    double *__restrict__ out)
{
    __shared__ double sh[TBD / 64];
    for (int c = 0; c < 2; ++c) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nb; i += TBD) s += part[c * NBD + i];
        s = wave_block_sum(s, sh);
        if (threadIdx.x == 0) out[c] = s;
    }
}

}  // namespace
}  // namespace fr

using namespace fr;

extern "C" int fr_diagnostics(fr_plan *pl, const double *U, double *out, fr_stream_t sv)
{
    if (!pl || !U || !out) return set_error(FR_EINVAL, "fr_diagnostics: NULL argument");
    hipStream_t s = (hipStream_t)sv;
    const int m = pl->m;
    const int64_t npts = pl->ne * m * m * m;
    int64_t nb = (npts + TBD - 1) / TBD;
    if (nb > NBD) nb = NBD;
    if (nb < 1) nb = 1;
    if (int rc = ensure_scratch(pl->diag, (2 * NBD + 2) * sizeof(double))) return rc;
    double *part = (double *)pl->diag.ptr;
    Weights wt{};
    for (int i = 0; i < m; ++i) wt.w[i] = pl->w[i];
    hipLaunchKernelGGL(k_diag, dim3((unsigned)nb), dim3(TBD), 0, s, U, wt, m, pl->ne, part);
    if (int rc = check_hip(hipGetLastError(), "k_diag launch")) return rc;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(TBD), 0, s, part, (int)nb, part + 2 * NBD);
    if (int rc = check_hip(hipGetLastError(), "k_diag_final launch")) return rc;
    double h[2];
    if (int rc = check_hip(hipMemcpyAsync(h, part + 2 * NBD, sizeof h, hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync(diag)"))
        return rc;
    if (int rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize")) return rc;
    const double vol = 8.0 * (double)pl->ne;  // reference volume per element; det J cancels
    out[0] = h[0] / vol;
    out[1] = pl->nu * h[1] / vol;
    return FR_OK;
}
