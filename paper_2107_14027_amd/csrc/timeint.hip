// Elementwise kernels of the time integrators: classical RK4 stage updates
// with double accumulators, the BDF physical-time source of dual time stepping
// (applied in double on the velocity only), a deterministic two-level
// reduction for the pseudo-residual norm, and polynomial extrapolation.
// All are HBM-bound streams; each thread handles consecutive 64-bit or 32-bit
// words of one state array so that every wave access is contiguous.
#include "fr_internal.h"

namespace fr {
namespace {

constexpr int TB = 256;        // threads per block
constexpr int NB_MAX = 2048;   // blocks of the grid-stride loops (fixed: makes sums deterministic)

inline unsigned grid_for(int64_t n)
{
    int64_t g = (n + TB - 1) / TB;
    return (unsigned)(g > NB_MAX ? NB_MAX : (g < 1 ? 1 : g));
}

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    // fixed-order reduction: wave64 butterfly, then the waves in order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

// One RK4 stage of dU/dtau = k*, with k* = k - [v in V] (a s + B) when bdf,
// plus D (a fixed source, when given):
//   first stage: acc = U + b k*,  else acc += b k*
//   then the next stage state  s' = U + cnext k*  -> st64 (double) and stT (T)
//   last stage:  U = acc + b k*, stT = (T) U
// s (the state that produced k) is U on the first stage and st64 otherwise.
// With norm, also writes per-block sums of (k*_V)^2 into partial[blockIdx].
template <typename T, bool BDF, bool NORM>
__global__ void __launch_bounds__(TB) k_stage(double *__restrict__ U, double *__restrict__ acc,
                                              double *st64, T *stT, const T *__restrict__ k,
                                              const double *__restrict__ B,
                                              const double *__restrict__ D, double a, double b,
                                              double cnext, int first, int last, int64_t n, int ns,
                                              double *__restrict__ partial)
{
    __shared__ double sh[TB / 64];
    double ss = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        double kv = (double)k[i];
        bool vel = false;
        if (BDF || NORM) {
            const int64_t r = i / ns;
            const int v = (int)(r % NV);
            vel = v >= 1 && v <= 3;
            if (BDF && vel) {
                const double sv = first ? U[i] : st64[i];
                const int64_t e = r / NV;
                kv -= fma(a, sv, B[(e * 3 + (v - 1)) * ns + (i - r * ns)]);
            }
        }
        if (D) kv += D[i];
        if (NORM && vel) ss = fma(kv, kv, ss);
        if (last) {
            const double un = fma(b, kv, acc[i]);
            U[i] = un;
            if (stT) stT[i] = (T)un;
        } else {
            const double u = U[i];
            acc[i] = fma(b, kv, first ? u : acc[i]);
            const double sn = fma(cnext, kv, u);
            if (st64 && (void *)st64 != (void *)stT) st64[i] = sn;
            stT[i] = (T)sn;
        }
    }
    if (NORM) {
        const double s = block_sum(ss, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// One stage of the RK3(2)4[2R+]C pair (Kennedy, Carpenter and Lewis: four
// stages, third order, embedded second order, two registers) with one
// pseudo-step h per value, on dU/dtau = k* (k* as in k_stage).  With
// hk = h k*:
//   stages 0..2:  next = U + acc + anext hk;  acc += b hk;  err += bd hk
//                 (acc, err start from zero on stage 0)
//   stage 3:      U = U + acc + b hk;  e = err + bd hk;
//                 h = clamp(h clamp(0.8 (|e|/atol)^(-1/3), 0.98, 1.01), h0/3, 3 h0)
// bd = b - bhat; e is the embedded error estimate.
template <typename T>
__global__ void __launch_bounds__(TB)
    k_stage34(double *__restrict__ U, double *__restrict__ acc, double *__restrict__ err,
              double *__restrict__ h, double *st64, T *stT, const T *__restrict__ k,
              const double *__restrict__ B, const double *__restrict__ D, double a, int stage,
              double anext, double bs, double bds, double atol, double h0, int64_t n, int ns,
              double *__restrict__ partial)
{
    __shared__ double sh[TB / 64];
    double ss = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        double kv = (double)k[i];
        const int64_t r = i / ns;
        const int v = (int)(r % NV);
        const bool vel = v >= 1 && v <= 3;
        if (B && vel) {
            const double sv = stage == 0 ? U[i] : st64[i];
            kv -= fma(a, sv, B[((r / NV) * 3 + (v - 1)) * ns + (i - r * ns)]);
        }
        if (D) kv += D[i];
        if (partial && vel) ss = fma(kv, kv, ss);
        const double hv = h[i];
        const double hk = hv * kv;
        if (stage == 3) {
            const double un = U[i] + (acc[i] + bs * hk);
            const double e = err[i] + bds * hk;
            const double q = fmax(fabs(e) / atol, 1e-300);
            const double fac = fmin(fmax(0.8 * pow(q, -1.0 / 3.0), 0.98), 1.01);
            h[i] = fmin(fmax(hv * fac, h0 / 3.0), h0 * 3.0);
            U[i] = un;
            if (stT) stT[i] = (T)un;
        } else {
            const double ac = stage == 0 ? 0.0 : acc[i];
            const double sn = U[i] + (ac + anext * hk);
            acc[i] = ac + bs * hk;
            err[i] = (stage == 0 ? 0.0 : err[i]) + bds * hk;
            if (st64 && (void *)st64 != (void *)stT) st64[i] = sn;
            stT[i] = (T)sn;
        }
    }
    if (partial) {
        const double s = block_sum(ss, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(TB) k_fill(double *__restrict__ x, double v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB)
        x[i] = v;
}

__global__ void __launch_bounds__(TB) k_final_sum(const double *__restrict__ partial, int nb,
                                                  double *__restrict__ out)
{
    __shared__ double sh[TB / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += TB) s += partial[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = s;
}

template <typename T>
__global__ void __launch_bounds__(TB) k_to_prec(const double *__restrict__ U, T *__restrict__ out,
                                                int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB)
        out[i] = (T)U[i];
}

// B = (-4 Un + Unm1) / (2 dt) (BDF2) or -Un / dt (BDF1) on the velocity only.
__global__ void __launch_bounds__(TB) k_bdf_const(const double *__restrict__ Un,
                                                  const double *__restrict__ Unm1, double dt,
                                                  double *__restrict__ B, int64_t ne, int ns)
{
    const int64_t n = ne * 3 * ns;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        const int64_t r = i / ns, q = i - r * ns;
        const int64_t e = r / 3;
        const int c = (int)(r - e * 3);
        const int64_t src = (e * NV + 1 + c) * ns + q;
        B[i] = Unm1 ? (Unm1[src] - 4.0 * Un[src]) / (2.0 * dt) : -Un[src] / dt;
    }
}

// keep_ns > 0: the pressure (variable 0 of every element, keep_ns points)
// is copied from Un instead of extrapolated
__global__ void __launch_bounds__(TB) k_extrap(const double *__restrict__ Un,
                                               const double *__restrict__ Unm1,
                                               const double *__restrict__ Unm2, int order,
                                               int keep_ns, double *__restrict__ G, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        if (keep_ns && (i / keep_ns) % NV == 0) G[i] = Un[i];
        else if (order == 1) G[i] = 2.0 * Un[i] - Unm1[i];
        else G[i] = 3.0 * (Un[i] - Unm1[i]) + Unm2[i];
    }
}

template <typename T>
int stage_dispatch(bool bdf, bool norm, double *U, double *acc, double *st64, void *stT,
                   const void *k, const double *B, const double *D, double a, double b,
                   double cnext, int first, int last, int64_t n, int ns, double *partial,
                   hipStream_t s)
{
    const unsigned g = grid_for(n);
    T *st = (T *)stT;
    const T *kk = (const T *)k;
    if (bdf && norm)
        hipLaunchKernelGGL((k_stage<T, true, true>), dim3(g), dim3(TB), 0, s, U, acc, st64, st, kk,
                           B, D, a, b, cnext, first, last, n, ns, partial);
    else if (bdf)
        hipLaunchKernelGGL((k_stage<T, true, false>), dim3(g), dim3(TB), 0, s, U, acc, st64, st,
                           kk, B, D, a, b, cnext, first, last, n, ns, partial);
    else if (norm)
        hipLaunchKernelGGL((k_stage<T, false, true>), dim3(g), dim3(TB), 0, s, U, acc, st64, st,
                           kk, B, D, a, b, cnext, first, last, n, ns, partial);
    else
        hipLaunchKernelGGL((k_stage<T, false, false>), dim3(g), dim3(TB), 0, s, U, acc, st64, st,
                           kk, B, D, a, b, cnext, first, last, n, ns, partial);
    return check_hip(hipGetLastError(), "k_stage launch");
}

}  // namespace

int stage_blocks(int64_t n) { return (int)grid_for(n); }

int launch_stage(fr_plan *pl, bool bdf, bool norm, double *U, double *acc, double *st64,
                 void *stT, const void *k, const double *B, double a, double b, double cnext,
                 int first, int last, double *partial, hipStream_t s, const double *D)
{
    const int64_t n = (int64_t)fr_state_len(pl);
    const int ns = pl->m * pl->m * pl->m;
    ProfScope ps(pl, FR_K_STAGE, s);
    if (pl->precision == FR_F64)
        return stage_dispatch<double>(bdf, norm, U, acc, st64, stT, k, B, D, a, b, cnext, first,
                                      last, n, ns, partial, s);
    return stage_dispatch<float>(bdf, norm, U, acc, st64, stT, k, B, D, a, b, cnext, first, last,
                                 n, ns, partial, s);
}

int launch_stage34(fr_plan *pl, int stage, double *U, double *acc, double *err, double *h,
                   double *st64, void *stT, const void *k, const double *B, const double *D,
                   double a, double atol, double h0, double *partial, hipStream_t s)
{
    // RK3(2)4[2R+]C: sub-diagonal a_{i+1,i}, weights b, b - bhat
    static const double anext[3] = {11847461282814.0 / 36547543011857.0,
                                    3943225443063.0 / 7078155732230.0,
                                    -346793006927.0 / 4029903576067.0};
    static const double b[4] = {1017324711453.0 / 9774461848756.0, 8237718856693.0 / 13685301971492.0,
                                57731312506979.0 / 19404895981398.0,
                                -101169746363290.0 / 37734290219643.0};
    static const double bhat[4] = {15763415370699.0 / 46270243929542.0,
                                   514528521746.0 / 5659431552419.0,
                                   27030193851939.0 / 9429696342944.0,
                                   -69544964788955.0 / 30262026368149.0};
    const int64_t n = (int64_t)fr_state_len(pl);
    const int ns = pl->m * pl->m * pl->m;
    const unsigned g = grid_for(n);
    const double an = stage < 3 ? anext[stage] : 0.0;
    ProfScope ps(pl, FR_K_STAGE, s);
    if (pl->precision == FR_F64)
        hipLaunchKernelGGL(k_stage34<double>, dim3(g), dim3(TB), 0, s, U, acc, err, h, st64,
                           (double *)stT, (const double *)k, B, D, a, stage, an, b[stage],
                           b[stage] - bhat[stage], atol, h0, n, ns, partial);
    else
        hipLaunchKernelGGL(k_stage34<float>, dim3(g), dim3(TB), 0, s, U, acc, err, h, st64,
                           (float *)stT, (const float *)k, B, D, a, stage, an, b[stage],
                           b[stage] - bhat[stage], atol, h0, n, ns, partial);
    return check_hip(hipGetLastError(), "k_stage34 launch");
}

int launch_fill(double *x, double v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(TB), 0, s, x, v, n);
    return check_hip(hipGetLastError(), "k_fill launch");
}

int launch_to_precision(fr_plan *pl, const double *U, void *out, int64_t n, hipStream_t s)
{
    const unsigned g = grid_for(n);
    if (pl->precision == FR_F64)
        hipLaunchKernelGGL((k_to_prec<double>), dim3(g), dim3(TB), 0, s, U, (double *)out, n);
    else
        hipLaunchKernelGGL((k_to_prec<float>), dim3(g), dim3(TB), 0, s, U, (float *)out, n);
    return check_hip(hipGetLastError(), "k_to_prec launch");
}

int launch_bdf_const(fr_plan *pl, const double *Un, const double *Unm1, double dt, double *B,
                     hipStream_t s)
{
    const int ns = pl->m * pl->m * pl->m;
    hipLaunchKernelGGL(k_bdf_const, dim3(grid_for(pl->ne * 3 * ns)), dim3(TB), 0, s, Un, Unm1, dt,
                       B, pl->ne, ns);
    return check_hip(hipGetLastError(), "k_bdf_const launch");
}

int launch_final_sum(const double *partial, int nblocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(TB), 0, s, partial, nblocks, out);
    return check_hip(hipGetLastError(), "k_final_sum launch");
}

int launch_extrap(const double *Un, const double *Unm1, const double *Unm2, int order, int keep_ns,
                  double *G, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_extrap, dim3(grid_for(n)), dim3(TB), 0, s, Un, Unm1, Unm2, order, keep_ns,
                       G, n);
    return check_hip(hipGetLastError(), "k_extrap launch");
}

}  // namespace fr
