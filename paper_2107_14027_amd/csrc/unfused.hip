// Unfused residual pipeline for gfx950: the six algorithmic stages of the
// paper's Table 1 as six kernels, every intermediate through HBM (the
// baseline the fused kernels are measured against).
//   k_u_project_lines  stage 1  U_f = solution projected to the six faces (13
//                      values), line tasks on an LDS-staged batch
//   k_u_flux     stage 2  F_s  = transformed flux at the points (3 x 13 values)
//   k_u_div_lds  stage 3  partially corrected divergence of F_s, staged in LDS
//                         one variable at a time
//   k_u_common   stage 4  common interface flux, one per unique face
//   k_u_correct  stage 5  correction with the common fluxes
//   k_u_negsrc   stage 6  negate, scale by 1/det J, add the source
#include "fr_device.h"

namespace fr {
namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// Unfused pipeline: Table 1 stages as separate kernels through HBM.
// Buffers: Uf[6][ne][13][NF], Fs[3][ne][13][NS], Dv[ne][13][NS], FI[3][ne][13][NF]
// ---------------------------------------------------------------------------

template <int P, typename T>
__global__ void __launch_bounds__(256) k_u_flux(const T *__restrict__ U, T *__restrict__ Fs,
                                                Consts<T> c, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * NS) return;
    const int64_t e = t / NS;
    const int q = (int)(t - e * NS);
    T u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[(e * NV + v) * NS + q];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T nv[3] = {c.nvec[d][0], c.nvec[d][1], c.nvec[d][2]};
        T f[NV];
        flux_dot<T>(u, nv, c.zeta, c.nu, c.invT, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fs[(((int64_t)d * ne + e) * NV + v) * NS + q] = f[v];
    }
}

// Common flux for the plus face of every element (one per unique face),
// all 13 variables, transformed by |n_d|.
template <int P, typename T>
__global__ void __launch_bounds__(256) k_u_common(const T *__restrict__ Uf, T *__restrict__ FI,
                                                  Consts<T> c, int nx, int ny, int nz)
{
    constexpr int M = P + 1, NF = M * M;
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * 3 * NF) return;
    const int fp = (int)(t % NF);
    const int64_t r = t / NF;
    const int64_t e = r % ne;
    const int d = (int)(r / ne);
    const int64_t nb = neighbour(e, 2 * d + 1, nx, ny, nz);
    T L[NV], Rr[NV];
    for (int v = 0; v < NV; ++v) {
        L[v] = Uf[(((int64_t)(2 * d + 1) * ne + e) * NV + v) * NF + fp];
        Rr[v] = Uf[(((int64_t)(2 * d) * ne + nb) * NV + v) * NF + fp];
    }
    T nh[3] = {c.nhat[d][0], c.nhat[d][1], c.nhat[d][2]};
    T fl[NV], fr[NV];
    flux_dot<T>(L, nh, c.zeta, c.nu, c.invT, fl);
    flux_dot<T>(Rr, nh, c.zeta, c.nu, c.invT, fr);
    T vnl = L[1] * nh[0] + L[2] * nh[1] + L[3] * nh[2];
    T vnr = Rr[1] * nh[0] + Rr[2] * nh[1] + Rr[3] * nh[2];
    const T al = fabs(vnl) + sqrt(vnl * vnl + c.zeta);
    const T ar = fabs(vnr) + sqrt(vnr * vnr + c.zeta);
    const T lam = al > ar ? al : ar;
    T *dst = FI + (((int64_t)d * ne + e) * NV) * NF + fp;
    for (int v = 0; v < NV; ++v) {
        T f = T(0.5) * (fl[v] + fr[v]);
        if (v < 4) f -= T(0.5) * lam * (Rr[v] - L[v]);
        dst[v * NF] = c.nmag[d] * f;
    }
}

template <int P, typename T>
__global__ void __launch_bounds__(256) k_u_correct(T *__restrict__ Dv, const T *__restrict__ FI,
                                                   const T *__restrict__ ops, int nx, int ny,
                                                   int nz)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    using OL = OpsLayout<M>;
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * NS) return;
    const int64_t e = t / NS;
    const int q = (int)(t - e * NS);
    const int idx[3] = {q % M, (q / M) % M, q / (M * M)};
    const int fa[3] = {idx[1], idx[0], idx[0]}, fb[3] = {idx[2], idx[2], idx[1]};
    int64_t lo[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) lo[d] = neighbour(e, 2 * d, nx, ny, nz);
    for (int v = 0; v < NV; ++v) {
        T acc = Dv[(e * NV + v) * NS + q];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int fp = fa[d] + M * fb[d];
            const T fm = FI[(((int64_t)d * ne + lo[d]) * NV + v) * NF + fp];
            const T fpl = FI[(((int64_t)d * ne + e) * NV + v) * NF + fp];
            acc = fma(ops[OL::gl + idx[d]], fm, fma(ops[OL::gr + idx[d]], fpl, acc));
        }
        Dv[(e * NV + v) * NS + q] = acc;
    }
}

template <int P, typename T>
__global__ void __launch_bounds__(256) k_u_negsrc(const T *__restrict__ Dv, const T *__restrict__ U,
                                                  T *__restrict__ R, Consts<T> c, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * NV * NS) return;
    const int v = (int)((t / NS) % NV);
    T r = -c.inv_det * Dv[t];
    if (v >= 4) r -= c.invT * U[t];
    R[t] = r;
}

// Stage 1 as line tasks: a workgroup copies a batch of E consecutive elements
// into LDS (the line form's tile), a lane owns one line of one direction d of
// one element and projects all 13 variables to both of its ends.
template <int P, typename T>
struct ProjectShape {
    static constexpr int M = P + 1, NF = M * M;
    static constexpr int E = P == 1 ? 16 : (P == 2 ? 7 : (P == 3 ? 4 : (P == 4 ? 5 : (P == 5 ? 3 : 1))));
    static constexpr int W = (E * NF + 63) / 64, NT = 192 * W;
};

template <int P, typename T>
__global__ void __launch_bounds__((ProjectShape<P, T>::NT))
    k_u_project_lines(const T *__restrict__ U, T *__restrict__ Uf, const T *__restrict__ ops,
                      int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    constexpr int E = ProjectShape<P, T>::E, W = ProjectShape<P, T>::W, NT = ProjectShape<P, T>::NT;
    using LL = LinesLds<P, T>;
    using OL = OpsLayout<M>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sU = reinterpret_cast<T *>(smem_raw);
    const int64_t e0 = (int64_t)blockIdx.x * E;
    const int nel = (int)min((int64_t)E, ne - e0);
    tile_load<P, T, NT>(U + e0 * LL::raw, sU, nel);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int d = wave / W;
    const int t = (wave - d * W) * 64 + (threadIdx.x & 63);
    const int el = t / NF, L = t - el * NF;
    if (el >= nel) return;
    T lm[M], lp[M];
#pragma unroll
    for (int l = 0; l < M; ++l) {
        lm[l] = ops[OL::lm + l];
        lp[l] = ops[OL::lp + l];
    }
    const int a = L % M, b = L / M;
    const int str = d == 0 ? 1 : (d == 1 ? M : M * M);
    const int base = d == 0 ? M * L : (d == 1 ? a + M * M * b : L);
    const T *Ue = sU + el * LL::EP + base;
    const int64_t e = e0 + el;
    T *dm = Uf + (((int64_t)(2 * d) * ne + e) * NV) * NF + L;
    T *dp = Uf + (((int64_t)(2 * d + 1) * ne + e) * NV) * NF + L;
    for (int v = 0; v < NV; ++v) {
        T am = T(0), ap = T(0);
#pragma unroll
        for (int l = 0; l < M; ++l) {
            const T x = Ue[v * NS + l * str];
            am = fma(lm[l], x, am);
            ap = fma(lp[l], x, ap);
        }
        dm[v * NF] = am;
        dp[v * NF] = ap;
    }
}

// Stage 3 with the element's flux staged in LDS one variable at a time: a
// workgroup takes E elements; per variable it copies the three directions'
// transformed flux of its elements (contiguous runs of m^3 values) into LDS and
// every thread contracts its points' three lines.
template <int P, typename T>
struct DivShape {
    static constexpr int M = P + 1, NS = M * M * M;
    static constexpr int E = NS >= 256 ? 1 : 256 / NS;
    static constexpr int NT = E * NS < 256 ? (E * NS + 63) / 64 * 64 : 256;
};

template <int P, typename T>
__global__ void __launch_bounds__((DivShape<P, T>::NT))
    k_u_div_lds(const T *__restrict__ Fs, T *__restrict__ Dv, const T *__restrict__ ops, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M;
    constexpr int E = DivShape<P, T>::E, NT = DivShape<P, T>::NT;
    using OL = OpsLayout<M>;
    __shared__ T sF[3][E][NS];
    const int64_t e0 = (int64_t)blockIdx.x * E;
    const int nel = (int)min((int64_t)E, ne - e0);
    for (int v = 0; v < NV; ++v) {
        if (v) __syncthreads();
        for (int k = threadIdx.x; k < 3 * nel * NS; k += NT) {
            const int dd = k / (nel * NS), r = k - dd * (nel * NS);
            const int el = r / NS, q = r - el * NS;
            sF[dd][el][q] = Fs[(((int64_t)dd * ne + e0 + el) * NV + v) * NS + q];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nel * NS; k += NT) {
            const int el = k / NS, q = k - el * NS;
            const int i = q % M, j = (q / M) % M, kk = q / (M * M);
            T acc = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) acc = fma(ops[OL::Dt + i * M + l], sF[0][el][q - i + l], acc);
#pragma unroll
            for (int l = 0; l < M; ++l) acc = fma(ops[OL::Dt + j * M + l], sF[1][el][q + (l - j) * M], acc);
#pragma unroll
            for (int l = 0; l < M; ++l)
                acc = fma(ops[OL::Dt + kk * M + l], sF[2][el][q + (l - kk) * M * M], acc);
            Dv[((e0 + el) * NV + v) * NS + q] = acc;
        }
    }
}

template <int P, typename T>
int unfused_impl(fr_plan *pl, const T *U, T *R, T *scratch, const T *ops, const Consts<T> &c,
                 hipStream_t s)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    const int64_t ne = pl->ne;
    T *Uf = scratch;
    T *Fs = Uf + (size_t)6 * ne * NV * NF;
    T *Dv = Fs + (size_t)3 * ne * NV * NS;
    T *FI = Dv + (size_t)ne * NV * NS;
    const int nt = 256;
    auto g = [&](int64_t n) { return dim3((unsigned)((n + nt - 1) / nt)); };
    {
        // LDS-staged line tasks (dynamic LDS above 64 KB at p = 4, 5 in double)
        using PS = ProjectShape<P, T>;
        const size_t lds = (size_t)PS::E * LinesLds<P, T>::EP * sizeof(T);
        int &set = pl->unfused_attr[P][sizeof(T) == 8];
        if (!set) {
            if (int rc = check_hip(hipFuncSetAttribute((const void *)k_u_project_lines<P, T>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)lds),
                                   "hipFuncSetAttribute"))
                return rc;
            set = 1;
        }
        ProfScope ps(pl, FR_K_U_PROJECT, s);
        hipLaunchKernelGGL((k_u_project_lines<P, T>), dim3((unsigned)((ne + PS::E - 1) / PS::E)),
                           dim3(PS::NT), lds, s, U, Uf, ops, ne);
    }
    {
        ProfScope ps(pl, FR_K_U_FLUX, s);
        hipLaunchKernelGGL((k_u_flux<P, T>), g(ne * NS), dim3(nt), 0, s, U, Fs, c, ne);
    }
    {
        ProfScope ps(pl, FR_K_U_DIV, s);
        using DS = DivShape<P, T>;
        hipLaunchKernelGGL((k_u_div_lds<P, T>), dim3((unsigned)((ne + DS::E - 1) / DS::E)),
                           dim3(DS::NT), 0, s, Fs, Dv, ops, ne);
    }
    {
        ProfScope ps(pl, FR_K_U_COMMON, s);
        hipLaunchKernelGGL((k_u_common<P, T>), g(ne * 3 * NF), dim3(nt), 0, s, Uf, FI, c, pl->nx,
                           pl->ny, pl->nz);
    }
    {
        ProfScope ps(pl, FR_K_U_CORRECT, s);
        hipLaunchKernelGGL((k_u_correct<P, T>), g(ne * NS), dim3(nt), 0, s, Dv, FI, ops, pl->nx,
                           pl->ny, pl->nz);
    }
    {
        ProfScope ps(pl, FR_K_U_NEGSRC, s);
        hipLaunchKernelGGL((k_u_negsrc<P, T>), g(ne * NV * NS), dim3(nt), 0, s, Dv, U, R, c, ne);
    }
    return check_hip(hipGetLastError(), "unfused launch");
}

template <typename T>
int dispatch_unfused(fr_plan *pl, const T *U, T *R, T *scr, const T *ops, const Consts<T> &c,
                     hipStream_t s)
{
    switch (pl->p) {
        case 1: return unfused_impl<1, T>(pl, U, R, scr, ops, c, s);
        case 2: return unfused_impl<2, T>(pl, U, R, scr, ops, c, s);
        case 3: return unfused_impl<3, T>(pl, U, R, scr, ops, c, s);
        case 4: return unfused_impl<4, T>(pl, U, R, scr, ops, c, s);
        case 5: return unfused_impl<5, T>(pl, U, R, scr, ops, c, s);
        case 6: return unfused_impl<6, T>(pl, U, R, scr, ops, c, s);
    }
    return set_error(FR_EINVAL, "order %d", pl->p);
}

}  // namespace

int launch_residual_unfused(fr_plan *pl, const void *U, void *R, hipStream_t s)
{
    const int m = pl->m;
    const size_t NS = (size_t)m * m * m, NF = (size_t)m * m;
    const size_t esz = pl->precision == FR_F64 ? 8 : 4;
    const size_t n = (size_t)pl->ne * NV * (6 * NF + 3 * NS + NS + 3 * NF);
    if (int rc = ensure_scratch(pl->unfused, n * esz)) return rc;
    if (pl->precision == FR_F64)
        return dispatch_unfused<double>(pl, (const double *)U, (double *)R,
                                        (double *)pl->unfused.ptr, (const double *)pl->ops64,
                                        pl->c64, s);
    return dispatch_unfused<float>(pl, (const float *)U, (float *)R, (float *)pl->unfused.ptr,
                                   (const float *)pl->ops32, pl->c32, s);
}

}  // namespace fr
