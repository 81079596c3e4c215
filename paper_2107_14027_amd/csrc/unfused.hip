// Unfused residual pipeline for gfx950: the six algorithmic stages of the
// paper's Table 1 as six kernels, every intermediate through HBM (the
// baseline the fused kernels are measured against).
//   k_u_project_lines  stage 1  U_f = solution projected to the six faces (13
//                      values), line tasks on an LDS-staged batch (k_u_project_flat:
//                      the same tile, one output value per lane, contiguous stores)
//   k_u_flux     stage 2  F_s  = transformed flux at the points (3 x 13 values)
//   k_u_div_lds  stage 3  partially corrected divergence of F_s, staged in LDS
//                         one direction at a time
//   k_u_common_lds   stage 4  common interface flux, one per unique face,
//                            face blocks staged in LDS
//   k_u_correct_lds  stage 5  correction with the common fluxes, staged in LDS
//   k_u_negsrc   stage 6  negate, scale by 1/det J, add the source
#include "fr_device.h"

namespace fr {
namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// Unfused pipeline: Table 1 stages as separate kernels through HBM.
// Buffers: Uf[6][ne][13][NF], Fs[3][ne][13][NS], Dv[ne][13][NS], FI[3][ne][13][NF],
// one after another, each starting 256-byte aligned
// ---------------------------------------------------------------------------

// Stage 2: VW consecutive points of one element per thread (VW = 1 unless
// m^3 is a multiple of the 16-byte vector width), every value read and
// written in coalesced (vector) accesses.
template <int P, typename T>
struct FluxShape {
    static constexpr int NS = (P + 1) * (P + 1) * (P + 1), W16 = 16 / (int)sizeof(T);
    static constexpr int VW = NS % W16 == 0 ? W16 : 1;
};

template <int P, typename T>
__global__ void __launch_bounds__(256) k_u_flux(const T *__restrict__ U, T *__restrict__ Fs,
                                                Consts<T> c, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M, VW = FluxShape<P, T>::VW;
    typedef T Vw __attribute__((ext_vector_type(VW)));
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * NS / VW) return;
    const int64_t e = t * VW / NS;
    const int q = (int)(t * VW - e * NS);
    Vw u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        u[v] = __builtin_nontemporal_load(reinterpret_cast<const Vw *>(U + (e * NV + v) * NS + q));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T nv[3] = {c.nvec[d][0], c.nvec[d][1], c.nvec[d][2]};
        Vw f[NV];
#pragma unroll
        for (int w = 0; w < VW; ++w) {
            T uw[NV], fw[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) uw[v] = u[v][w];
            flux_dot<T>(uw, nv, c.zeta, c.nu, c.invT, fw);
#pragma unroll
            for (int v = 0; v < NV; ++v) f[v][w] = fw[v];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v)
            __builtin_nontemporal_store(
                f[v], reinterpret_cast<Vw *>(Fs + (((int64_t)d * ne + e) * NV + v) * NS + q));
    }
}

// Which stage-2 kernel runs, per order and precision (measured).
#ifndef FR_UFLUX_LDS
#define FR_UFLUX_LDS 1
#endif
// Stage 2's outputs in 16-byte stores (VW consecutive values per lane): in
// single precision at p = 1 and 5, where that measured faster (0.52 -> 0.56
// and 0.57 -> 0.65 of 8 TB/s); one value per lane elsewhere.
#ifndef FR_UFLUX_VEC
#define FR_UFLUX_VEC 1
#endif
template <int P, typename T>
constexpr bool unfused_flux_vec()
{
    return FR_UFLUX_VEC != 0 && sizeof(T) == 4 && (P == 1 || P == 5);
}
template <int P, typename T>
constexpr bool unfused_flux_lds()
{
    return FR_UFLUX_LDS != 0;
}

// Stage 2 with contiguous writes: a workgroup copies a batch of E consecutive
// elements' states into LDS (one contiguous block), then writes the batch's
// block of F_s for each direction as one contiguous stream, every output value
// formed from the staged state with flux_dot's arithmetic for that component.
template <int P, typename T>
struct FluxLdsShape {
    static constexpr int NS = (P + 1) * (P + 1) * (P + 1), RAW = NV * NS, NT = 256;
    // about 24 KB of state per workgroup (one element where that is larger),
    // rounded down to a whole number of 16-byte chunks per batch where that
    // leaves at least one element, so that every batch starts on a 16-byte
    // boundary (else the copy is scalar)
    static constexpr int AL = 16 / sizeof(T);
    static constexpr int E0 = 24576 / (RAW * (int)sizeof(T)) > 0 ? 24576 / (RAW * (int)sizeof(T)) : 1;
    static constexpr int step = RAW % AL == 0 ? 1 : (RAW % 2 == 0 ? AL / 2 : AL);
    static constexpr int E = E0 >= step ? E0 / step * step : E0;
    static constexpr bool VEC = (E * RAW) % AL == 0;
};

// Component v of flux_dot(U, nv) at one point: u[w * NS] is variable w there.
// The same operations in the same order as flux_dot, so the same bits.
template <typename T, int NS>
__device__ __forceinline__ T flux_component(int v, const T *__restrict__ u, const T nv[3], T zeta,
                                            T nu, T invT)
{
    if (v == 0) {
        T vn = u[NS] * nv[0];
        vn = fma(u[2 * NS], nv[1], vn);
        vn = fma(u[3 * NS], nv[2], vn);
        return zeta * vn;
    }
    if (v < 4) {
        const int i = v - 1;
        T vn = u[NS] * nv[0];
        vn = fma(u[2 * NS], nv[1], vn);
        vn = fma(u[3 * NS], nv[2], vn);
        const T *S = u + (4 + 3 * i) * NS;
        T sn = S[0] * nv[0];
        sn = fma(S[NS], nv[1], sn);
        sn = fma(S[2 * NS], nv[2], sn);
        return fma(u[(1 + i) * NS], vn, fma(u[0], nv[i], -nu * sn));
    }
    const int i = (v - 4) / 3, k = v - 4 - 3 * i;
    return -invT * u[(1 + i) * NS] * nv[k];
}

template <int P, typename T>
__global__ void __launch_bounds__(256) k_u_flux_lds(const T *__restrict__ U, T *__restrict__ Fs,
                                                    Consts<T> c, int64_t ne)
{
    using FS = FluxLdsShape<P, T>;
    constexpr int NS = FS::NS, RAW = FS::RAW, E = FS::E, NT = FS::NT;
    __shared__ __align__(16) T sU[E * RAW];
    const int64_t e0 = (int64_t)blockIdx.x * E;
    const int nel = (int)min((int64_t)E, ne - e0);
    const int cnt = nel * RAW;
    const T *src = U + e0 * RAW;
    if constexpr (FS::VEC) {
        using V = typename V16<T>::type;
        constexpr int VW = 16 / sizeof(T);
        const int nv = cnt / VW;
        for (int k = threadIdx.x; k < nv; k += NT)
            reinterpret_cast<V *>(sU)[k] = __builtin_nontemporal_load(reinterpret_cast<const V *>(src) + k);
        for (int k = nv * VW + threadIdx.x; k < cnt; k += NT) sU[k] = __builtin_nontemporal_load(src + k);
    } else {
        for (int k = threadIdx.x; k < cnt; k += NT) sU[k] = __builtin_nontemporal_load(src + k);
    }
    __syncthreads();
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        const T nvd[3] = {c.nvec[d][0], c.nvec[d][1], c.nvec[d][2]};
        T *dst = Fs + ((int64_t)d * ne + e0) * RAW;
        int o0 = 0;
        if (unfused_flux_vec<P, T>() && (((uintptr_t)dst) & 15) == 0) {
            // VW consecutive outputs per lane, one 16-byte store
            using V = typename V16<T>::type;
            constexpr int VW = 16 / sizeof(T);
            const int nvec = cnt / VW;
            for (int k = threadIdx.x; k < nvec; k += NT) {
                V r;
#pragma unroll
                for (int w = 0; w < VW; ++w) {
                    const int o = k * VW + w;
                    const int el = o / RAW, rr = o - el * RAW;
                    const int v = rr / NS, q = rr - v * NS;
                    r[w] = flux_component<T, NS>(v, sU + el * RAW + q, nvd, c.zeta, c.nu, c.invT);
                }
                __builtin_nontemporal_store(r, reinterpret_cast<V *>(dst) + k);
            }
            o0 = nvec * VW;
        }
        for (int o = o0 + threadIdx.x; o < cnt; o += NT) {
            const int el = o / RAW, r = o - el * RAW;
            const int v = r / NS, q = r - v * NS;
            __builtin_nontemporal_store(
                flux_component<T, NS>(v, sU + el * RAW + q, nvd, c.zeta, c.nu, c.invT), dst + o);
        }
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

// Stage 6 in 16-byte vectors over the flat [ne][13][m^3] arrays (all three
// aligned): each component takes the variable of its own index, so a vector
// may hold the end of one variable's block and the start of the next (m^3 >=
// the vector width: at most one such boundary); U is read for the vectors that
// hold an auxiliary variable.  The last n mod VW values (n = 13 ne m^3) go one
// per thread to the first threads.  Per value the same arithmetic as k_u_negsrc.
template <int P, typename T>
__global__ void __launch_bounds__(256) k_u_negsrc_vec(const T *__restrict__ Dv, const T *__restrict__ U,
                                                      T *__restrict__ R, Consts<T> c, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M, VW = 16 / (int)sizeof(T);
    static_assert(NS >= VW, "a vector crosses at most one variable boundary");
    using V = typename V16<T>::type;
    const int64_t n = ne * NV * NS, nvec = n / VW;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nvec) {
        const int64_t k0 = t * VW, blk = k0 / NS;   // blk = e * 13 + v of component 0
        const int r0 = (int)(k0 - blk * NS);
        const int v0 = (int)(blk % NV), v1 = v0 + 1 == NV ? 0 : v0 + 1;
        int vw[VW];
        bool aux = false;
#pragma unroll
        for (int w = 0; w < VW; ++w) {
            vw[w] = r0 + w < NS ? v0 : v1;
            aux |= vw[w] >= 4;
        }
        const V dv = __builtin_nontemporal_load(reinterpret_cast<const V *>(Dv) + t);
        V r;
#pragma unroll
        for (int w = 0; w < VW; ++w) r[w] = -c.inv_det * dv[w];
        if (aux) {
            const V u = __builtin_nontemporal_load(reinterpret_cast<const V *>(U) + t);
#pragma unroll
            for (int w = 0; w < VW; ++w)
                if (vw[w] >= 4) r[w] -= c.invT * u[w];
        }
        __builtin_nontemporal_store(r, reinterpret_cast<V *>(R) + t);
    }
    if (t < n - nvec * VW) {
        const int64_t k = nvec * VW + t;
        T r = -c.inv_det * Dv[k];
        if ((k / NS) % NV >= 4) r -= c.invT * U[k];
        R[k] = r;
    }
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

// Stage 1 with contiguous stores: the same LDS tile, then for each direction d
// the outputs of both faces flat over (element, variable, face point), the
// layout of a face block, so that consecutive lanes store consecutive values.
// Each output is its line's projection with the operations of
// k_u_project_lines in the same order (the same bits).
template <int P, typename T>
__global__ void __launch_bounds__(256)
    k_u_project_flat(const T *__restrict__ U, T *__restrict__ Uf, const T *__restrict__ ops, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M, BL = NV * NF, NT = 256;
    constexpr int E = ProjectShape<P, T>::E;
    using LL = LinesLds<P, T>;
    using OL = OpsLayout<M>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sU = reinterpret_cast<T *>(smem_raw);
    const int64_t e0 = (int64_t)blockIdx.x * E;
    const int nel = (int)min((int64_t)E, ne - e0);
    tile_load<P, T, NT>(U + e0 * LL::raw, sU, nel);
    __syncthreads();
    T lm[M], lp[M];
#pragma unroll
    for (int l = 0; l < M; ++l) {
        lm[l] = ops[OL::lm + l];
        lp[l] = ops[OL::lp + l];
    }
    const int n = nel * BL;
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        const int str = d == 0 ? 1 : (d == 1 ? M : M * M);
        T *dm = Uf + ((int64_t)(2 * d) * ne + e0) * BL;
        T *dp = Uf + ((int64_t)(2 * d + 1) * ne + e0) * BL;
        for (int o = threadIdx.x; o < n; o += NT) {
            const int el = o / BL, r = o - el * BL, v = r / NF, L = r - v * NF;
            const int a = L % M, b = L / M;
            const int base = d == 0 ? M * L : (d == 1 ? a + M * M * b : L);
            const T *x = sU + el * LL::EP + v * NS + base;
            T am = T(0), ap = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) {
                am = fma(lm[l], x[l * str], am);
                ap = fma(lp[l], x[l * str], ap);
            }
            dm[o] = am;
            dp[o] = ap;
        }
    }
}

// Which stage-1 kernel runs: the flat form at p <= 2 (the line form's stores
// are runs of m^2 values scattered over 13 m^2-value blocks) and at p = 3 in
// single precision, the line form elsewhere (measured faster or equal).
#ifndef FR_UPROJECT_FLAT
#define FR_UPROJECT_FLAT 1
#endif
template <int P, typename T>
constexpr bool unfused_project_flat()
{
    return FR_UPROJECT_FLAT != 0 && (P <= 2 || (P == 3 && sizeof(T) == 4));
}

// The staging copies below move CU values per thread per round: all CU loads
// are issued before the first store, so each thread keeps CU loads in flight
// instead of waiting out one memory latency per value.
constexpr int CU = 8;

// Copy of n contiguous values from global src to LDS dst (16-byte vectors
// when both ends and the count allow).
template <typename T, int NT>
__device__ __forceinline__ void block_copy_in(const T *__restrict__ src, T *__restrict__ dst, int n)
{
    using V = typename V16<T>::type;
    constexpr int VW = 16 / sizeof(T);
    if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0 && n % VW == 0) {
        const V *vs = reinterpret_cast<const V *>(src);
        V *vd = reinterpret_cast<V *>(dst);
        for (int k0 = threadIdx.x; k0 < n / VW; k0 += CU * NT) {
            V r[CU];
#pragma unroll
            for (int u = 0; u < CU; ++u)
                if (k0 + u * NT < n / VW) r[u] = __builtin_nontemporal_load(vs + k0 + u * NT);
#pragma unroll
            for (int u = 0; u < CU; ++u)
                if (k0 + u * NT < n / VW) vd[k0 + u * NT] = r[u];
        }
    } else {
        for (int k0 = threadIdx.x; k0 < n; k0 += CU * NT) {
            T r[CU];
#pragma unroll
            for (int u = 0; u < CU; ++u)
                if (k0 + u * NT < n) r[u] = __builtin_nontemporal_load(src + k0 + u * NT);
#pragma unroll
            for (int u = 0; u < CU; ++u)
                if (k0 + u * NT < n) dst[k0 + u * NT] = r[u];
        }
    }
}

template <typename T, int NT>
__device__ __forceinline__ void block_copy_out(const T *__restrict__ src, T *__restrict__ dst, int n)
{
    using V = typename V16<T>::type;
    constexpr int VW = 16 / sizeof(T);
    if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0 && n % VW == 0) {
        for (int k = threadIdx.x; k < n / VW; k += NT)
            __builtin_nontemporal_store(reinterpret_cast<const V *>(src)[k], reinterpret_cast<V *>(dst) + k);
    } else {
        for (int k = threadIdx.x; k < n; k += NT) __builtin_nontemporal_store(src[k], dst + k);
    }
}

// Gather of nel blocks of BL contiguous values, block el from src + nb[el] * BL,
// into consecutive LDS blocks (16-byte vectors when BL allows).
template <typename T, int NT, int BL>
__device__ __forceinline__ void copy_blocks(const T *__restrict__ src, const int64_t *nb,
                                            T *__restrict__ dst, int nel)
{
    using V = typename V16<T>::type;
    constexpr int VW = 16 / sizeof(T);
    if constexpr ((BL * sizeof(T)) % 16 == 0) {
        constexpr int CB = BL / VW;
        for (int k0 = threadIdx.x; k0 < nel * CB; k0 += CU * NT) {
            V r[CU];
#pragma unroll
            for (int u = 0; u < CU; ++u) {
                const int k = k0 + u * NT;
                if (k < nel * CB) {
                    const int el = k / CB, o = k - el * CB;
                    r[u] = __builtin_nontemporal_load(reinterpret_cast<const V *>(src + nb[el] * BL) + o);
                }
            }
#pragma unroll
            for (int u = 0; u < CU; ++u)
                if (k0 + u * NT < nel * CB) reinterpret_cast<V *>(dst)[k0 + u * NT] = r[u];
        }
    } else {
        for (int k0 = threadIdx.x; k0 < nel * BL; k0 += CU * NT) {
            T r[CU];
#pragma unroll
            for (int u = 0; u < CU; ++u) {
                const int k = k0 + u * NT;
                if (k < nel * BL) {
                    const int el = k / BL, o = k - el * BL;
                    r[u] = __builtin_nontemporal_load(src + nb[el] * BL + o);
                }
            }
#pragma unroll
            for (int u = 0; u < CU; ++u)
                if (k0 + u * NT < nel * BL) dst[k0 + u * NT] = r[u];
        }
    }
}

template <int P, typename T>
struct DivShape {
    static constexpr int M = P + 1, NS = M * M * M;
    static constexpr int E = NS >= 256 ? 1 : 256 / NS;
    // one point per thread (p = 6: 343 points on 384 threads)
    static constexpr int NT = NS > 256 ? 64 * ((NS + 63) / 64) : 256;
    static constexpr int KP = (E * NS + NT - 1) / NT;   // points per thread
};

template <int P, typename T>
__global__ void __launch_bounds__((DivShape<P, T>::NT))
    k_u_div_lds(const T *__restrict__ Fs, T *__restrict__ Dv, const T *__restrict__ ops0, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M;
    constexpr int E = DivShape<P, T>::E, NT = DivShape<P, T>::NT, KP = DivShape<P, T>::KP;
    using OL = OpsLayout<M>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sF = reinterpret_cast<T *>(smem_raw);   // [E][13][NS] of one direction
    __shared__ T ops[M * M];                   // the operator Dt
    if (threadIdx.x < M * M) ops[threadIdx.x] = ops0[OL::Dt + threadIdx.x];
    const int64_t e0 = (int64_t)blockIdx.x * E;
    const int nel = (int)min((int64_t)E, ne - e0);
    T acc[KP][NV];
#pragma unroll
    for (int u = 0; u < KP; ++u)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[u][v] = T(0);
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
        if (dd) __syncthreads();
        block_copy_in<T, NT>(Fs + ((int64_t)dd * ne + e0) * NV * NS, sF, nel * NV * NS);
        __syncthreads();
        const int str = dd == 0 ? 1 : (dd == 1 ? M : M * M);
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            const int k = threadIdx.x + u * NT;
            if (k >= nel * NS) continue;
            const int el = k / NS, q = k - el * NS;
            const int id = dd == 0 ? q % M : (dd == 1 ? (q / M) % M : q / (M * M));
            const T *Fe = sF + el * NV * NS + q - id * str;
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int l = 0; l < M; ++l)
                    acc[u][v] = fma(ops[id * M + l], Fe[v * NS + l * str], acc[u][v]);
        }
    }
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const int k = threadIdx.x + u * NT;
        if (k >= nel * NS) continue;
        const int el = k / NS, q = k - el * NS;
#pragma unroll
        for (int v = 0; v < NV; ++v) Dv[((e0 + el) * NV + v) * NS + q] = acc[u][v];
    }
}

// Stage 4 with the face blocks staged in LDS: a workgroup takes direction d and
// E consecutive elements, copies their +d face blocks and the -d face blocks
// of their +d neighbours (contiguous runs), forms the common flux of every face
// point, puts it in place of the +d blocks in LDS and writes the E output
// blocks as one contiguous run.
template <int P, typename T>
struct CommonShape {
    static constexpr int M = P + 1, NF = M * M;
    // as many elements as keep the two face-block buffers within 48 KB
    static constexpr int EMAX = (48 * 1024) / (2 * NV * NF * (int)sizeof(T));
    static constexpr int E = EMAX < 32 ? EMAX : 32;
    static constexpr int NT = 64 * ((E * NF + 63) / 64);
};

template <int P, typename T>
__global__ void __launch_bounds__((CommonShape<P, T>::NT))
    k_u_common_lds(const T *__restrict__ Uf, T *__restrict__ FI, Consts<T> c, int nx, int ny, int nz)
{
    constexpr int M = P + 1, NF = M * M, BL = NV * NF;
    constexpr int E = CommonShape<P, T>::E, NT = CommonShape<P, T>::NT;
    __shared__ __align__(16) T sL[E * BL], sR[E * BL];
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t nb_blocks = (ne + E - 1) / E;
    const int d = (int)(blockIdx.x / nb_blocks);
    const int64_t e0 = (int64_t)(blockIdx.x - (int64_t)d * nb_blocks) * E;
    const int nel = (int)min((int64_t)E, ne - e0);
    block_copy_in<T, NT>(Uf + ((int64_t)(2 * d + 1) * ne + e0) * BL, sL, nel * BL);
    // the neighbours' -d blocks, one contiguous block per element
    __shared__ int64_t sNb[E];
    if (threadIdx.x < nel) sNb[threadIdx.x] = neighbour(e0 + threadIdx.x, 2 * d + 1, nx, ny, nz);
    __syncthreads();
    copy_blocks<T, NT, BL>(Uf + (int64_t)(2 * d) * ne * BL, sNb, sR, nel);
    __syncthreads();
    const int t = threadIdx.x;
    const bool act = t < nel * NF;
    const int el = act ? t / NF : 0, fp = act ? t - el * NF : 0;
    T out[NV];
    if (act) {
        T L[NV], Rr[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            L[v] = sL[el * BL + v * NF + fp];
            Rr[v] = sR[el * BL + v * NF + fp];
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
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T f = T(0.5) * (fl[v] + fr[v]);
            if (v < 4) f -= T(0.5) * lam * (Rr[v] - L[v]);
            out[v] = c.nmag[d] * f;
        }
    }
    __syncthreads();   // every thread has read its +d values
    if (act) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sL[el * BL + v * NF + fp] = out[v];
    }
    __syncthreads();
    block_copy_out<T, NT>(sL, FI + ((int64_t)d * ne + e0) * BL, nel * BL);
}

// Stage 5 with the common-flux blocks staged in LDS: a workgroup takes E
// consecutive elements, copies for each direction their own blocks (+d faces)
// and their -d neighbours' blocks, and corrects every point's 13 values.
template <int P, typename T>
struct CorrectShape {
    static constexpr int M = P + 1, NS = M * M * M;
    static constexpr int E = NS >= 256 ? 1 : (256 / NS < 16 ? 256 / NS : 16);
    static constexpr int NT = 256;
};

template <int P, typename T>
__global__ void __launch_bounds__(256)
    k_u_correct_lds(T *__restrict__ Dv, const T *__restrict__ FI, const T *__restrict__ ops, int nx,
                    int ny, int nz)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M, BL = NV * NF;
    constexpr int E = CorrectShape<P, T>::E, NT = CorrectShape<P, T>::NT;
    using OL = OpsLayout<M>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sP = reinterpret_cast<T *>(smem_raw);   // [3][E][BL] own (+d) blocks
    T *sM = sP + 3 * E * BL;                    // [3][E][BL] -d neighbours' blocks
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t e0 = (int64_t)blockIdx.x * E;
    const int nel = (int)min((int64_t)E, ne - e0);
    __shared__ int64_t sNb[3][E];
    if (threadIdx.x < 3 * nel)
        sNb[threadIdx.x / nel][threadIdx.x % nel] =
            neighbour(e0 + threadIdx.x % nel, 2 * (threadIdx.x / nel), nx, ny, nz);
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        block_copy_in<T, NT>(FI + ((int64_t)d * ne + e0) * BL, sP + d * E * BL, nel * BL);
        copy_blocks<T, NT, BL>(FI + (int64_t)d * ne * BL, sNb[d], sM + d * E * BL, nel);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nel * NS; k += NT) {
        const int el = k / NS, q = k - el * NS;
        const int idx[3] = {q % M, (q / M) % M, q / (M * M)};
        const int fps[3] = {idx[1] + M * idx[2], idx[0] + M * idx[2], idx[0] + M * idx[1]};
        T *Dq = Dv + ((e0 + el) * NV) * NS + q;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T acc = Dq[v * NS];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T fm = sM[(d * E + el) * BL + v * NF + fps[d]];
                const T fpl = sP[(d * E + el) * BL + v * NF + fps[d]];
                acc = fma(ops[OL::gl + idx[d]], fm, fma(ops[OL::gr + idx[d]], fpl, acc));
            }
            Dq[v * NS] = acc;
        }
    }
}

// Stage 5 without LDS: one thread per point reads its six face values of every
// variable straight from the common-flux blocks (its own +d blocks and the -d
// neighbours' blocks) and corrects its 13 divergence values in place.
template <int P, typename T>
__global__ void __launch_bounds__(256)
    k_u_correct_direct(T *__restrict__ Dv, const T *__restrict__ FI, const T *__restrict__ ops, int nx,
                       int ny, int nz)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M, BL = NV * NF;
    using OL = OpsLayout<M>;
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * NS) return;
    const int64_t e = t / NS;
    const int q = (int)(t - e * NS);
    const int idx[3] = {q % M, (q / M) % M, q / (M * M)};
    const int fps[3] = {idx[1] + M * idx[2], idx[0] + M * idx[2], idx[0] + M * idx[1]};
    const T *fm[3], *fpl[3];
    T glv[3], grv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t nb = neighbour(e, 2 * d, nx, ny, nz);
        fm[d] = FI + ((int64_t)d * ne + nb) * BL + fps[d];
        fpl[d] = FI + ((int64_t)d * ne + e) * BL + fps[d];
        glv[d] = ops[OL::gl + idx[d]];
        grv[d] = ops[OL::gr + idx[d]];
    }
    T *Dq = Dv + (e * NV) * NS + q;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T acc = Dq[v * NS];
#pragma unroll
        for (int d = 0; d < 3; ++d) acc = fma(glv[d], fm[d][v * NF], fma(grv[d], fpl[d][v * NF], acc));
        Dq[v * NS] = acc;
    }
}

// Which stage-5 kernel runs: without LDS at p = 3 in single precision, staged
// in LDS elsewhere (measured faster).
#ifndef FR_UCORRECT_DIRECT
#define FR_UCORRECT_DIRECT 1
#endif

template <int P, typename T>
constexpr bool unfused_correct_direct()
{
    return FR_UCORRECT_DIRECT != 0 && P == 3 && sizeof(T) == 4;
}

// Length of one stage buffer in the unfused scratch, rounded up to 64 values so
// that every buffer starts 256-byte aligned (the 16-byte vector paths need it).
inline size_t ubuf(size_t n)
{
    return (n + 63) & ~(size_t)63;
}

template <int P, typename T>
int unfused_impl(fr_plan *pl, const T *U, T *R, T *scratch, const T *ops, const Consts<T> &c,
                 hipStream_t s)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    const int64_t ne = pl->ne;
    T *Uf = scratch;
    T *Fs = Uf + ubuf((size_t)6 * ne * NV * NF);
    T *Dv = Fs + ubuf((size_t)3 * ne * NV * NS);
    T *FI = Dv + ubuf((size_t)ne * NV * NS);
    const int nt = 256;
    auto g = [&](int64_t n) { return dim3((unsigned)((n + nt - 1) / nt)); };
    {
        // LDS-staged line tasks (dynamic LDS above 64 KB at p = 4, 5 in double)
        using PS = ProjectShape<P, T>;
        const size_t lds = (size_t)PS::E * LinesLds<P, T>::EP * sizeof(T);
        int &set = pl->unfused_attr[P][sizeof(T) == 8];
        if (!set) {
            for (const void *k : {(const void *)k_u_project_lines<P, T>, (const void *)k_u_project_flat<P, T>})
                if (int rc = check_hip(
                        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                        "hipFuncSetAttribute"))
                    return rc;
            set = 1;
        }
        ProfScope ps(pl, FR_K_U_PROJECT, s);
        if (unfused_project_flat<P, T>())
            hipLaunchKernelGGL((k_u_project_flat<P, T>), dim3((unsigned)((ne + PS::E - 1) / PS::E)),
                               dim3(256), lds, s, U, Uf, ops, ne);
        else
            hipLaunchKernelGGL((k_u_project_lines<P, T>), dim3((unsigned)((ne + PS::E - 1) / PS::E)),
                               dim3(PS::NT), lds, s, U, Uf, ops, ne);
    }
    {
        ProfScope ps(pl, FR_K_U_FLUX, s);
        if (unfused_flux_lds<P, T>())
            hipLaunchKernelGGL((k_u_flux_lds<P, T>),
                               dim3((unsigned)((ne + FluxLdsShape<P, T>::E - 1) / FluxLdsShape<P, T>::E)),
                               dim3(FluxLdsShape<P, T>::NT), 0, s, U, Fs, c, ne);
        else
            hipLaunchKernelGGL((k_u_flux<P, T>), g(ne * NS / FluxShape<P, T>::VW), dim3(nt), 0, s, U,
                               Fs, c, ne);
    }
    {
        ProfScope ps(pl, FR_K_U_DIV, s);
        using DS = DivShape<P, T>;
        hipLaunchKernelGGL((k_u_div_lds<P, T>), dim3((unsigned)((ne + DS::E - 1) / DS::E)),
                           dim3(DS::NT), (size_t)DS::E * NV * NS * sizeof(T), s, Fs, Dv, ops, ne);
    }
    {
        ProfScope ps(pl, FR_K_U_COMMON, s);
        using CS = CommonShape<P, T>;
        hipLaunchKernelGGL((k_u_common_lds<P, T>), dim3((unsigned)(3 * ((ne + CS::E - 1) / CS::E))),
                           dim3(CS::NT), 0, s, Uf, FI, c, pl->nx, pl->ny, pl->nz);
    }
    {
        ProfScope ps(pl, FR_K_U_CORRECT, s);
        using RS = CorrectShape<P, T>;
        if (unfused_correct_direct<P, T>())
            hipLaunchKernelGGL((k_u_correct_direct<P, T>), g(ne * NS), dim3(nt), 0, s, Dv, FI, ops,
                               pl->nx, pl->ny, pl->nz);
        else
            hipLaunchKernelGGL((k_u_correct_lds<P, T>), dim3((unsigned)((ne + RS::E - 1) / RS::E)),
                               dim3(RS::NT), (size_t)6 * RS::E * NV * NF * sizeof(T), s, Dv, FI, ops,
                               pl->nx, pl->ny, pl->nz);
    }
    {
        ProfScope ps(pl, FR_K_U_NEGSRC, s);
        if ((((uintptr_t)Dv | (uintptr_t)U | (uintptr_t)R) & 15) == 0)
            hipLaunchKernelGGL((k_u_negsrc_vec<P, T>), g((ne * NV * NS + 16 / sizeof(T) - 1) /
                                                        (16 / sizeof(T))),
                               dim3(nt), 0, s, Dv, U, R, c, ne);
        else
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
    const size_t ne = (size_t)pl->ne;
    const size_t n = ubuf(ne * NV * 6 * NF) + ubuf(ne * NV * 3 * NS) + ubuf(ne * NV * NS) +
                     ubuf(ne * NV * 3 * NF);
    if (int rc = ensure_scratch(pl->unfused, n * esz)) return rc;
    if (pl->precision == FR_F64)
        return dispatch_unfused<double>(pl, (const double *)U, (double *)R,
                                        (double *)pl->unfused.ptr, (const double *)pl->ops64,
                                        pl->c64, s);
    return dispatch_unfused<float>(pl, (const float *)U, (float *)R, (float *)pl->unfused.ptr,
                                   (const float *)pl->ops32, pl->c32, s);
}

}  // namespace fr
