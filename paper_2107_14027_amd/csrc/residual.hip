// Residual kernels for gfx950: R = -div F + S of ACM-HD by flux reconstruction
// on constant-Jacobian hexahedra (paper Sec. 2.1, 2.2; Table 1 stages 1-6).
//
// Fused path (two launches per residual):
//   k_trace   stage 1 only for what the neighbours need: per element and face,
//             7 trace values per face point (P, V, (S n_hat)) -> trace buffer
//             TR[6][ne][7][m^2].  Reads U once (13 values/point).
//   k_fused   stages 2-6 for a block of E elements staged in LDS: flux at the
//             points, partially corrected divergence along the three line
//             families, own face traces recomputed on chip, Rusanov/mean common
//             flux against the neighbour traces, correction, source.  Reads U
//             once, the neighbours' traces once, writes R once.
// Unfused path (six launches, Table 1 as written, every intermediate in HBM):
//   k_u_project, k_u_flux, k_u_div, k_u_common, k_u_correct, k_u_negsrc.
//
// Face numbering: f = 2 d + s (d = direction, s = 0 minus / 1 plus side).
// A face point is (a, b): the two tangential point indices in increasing
// direction order, flattened a + m b.  Every element has the same
// orientation, so face point (a, b) of face (d, 1) meets point (a, b) of the
// neighbour's face (d, 0).
#include "fr_internal.h"

namespace fr {
namespace {

template <int M>
__device__ __forceinline__ int qidx(int i, int j, int k) { return i + M * (j + M * k); }

template <int M>
__device__ __forceinline__ int line_pt(int d, int a, int b, int l)
{
    return d == 0 ? qidx<M>(l, a, b) : (d == 1 ? qidx<M>(a, l, b) : qidx<M>(a, b, l));
}

__device__ __forceinline__ int64_t neighbour(int64_t e, int f, int nx, int ny, int nz)
{
    int ex = (int)(e % nx);
    int64_t r = e / nx;
    int ey = (int)(r % ny);
    int ez = (int)(r / ny);
    const int d = f >> 1, up = f & 1;
    if (d == 0) ex = up ? (ex + 1 == nx ? 0 : ex + 1) : (ex == 0 ? nx - 1 : ex - 1);
    else if (d == 1) ey = up ? (ey + 1 == ny ? 0 : ey + 1) : (ey == 0 ? ny - 1 : ey - 1);
    else ez = up ? (ez + 1 == nz ? 0 : ez + 1) : (ez == 0 ? nz - 1 : ez - 1);
    return (int64_t)ex + (int64_t)nx * ((int64_t)ey + (int64_t)ny * ez);
}

// Face trace of one element at face point (a, b) of direction d, using the
// endpoint basis values lf[] (l(-1) or l(+1)).  Written as an explicit fma
// chain so that every kernel computing the same trace gets the same bits.
template <int M, typename T>
__device__ __forceinline__ void face_trace(const T *__restrict__ Ue, int d, int a, int b,
                                           const T *__restrict__ lf, const T nh[3], T tr[NTR])
{
    constexpr int NS = M * M * M;
#pragma unroll
    for (int c = 0; c < NTR; ++c) tr[c] = T(0);
#pragma unroll
    for (int l = 0; l < M; ++l) {
        const int q = line_pt<M>(d, a, b, l);
        const T wl = lf[l];
#pragma unroll
        for (int v = 0; v < 4; ++v) tr[v] = fma(wl, Ue[v * NS + q], tr[v]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T sn = Ue[(4 + 3 * i) * NS + q] * nh[0];
            sn = fma(Ue[(5 + 3 * i) * NS + q], nh[1], sn);
            sn = fma(Ue[(6 + 3 * i) * NS + q], nh[2], sn);
            tr[4 + i] = fma(wl, sn, tr[4 + i]);
        }
    }
}

// Common normal flux through a face of direction d between the state L on the
// minus side and R on the plus side (normal n_hat_d pointing from L to R),
// already multiplied by |n_d| (the reference-face scaling).  Outputs:
//   out[0]     Rusanov dissipation on P: -|n| lambda (P_R - P_L) / 2
//              (the central part of the P flux, zeta n.V_mean, is carried by
//               the corrected velocity derivatives)
//   out[1..3]  momentum common flux
//   out[4..6]  mean velocity (V_L + V_R) / 2 (the auxiliary equations' mean flux
//              is -(1/T) n_d,k V_mean_i)
template <typename T>
__device__ __forceinline__ void common_flux(const T L[NTR], const T R[NTR], const T nh[3],
                                            T nmag, T zeta, T nu, T out[NTR])
{
    T vnl = L[1] * nh[0];
    vnl = fma(L[2], nh[1], vnl);
    vnl = fma(L[3], nh[2], vnl);
    T vnr = R[1] * nh[0];
    vnr = fma(R[2], nh[1], vnr);
    vnr = fma(R[3], nh[2], vnr);
    const T al = fabs(vnl) + sqrt(fma(vnl, vnl, zeta));
    const T ar = fabs(vnr) + sqrt(fma(vnr, vnr, zeta));
    const T lam = al > ar ? al : ar;
    const T hm = T(0.5) * nmag;
    out[0] = -hm * lam * (R[0] - L[0]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T fl = fma(L[1 + i], vnl, fma(L[0], nh[i], -nu * L[4 + i]));
        T fr = fma(R[1 + i], vnr, fma(R[0], nh[i], -nu * R[4 + i]));
        out[1 + i] = hm * (fl + fr - lam * (R[1 + i] - L[1 + i]));
        out[4 + i] = T(0.5) * (L[1 + i] + R[1 + i]);
    }
}

// Cooperative copy global -> LDS with 16-byte vectors where alignment allows.
template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = double2; };
template <> struct Vec16<float> { using type = float4; };

template <typename T>
__device__ __forceinline__ void copy_to_lds(T *__restrict__ dst, const T *__restrict__ src, int n)
{
    using V = typename Vec16<T>::type;
    constexpr int W = 16 / sizeof(T);
    if ((((uintptr_t)src) & 15) == 0 && (((uintptr_t)dst) & 15) == 0) {
        const int nv = n / W;
        const V *s = reinterpret_cast<const V *>(src);
        V *d = reinterpret_cast<V *>(dst);
        for (int t = threadIdx.x; t < nv; t += blockDim.x) d[t] = s[t];
        for (int t = nv * W + threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
    } else {
        for (int t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
    }
}

// ---------------------------------------------------------------------------
// k_trace: stage 1 restricted to the 7 values the common flux needs.
// ---------------------------------------------------------------------------
template <int P, typename T>
__global__ void __launch_bounds__(256) k_trace(const T *__restrict__ U, T *__restrict__ TR,
                                               const T *__restrict__ ops, Consts<T> c, int64_t ne,
                                               int E)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    using OL = OpsLayout<M>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sU = reinterpret_cast<T *>(smem_raw);
    T *sl = sU + (size_t)E * NV * NS;  // lm[M], lp[M]
    const int64_t e0 = (int64_t)blockIdx.x * E;
    const int nel = (int)min<int64_t>(E, ne - e0);
    copy_to_lds(sU, U + e0 * NV * NS, nel * NV * NS);
    if (threadIdx.x < 2 * M) sl[threadIdx.x] = ops[OL::lm + threadIdx.x];
    __syncthreads();
    const int per_face = nel * NF;
    for (int t = threadIdx.x; t < 6 * per_face; t += blockDim.x) {
        const int f = t / per_face, r = t - f * per_face;
        const int el = r / NF, fp = r - el * NF;
        const int d = f >> 1, s = f & 1;
        const int a = fp % M, b = fp / M;
        T nh[3] = {c.nhat[d][0], c.nhat[d][1], c.nhat[d][2]};
        T tr[NTR];
        face_trace<M, T>(sU + el * NV * NS, d, a, b, sl + s * M, nh, tr);
        T *dst = TR + (((int64_t)f * ne + e0 + el) * NTR) * NF + fp;
#pragma unroll
        for (int cc = 0; cc < NTR; ++cc) dst[cc * NF] = tr[cc];
    }
}

// ---------------------------------------------------------------------------
// k_fused: stages 2-6 for E elements per workgroup.
// LDS: sU[E][13][NS] | sF[E][9][NS] | sFI[E][6][7][NF] | ops
// ---------------------------------------------------------------------------
template <int P, typename T>
__global__ void __launch_bounds__(256) k_fused(const T *__restrict__ U, const T *__restrict__ TR,
                                               T *__restrict__ R, const T *__restrict__ ops,
                                               Consts<T> c, int nx, int ny, int nz, int E)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    using OL = OpsLayout<M>;
    const int64_t ne = (int64_t)nx * ny * nz;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sU = reinterpret_cast<T *>(smem_raw);
    T *sF = sU + (size_t)E * NV * NS;
    T *sFI = sF + (size_t)E * 9 * NS;
    T *sop = sFI + (size_t)E * 6 * NTR * NF;

    const int64_t e0 = (int64_t)blockIdx.x * E;
    const int nel = (int)min<int64_t>(E, ne - e0);

    // ---- load: own states, neighbour traces (into sFI as the outer state), operators
    copy_to_lds(sU, U + e0 * NV * NS, nel * NV * NS);
    for (int t = threadIdx.x; t < OL::size; t += blockDim.x) sop[t] = ops[t];
    {
        const int chunk = NTR * NF;
        const int per_face = nel * chunk;
        for (int t = threadIdx.x; t < 6 * per_face; t += blockDim.x) {
            const int f = t / per_face, r = t - f * per_face;
            const int el = r / chunk, o = r - el * chunk;
            const int64_t nb = neighbour(e0 + el, f, nx, ny, nz);
            sFI[(el * 6 + f) * chunk + o] = TR[((int64_t)(f ^ 1) * ne + nb) * chunk + o];
        }
    }
    __syncthreads();

    // ---- stage 2: transformed momentum flux at every point,
    //      Fhat_{d,i} = u_i (n_d . V) + P n_d,i - nu sum_j n_d,j S_ij
    for (int t = threadIdx.x; t < nel * NS; t += blockDim.x) {
        const int el = t / NS, q = t - el * NS;
        const T *Ue = sU + el * NV * NS;
        T u[3] = {Ue[1 * NS + q], Ue[2 * NS + q], Ue[3 * NS + q]};
        const T Pq = Ue[q];
        T S[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) S[v] = Ue[(4 + v) * NS + q];
        T *Fe = sF + el * 9 * NS;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T n0 = c.nvec[d][0], n1 = c.nvec[d][1], n2 = c.nvec[d][2];
            T vn = u[0] * n0;
            vn = fma(u[1], n1, vn);
            vn = fma(u[2], n2, vn);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T sn = S[3 * i] * n0;
                sn = fma(S[3 * i + 1], n1, sn);
                sn = fma(S[3 * i + 2], n2, sn);
                Fe[(3 * d + i) * NS + q] = fma(u[i], vn, fma(Pq, c.nvec[d][i], -c.nu * sn));
            }
        }
    }
    // ---- stages 1 + 4 on chip: own trace, common flux with the neighbour trace
    {
        const int per_face = nel * NF;
        for (int t = threadIdx.x; t < 6 * per_face; t += blockDim.x) {
            const int f = t / per_face, r = t - f * per_face;
            const int el = r / NF, fp = r - el * NF;
            const int d = f >> 1, s = f & 1;
            const int a = fp % M, b = fp / M;
            T nh[3] = {c.nhat[d][0], c.nhat[d][1], c.nhat[d][2]};
            T own[NTR], oth[NTR], out[NTR];
            face_trace<M, T>(sU + el * NV * NS, d, a, b, sop + (s ? OL::lp : OL::lm), nh, own);
            T *slot = sFI + ((el * 6 + f) * NTR) * NF + fp;
#pragma unroll
            for (int cc = 0; cc < NTR; ++cc) oth[cc] = slot[cc * NF];
            if (s) common_flux<T>(own, oth, nh, c.nmag[d], c.zeta, c.nu, out);
            else common_flux<T>(oth, own, nh, c.nmag[d], c.zeta, c.nu, out);
#pragma unroll
            for (int cc = 0; cc < NTR; ++cc) slot[cc * NF] = out[cc];
        }
    }
    __syncthreads();

    // ---- stages 3, 5, 6: partially corrected divergence along the three line
    //      families, correction with the common fluxes, negate, source.
    const T *Dt = sop + OL::Dt;
    const T *gl = sop + OL::gl;
    const T *gr = sop + OL::gr;
    for (int t = threadIdx.x; t < nel * NS; t += blockDim.x) {
        const int el = t / NS, q = t - el * NS;
        const int i0 = q % M, i1 = (q / M) % M, i2 = q / (M * M);
        const int idx[3] = {i0, i1, i2};
        const int fa[3] = {i1, i0, i0}, fb[3] = {i2, i2, i1};
        const T *Ue = sU + el * NV * NS;
        const T *Fe = sF + el * 9 * NS;
        const T *FIe = sFI + el * 6 * NTR * NF;
        T cdu[3][3];   // corrected d u_a / d xi_d
        T mom[3] = {T(0), T(0), T(0)};
        T dissP = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int id = idx[d];
            const int fp = fa[d] + M * fb[d];
            const T *FIm = FIe + (2 * d) * NTR * NF + fp;
            const T *FIp = FIe + (2 * d + 1) * NTR * NF + fp;
            const T gld = gl[id], grd = gr[id];
            T du[3] = {T(0), T(0), T(0)}, df[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int l = 0; l < M; ++l) {
                const int ql = line_pt<M>(d, fa[d], fb[d], l);
                const T w = Dt[id * M + l];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    du[a] = fma(w, Ue[(1 + a) * NS + ql], du[a]);
                    df[a] = fma(w, Fe[(3 * d + a) * NS + ql], df[a]);
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cdu[a][d] = fma(gld, FIm[(4 + a) * NF], fma(grd, FIp[(4 + a) * NF], du[a]));
                mom[a] += fma(gld, FIm[(1 + a) * NF], fma(grd, FIp[(1 + a) * NF], df[a]));
            }
            dissP = fma(gld, FIm[0], fma(grd, FIp[0], dissP));
        }
        T *Re = R + (e0 + el) * NV * NS + q;
        // P: -(1/detJ) [ zeta sum_d n_d . (corrected dV/dxi_d) + dissipation ]
        T divV = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int a = 0; a < 3; ++a) divV = fma(c.nvec[d][a], cdu[a][d], divV);
        Re[0] = -c.inv_det * fma(c.zeta, divV, dissP);
#pragma unroll
        for (int a = 0; a < 3; ++a) Re[(1 + a) * NS] = -c.inv_det * mom[a];
        // aux (a, k): (1/T) [ (1/detJ) sum_d n_d,k cdu[a][d] - S_ak ]
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T g = cdu[a][0] * c.nvec[0][k];
                g = fma(cdu[a][1], c.nvec[1][k], g);
                g = fma(cdu[a][2], c.nvec[2][k], g);
                Re[(4 + 3 * a + k) * NS] = c.invT * fma(c.inv_det, g, -Ue[(4 + 3 * a + k) * NS + q]);
            }
    }
}

// ---------------------------------------------------------------------------
// Unfused pipeline: Table 1 stages as separate kernels through HBM.
// Buffers: Uf[6][ne][13][NF], Fs[3][ne][13][NS], Dv[ne][13][NS], FI[3][ne][13][NF]
// ---------------------------------------------------------------------------

// Full 13-variable physical flux dotted with a vector nv (transformed when
// nv = n_d): out[v] = sum_j F_j,v nv_j.
template <typename T>
__device__ __forceinline__ void flux_dot(const T U[NV], const T nv[3], T zeta, T nu, T invT,
                                         T out[NV])
{
    T vn = U[1] * nv[0];
    vn = fma(U[2], nv[1], vn);
    vn = fma(U[3], nv[2], vn);
    out[0] = zeta * vn;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T sn = U[4 + 3 * i] * nv[0];
        sn = fma(U[5 + 3 * i], nv[1], sn);
        sn = fma(U[6 + 3 * i], nv[2], sn);
        out[1 + i] = fma(U[1 + i], vn, fma(U[0], nv[i], -nu * sn));
#pragma unroll
        for (int k = 0; k < 3; ++k) out[4 + 3 * i + k] = -invT * U[1 + i] * nv[k];
    }
}

template <int P, typename T>
__global__ void __launch_bounds__(256) k_u_project(const T *__restrict__ U, T *__restrict__ Uf,
                                                   const T *__restrict__ ops, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    using OL = OpsLayout<M>;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * 6 * NF) return;
    const int fp = (int)(t % NF);
    const int64_t r = t / NF;
    const int64_t e = r % ne;
    const int f = (int)(r / ne);
    const int d = f >> 1, s = f & 1;
    const T *lf = ops + (s ? OL::lp : OL::lm);
    const int a = fp % M, b = fp / M;
    const T *Ue = U + e * NV * NS;
    T *dst = Uf + (((int64_t)f * ne + e) * NV) * NF + fp;
    for (int v = 0; v < NV; ++v) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < M; ++l) acc = fma(lf[l], Ue[v * NS + line_pt<M>(d, a, b, l)], acc);
        dst[v * NF] = acc;
    }
}

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

template <int P, typename T>
__global__ void __launch_bounds__(256) k_u_div(const T *__restrict__ Fs, T *__restrict__ Dv,
                                               const T *__restrict__ ops, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M;
    using OL = OpsLayout<M>;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * NS) return;
    const int64_t e = t / NS;
    const int q = (int)(t - e * NS);
    const int idx[3] = {q % M, (q / M) % M, q / (M * M)};
    const int fa[3] = {idx[1], idx[0], idx[0]}, fb[3] = {idx[2], idx[2], idx[1]};
    for (int v = 0; v < NV; ++v) {
        T acc = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T *Fd = Fs + (((int64_t)d * ne + e) * NV + v) * NS;
#pragma unroll
            for (int l = 0; l < M; ++l)
                acc = fma(ops[OL::Dt + idx[d] * M + l], Fd[line_pt<M>(d, fa[d], fb[d], l)], acc);
        }
        Dv[(e * NV + v) * NS + q] = acc;
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

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
inline int default_block(int p, int prec)
{
    // elements per workgroup of k_fused / k_trace (LDS budget and lane fill)
    static const int f64[7] = {0, 16, 8, 4, 2, 1, 1};
    static const int f32[7] = {0, 32, 8, 4, 2, 1, 1};
    return prec == FR_F64 ? f64[p] : f32[p];
}

inline int threads_for(int pts)
{
    int t = ((pts + 63) / 64) * 64;
    return t > 256 ? 256 : (t < 64 ? 64 : t);
}

template <int P, typename T>
int fused_impl(fr_plan *pl, const T *U, T *R, T *TR, const T *ops, const Consts<T> &c,
               hipStream_t s)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    const int prec = sizeof(T) == 8 ? FR_F64 : FR_F32;
    int E = pl->block ? pl->block : default_block(P, prec);
    const int64_t ne = pl->ne;
    if (E > ne) E = (int)ne;
    const unsigned grid = (unsigned)((ne + E - 1) / E);
    const size_t lds_tr = ((size_t)E * NV * NS + 2 * M) * sizeof(T);
    const size_t lds_fu =
        ((size_t)E * (NV + 9) * NS + (size_t)E * 6 * NTR * NF + OpsLayout<M>::size) * sizeof(T);
    if (lds_fu > 160 * 1024)
        return set_error(FR_EINVAL, "fused kernel: %d elements per block need %zu B of LDS", E,
                         lds_fu);
    static bool attr_done = false;
    if (!attr_done) {
        if (int rc = check_hip(hipFuncSetAttribute((const void *)k_trace<P, T>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   160 * 1024),
                               "hipFuncSetAttribute(k_trace)"))
            return rc;
        if (int rc = check_hip(hipFuncSetAttribute((const void *)k_fused<P, T>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   160 * 1024),
                               "hipFuncSetAttribute(k_fused)"))
            return rc;
        attr_done = true;
    }
    const int nt_tr = threads_for(E * 6 * NF);
    const int nt_fu = threads_for(E * NS);
    hipLaunchKernelGGL((k_trace<P, T>), dim3(grid), dim3(nt_tr), lds_tr, s, U, TR, ops, c, ne, E);
    hipLaunchKernelGGL((k_fused<P, T>), dim3(grid), dim3(nt_fu), lds_fu, s, U, TR, R, ops, c,
                       pl->nx, pl->ny, pl->nz, E);
    return check_hip(hipGetLastError(), "k_fused launch");
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
    hipLaunchKernelGGL((k_u_project<P, T>), g(ne * 6 * NF), dim3(nt), 0, s, U, Uf, ops, ne);
    hipLaunchKernelGGL((k_u_flux<P, T>), g(ne * NS), dim3(nt), 0, s, U, Fs, c, ne);
    hipLaunchKernelGGL((k_u_div<P, T>), g(ne * NS), dim3(nt), 0, s, Fs, Dv, ops, ne);
    hipLaunchKernelGGL((k_u_common<P, T>), g(ne * 3 * NF), dim3(nt), 0, s, Uf, FI, c, pl->nx,
                       pl->ny, pl->nz);
    hipLaunchKernelGGL((k_u_correct<P, T>), g(ne * NS), dim3(nt), 0, s, Dv, FI, ops, pl->nx,
                       pl->ny, pl->nz);
    hipLaunchKernelGGL((k_u_negsrc<P, T>), g(ne * NV * NS), dim3(nt), 0, s, Dv, U, R, c, ne);
    return check_hip(hipGetLastError(), "unfused launch");
}

template <typename T>
int dispatch_fused(fr_plan *pl, const T *U, T *R, T *TR, const T *ops, const Consts<T> &c,
                   hipStream_t s)
{
    switch (pl->p) {
        case 1: return fused_impl<1, T>(pl, U, R, TR, ops, c, s);
        case 2: return fused_impl<2, T>(pl, U, R, TR, ops, c, s);
        case 3: return fused_impl<3, T>(pl, U, R, TR, ops, c, s);
        case 4: return fused_impl<4, T>(pl, U, R, TR, ops, c, s);
        case 5: return fused_impl<5, T>(pl, U, R, TR, ops, c, s);
        case 6: return fused_impl<6, T>(pl, U, R, TR, ops, c, s);
    }
    return set_error(FR_EINVAL, "order %d", pl->p);
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

int launch_residual_fused(fr_plan *pl, const void *U, void *R, hipStream_t s)
{
    const int m = pl->m;
    const size_t esz = pl->precision == FR_F64 ? 8 : 4;
    const size_t tr_bytes = (size_t)6 * pl->ne * NTR * m * m * esz;
    if (int rc = ensure_scratch(pl->traces, tr_bytes)) return rc;
    if (pl->precision == FR_F64)
        return dispatch_fused<double>(pl, (const double *)U, (double *)R, (double *)pl->traces.ptr,
                                      (const double *)pl->ops64, pl->c64, s);
    return dispatch_fused<float>(pl, (const float *)U, (float *)R, (float *)pl->traces.ptr,
                                 (const float *)pl->ops32, pl->c32, s);
}

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
