// Device helpers shared by the residual kernels (fused and unfused paths).
//
// Face numbering: f = 2 d + s (d = direction, s = 0 minus / 1 plus side).
// A face point is (a, b): the two tangential point indices in increasing
// direction order, flattened a + m b.  Every element has the same
// orientation, so face point (a, b) of face (d, 1) meets point (a, b) of the
// neighbour's face (d, 0).
#pragma once

#include "fr_internal.h"

namespace fr {
namespace dev {

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

// First point and point stride of the direction-d line through face point (a, b).
template <int M>
__device__ __forceinline__ void line_of(int d, int a, int b, int &base, int &stride)
{
    stride = d == 0 ? 1 : (d == 1 ? M : M * M);
    base = d == 0 ? M * (a + M * b) : (d == 1 ? a + M * M * b : a + M * b);
}

// One face-trace value of one element along the line (base, stride), using the
// endpoint basis values lf[] (l(-1) or l(+1)):
//   c = 0..3   P, u, v, w projected to the face
//   c = 4..6   (S n_hat)_i projected to the face, S_ik = d u_i / d x_k
// Written as one explicit fma chain so that every kernel that computes the
// same trace value produces the same bits.
//
// With diag (the reference-face normals are the coordinate axes: a diagonal
// Jacobian) (S n_hat)_i = S_id exactly, and the product with the unit normal is
// skipped; the result has the same bits as the general expression, whose other
// terms are exact zeros and whose product with 1 is exact.
// VS is the distance between consecutive variables of Ue (m^3 unless the
// caller pads its lines).
template <int M, typename T, int VS = M * M * M>
__device__ __forceinline__ T trace_value(const T *__restrict__ Ue, int d, int base, int stride,
                                         const T *__restrict__ lf, const T nh[3], int c,
                                         bool diag = false)
{
    constexpr int NS = VS;
    T acc = T(0);
    if (c < 4) {
        const T *X = Ue + c * NS + base;
#pragma unroll
        for (int l = 0; l < M; ++l) acc = fma(lf[l], X[l * stride], acc);
    } else if (diag) {
        const T *X = Ue + (4 + 3 * (c - 4) + d) * NS + base;
#pragma unroll
        for (int l = 0; l < M; ++l) acc = fma(lf[l], X[l * stride], acc);
    } else {
        const T *X = Ue + (4 + 3 * (c - 4)) * NS + base;
#pragma unroll
        for (int l = 0; l < M; ++l) {
            const int q = l * stride;
            T sn = X[q] * nh[0];
            sn = fma(X[NS + q], nh[1], sn);
            sn = fma(X[2 * NS + q], nh[2], sn);
            acc = fma(lf[l], sn, acc);
        }
    }
    return acc;
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
    // lambda = max over both sides of |v| + sqrt(v^2 + zeta); the expression is
    // monotone in |v| (also after rounding), so it is evaluated once at the
    // larger |v|, with the same bits as the maximum of the two evaluations.
    const T vm = fmax(fabs(vnl), fabs(vnr));
    const T lam = vm + sqrt(fma(vm, vm, zeta));
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

// 16-byte vector of the working precision
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
template <typename T> struct V16;
template <> struct V16<double> { using type = d2v; };
template <> struct V16<float> { using type = f4v; };

// LDS layout of the line form: the batch's elements at a pitch of EP values
// (13 m^3 padded so that consecutive elements start at bank offsets m^2 apart:
// lanes of neighbouring elements then read neighbouring banks).
template <int P, typename T>
struct LinesLds {
    static constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    static constexpr int BANKV = sizeof(T) == 8 ? 32 : 64;  // values per bank sweep of a read
    static constexpr int raw = NV * NS;
    static constexpr int EP = raw + ((NF - raw % BANKV) % BANKV + BANKV) % BANKV;
    // whole 16-byte chunks per element, so that the copy can use vectors
    static constexpr bool VEC = (raw * sizeof(T)) % 16 == 0 && (EP * sizeof(T)) % 16 == 0;
    // the operator block, padded to 16 bytes
    static constexpr int OPS = (OpsLayout<M>::size * (int)sizeof(T) + 15) / 16 * 16 / (int)sizeof(T);
    // LDS values of a batch of E elements: operators, state tile, and the
    // directions' P and momentum parts that wait in LDS (three directions for
    // xr = 0, two for xr = 1, none for xr = 2, 3)
    static constexpr int values(int E, int xr)
    {
        return OPS + E * EP + (xr >= 2 ? 0 : (xr == 1 ? 8 : 12)) * E * NS;
    }
};

// Whether the line form's tile loads are marked nontemporal.  They are not:
// the halo form reads the neighbours' lines of the same state again, and
// plain loads leave the state in the caches for them (measured 2-9% faster
// at every order than nontemporal loads).
#ifndef FR_TILE_NT
#define FR_TILE_NT 0
#endif
template <typename V>
__device__ __forceinline__ V tile_ld(const V *p)
{
    if constexpr (FR_TILE_NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// A batch's contiguous state block (nel elements from src) into the line
// form's LDS tile (element pitch EP), in 16-byte vectors where the element
// size allows.
template <int P, typename T, int NT>
__device__ __forceinline__ void tile_load(const T *__restrict__ src, T *__restrict__ sU, int nel)
{
    using LL = LinesLds<P, T>;
    constexpr int EP = LL::EP, RAW = LL::raw;
    if constexpr (LL::VEC) {
        using V = typename V16<T>::type;
        constexpr int VW = 16 / sizeof(T), CPE = RAW / VW;  // chunks per element
        const int nch = nel * CPE;
        const V *sv = reinterpret_cast<const V *>(src);
#pragma unroll 4
        for (int k = threadIdx.x; k < nch; k += NT) {
            const int ek = k / CPE, o = k - ek * CPE;
            reinterpret_cast<V *>(sU + ek * EP)[o] = tile_ld(sv + k);
        }
    } else {
        const int nv = nel * RAW;
#pragma unroll 4
        for (int k = threadIdx.x; k < nv; k += NT) {
            const int ek = k / RAW, o = k - ek * RAW;
            sU[ek * EP + o] = tile_ld(src + k);
        }
    }
}

// The reverse of tile_load: nel finished elements of the tile (pitch EP) to
// their contiguous block at dst.
template <int P, typename T, int NT>
__device__ __forceinline__ void tile_store(const T *__restrict__ sU, T *__restrict__ dst, int nel)
{
    using LL = LinesLds<P, T>;
    constexpr int EP = LL::EP, RAW = LL::raw;
    if constexpr (LL::VEC) {
        using V = typename V16<T>::type;
        constexpr int VW = 16 / sizeof(T), CPE = RAW / VW;
        const int nch = nel * CPE;
        V *dv = reinterpret_cast<V *>(dst);
#pragma unroll 4
        for (int k = threadIdx.x; k < nch; k += NT) {
            const int ek = k / CPE, o = k - ek * CPE;
            __builtin_nontemporal_store(reinterpret_cast<const V *>(sU + ek * EP)[o], dv + k);
        }
    } else {
        const int nv = nel * RAW;
#pragma unroll 4
        for (int k = threadIdx.x; k < nv; k += NT) {
            const int ek = k / RAW, o = k - ek * RAW;
            __builtin_nontemporal_store(sU[ek * EP + o], dst + k);
        }
    }
}

}  // namespace dev
}  // namespace fr
