// Fused residual kernels for gfx950: R = -div F + S of ACM-HD by flux
// reconstruction on constant-Jacobian hexahedra (paper Sec. 2.1, 2.2;
// Table 1 stages 1-6, with the fusion of Sec. 3: stages 2, 3 and 6 in one
// kernel, and here stages 4 and 5 as well).
//
//   k_trace  stage 1 restricted to what the neighbours need: per element and
//            face, 7 trace values per face point (P, V, (S n_hat)) written to
//            TR[6][ne][7][m^2].  Reads U once.
//   k_fused  stages 2-6 for a batch of E elements staged in LDS: transformed
//            momentum flux at the points, partially corrected divergence along
//            the three line families, own face traces recomputed on chip,
//            Rusanov / mean common flux against the neighbour traces,
//            correction, source.  Reads U and the neighbour traces once,
//            writes R once.
//
// Both kernels loop over element batches (batch b = blockIdx.x + k gridDim.x)
// and prefetch the next batch's global data into registers before computing
// the current one, so every workgroup keeps a batch of loads in flight while
// it works on LDS; the grid is sized to the number of co-resident workgroups.
#include <mutex>

#include "fr_device.h"

namespace fr {
namespace {
using namespace dev;


// Launch shape per order and precision: EMAX elements per batch (a runtime
// block size E <= EMAX may be chosen) and NT threads per workgroup.  Each
// value can be overridden at build time (FR_E<p>_<D|F>, FR_NT<p>_<D|F>).
#ifndef FR_E1_D
#define FR_E1_D 8
#endif
#ifndef FR_NT1_D
#define FR_NT1_D 64
#endif
#ifndef FR_E2_D
#define FR_E2_D 9
#endif
#ifndef FR_NT2_D
#define FR_NT2_D 256
#endif
#ifndef FR_E3_D
#define FR_E3_D 2
#endif
#ifndef FR_NT3_D
#define FR_NT3_D 128
#endif
#ifndef FR_E4_D
#define FR_E4_D 1
#endif
#ifndef FR_NT4_D
#define FR_NT4_D 192
#endif
#ifndef FR_E5_D
#define FR_E5_D 1
#endif
#ifndef FR_NT5_D
#define FR_NT5_D 256
#endif
#ifndef FR_E6_D
#define FR_E6_D 1
#endif
#ifndef FR_NT6_D
#define FR_NT6_D 256
#endif
#ifndef FR_E1_F
#define FR_E1_F 8
#endif
#ifndef FR_NT1_F
#define FR_NT1_F 64
#endif
#ifndef FR_E2_F
#define FR_E2_F 4
#endif
#ifndef FR_NT2_F
#define FR_NT2_F 128
#endif
#ifndef FR_E3_F
#define FR_E3_F 1
#endif
#ifndef FR_NT3_F
#define FR_NT3_F 64
#endif
#ifndef FR_E4_F
#define FR_E4_F 1
#endif
#ifndef FR_NT4_F
#define FR_NT4_F 128
#endif
#ifndef FR_E5_F
#define FR_E5_F 1
#endif
#ifndef FR_NT5_F
#define FR_NT5_F 256
#endif
#ifndef FR_E6_F
#define FR_E6_F 1
#endif
#ifndef FR_NT6_F
#define FR_NT6_F 256
#endif
template <int P, typename T> struct Shape;
template <> struct Shape<1, double> { static constexpr int EMAX = FR_E1_D, NT = FR_NT1_D; };
template <> struct Shape<2, double> { static constexpr int EMAX = FR_E2_D, NT = FR_NT2_D; };
template <> struct Shape<3, double> { static constexpr int EMAX = FR_E3_D, NT = FR_NT3_D; };
template <> struct Shape<4, double> { static constexpr int EMAX = FR_E4_D, NT = FR_NT4_D; };
template <> struct Shape<5, double> { static constexpr int EMAX = FR_E5_D, NT = FR_NT5_D; };
template <> struct Shape<6, double> { static constexpr int EMAX = FR_E6_D, NT = FR_NT6_D; };
template <> struct Shape<1, float> { static constexpr int EMAX = FR_E1_F, NT = FR_NT1_F; };
template <> struct Shape<2, float> { static constexpr int EMAX = FR_E2_F, NT = FR_NT2_F; };
template <> struct Shape<3, float> { static constexpr int EMAX = FR_E3_F, NT = FR_NT3_F; };
template <> struct Shape<4, float> { static constexpr int EMAX = FR_E4_F, NT = FR_NT4_F; };
template <> struct Shape<5, float> { static constexpr int EMAX = FR_E5_F, NT = FR_NT5_F; };
template <> struct Shape<6, float> { static constexpr int EMAX = FR_E6_F, NT = FR_NT6_F; };

// Shape of the trace kernel (it carries no face data and prefers larger batches).
#ifndef FR_TE1_D
#define FR_TE1_D 64
#endif
#ifndef FR_TNT1_D
#define FR_TNT1_D 256
#endif
#ifndef FR_TE2_D
#define FR_TE2_D 16
#endif
#ifndef FR_TNT2_D
#define FR_TNT2_D 256
#endif
#ifndef FR_TE3_D
#define FR_TE3_D 8
#endif
#ifndef FR_TNT3_D
#define FR_TNT3_D 256
#endif
#ifndef FR_TE4_D
#define FR_TE4_D 4
#endif
#ifndef FR_TNT4_D
#define FR_TNT4_D 256
#endif
#ifndef FR_TE5_D
#define FR_TE5_D 2
#endif
#ifndef FR_TNT5_D
#define FR_TNT5_D 256
#endif
#ifndef FR_TE6_D
#define FR_TE6_D 1
#endif
#ifndef FR_TNT6_D
#define FR_TNT6_D 512
#endif
#ifndef FR_TE1_F
#define FR_TE1_F 64
#endif
#ifndef FR_TNT1_F
#define FR_TNT1_F 256
#endif
#ifndef FR_TE2_F
#define FR_TE2_F 8
#endif
#ifndef FR_TNT2_F
#define FR_TNT2_F 256
#endif
#ifndef FR_TE3_F
#define FR_TE3_F 4
#endif
#ifndef FR_TNT3_F
#define FR_TNT3_F 256
#endif
#ifndef FR_TE4_F
#define FR_TE4_F 4
#endif
#ifndef FR_TNT4_F
#define FR_TNT4_F 256
#endif
#ifndef FR_TE5_F
#define FR_TE5_F 1
#endif
#ifndef FR_TNT5_F
#define FR_TNT5_F 256
#endif
#ifndef FR_TE6_F
#define FR_TE6_F 1
#endif
#ifndef FR_TNT6_F
#define FR_TNT6_F 256
#endif
template <int P, typename T> struct TraceShape;
template <> struct TraceShape<1, double> { static constexpr int EMAX = FR_TE1_D, NT = FR_TNT1_D; };
template <> struct TraceShape<2, double> { static constexpr int EMAX = FR_TE2_D, NT = FR_TNT2_D; };
template <> struct TraceShape<3, double> { static constexpr int EMAX = FR_TE3_D, NT = FR_TNT3_D; };
template <> struct TraceShape<4, double> { static constexpr int EMAX = FR_TE4_D, NT = FR_TNT4_D; };
template <> struct TraceShape<5, double> { static constexpr int EMAX = FR_TE5_D, NT = FR_TNT5_D; };
template <> struct TraceShape<6, double> { static constexpr int EMAX = FR_TE6_D, NT = FR_TNT6_D; };
template <> struct TraceShape<1, float> { static constexpr int EMAX = FR_TE1_F, NT = FR_TNT1_F; };
template <> struct TraceShape<2, float> { static constexpr int EMAX = FR_TE2_F, NT = FR_TNT2_F; };
template <> struct TraceShape<3, float> { static constexpr int EMAX = FR_TE3_F, NT = FR_TNT3_F; };
template <> struct TraceShape<4, float> { static constexpr int EMAX = FR_TE4_F, NT = FR_TNT4_F; };
template <> struct TraceShape<5, float> { static constexpr int EMAX = FR_TE5_F, NT = FR_TNT5_F; };
template <> struct TraceShape<6, float> { static constexpr int EMAX = FR_TE6_F, NT = FR_TNT6_F; };

// Face-trace blocks in HBM, indexed by the element that consumes them:
// TR[f][e] holds the 7 x m^2 trace values that element e needs on its face f,
// i.e. the values of the neighbour across that face, on the neighbour's face
// f ^ 1.  Each block is padded to a whole number of 16-byte chunks so that a
// batch of consecutive elements reads, for every face, one contiguous and
// aligned run of blocks.
template <int M, typename T>
struct TraceLayout {
    static constexpr int NF = M * M, CH = NTR * NF;
    static constexpr int W = 16 / sizeof(T);
    static constexpr int CHP = (CH + W - 1) / W * W;
    static constexpr int CHV = CHP / W;
};

// LDS point pitch of the trace kernel: at p = 3, 5 its x-face reads walk the
// points with a stride of one x-line per lane; padding every x-line by one
// value makes that stride odd, so the reads of a wave spread over the banks.
template <int M>
struct TracePad {
    static constexpr int MP = (M % 2 == 0 && M >= 4) ? M + 1 : M;
    static constexpr int NSP = MP * M * M;
    __device__ __forceinline__ static unsigned idx(unsigned q) { return q + (MP - M) * (q / M); }
};

// Register staging of one batch's contiguous state block U[e0 .. e0+nel).
// Chunk k of W values (W = 16 bytes) belongs to thread k mod NT.  A full batch
// (count == NVAL) whose start is 16-byte aligned takes a branch-free path with
// one 16-byte access per chunk; other batches check every value.
template <typename T, int NVAL, int NT>
struct StateStage {
    static constexpr int W = 16 / sizeof(T);
    static constexpr int NCH = (NVAL + W - 1) / W;   // chunks in a full batch
    static constexpr int PV = (NCH + NT - 1) / NT;   // chunks per thread
    static constexpr bool EXACT = NVAL % W == 0;
    T r[PV * W];

    __device__ __forceinline__ void load(const T *__restrict__ src, int count, int tid)
    {
        using V = typename V16<T>::type;
        if (EXACT && count == NVAL && (((uintptr_t)src) & 15) == 0) {
#pragma unroll
            for (int i = 0; i < PV; ++i) {
                const int k = tid + i * NT;
                if ((i + 1) * NT <= NCH || k < NCH) {
                    V x = __builtin_nontemporal_load(reinterpret_cast<const V *>(src) + k);
#pragma unroll
                    for (int w = 0; w < W; ++w) r[i * W + w] = x[w];
                }
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < PV; ++i) {
            const int v0 = (tid + i * NT) * W;
#pragma unroll
            for (int w = 0; w < W; ++w)
                if (v0 + w < count) r[i * W + w] = src[v0 + w];
        }
    }
    // store into LDS with the x-lines of every variable padded to TracePad<M>::MP
    template <int M>
    __device__ __forceinline__ void store_padded(T *__restrict__ dst, int count, int tid) const
    {
        constexpr int NS = M * M * M, NSP = TracePad<M>::NSP;
        static_assert(TracePad<M>::MP == M || NS % W == 0, "a chunk must not straddle variables");
        if (TracePad<M>::MP == M) {
            store(dst, count, tid);
            return;
        }
#pragma unroll
        for (int i = 0; i < PV; ++i) {
            const unsigned v0 = (tid + i * NT) * W;
            const unsigned ev = v0 / NS, q = v0 - ev * NS;  // ev = element * NV + variable
#pragma unroll
            for (int w = 0; w < W; ++w)
                if ((int)(v0 + w) < count) dst[ev * NSP + TracePad<M>::idx(q + w)] = r[i * W + w];
        }
    }
    __device__ __forceinline__ void store(T *__restrict__ dst, int count, int tid) const
    {
        using V = typename V16<T>::type;
        if (EXACT && count == NVAL) {
#pragma unroll
            for (int i = 0; i < PV; ++i) {
                const int k = tid + i * NT;
                if ((i + 1) * NT <= NCH || k < NCH) {
                    V x;
#pragma unroll
                    for (int w = 0; w < W; ++w) x[w] = r[i * W + w];
                    reinterpret_cast<V *>(dst)[k] = x;
                }
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < PV; ++i) {
            const int v0 = (tid + i * NT) * W;
#pragma unroll
            for (int w = 0; w < W; ++w)
                if (v0 + w < count) dst[v0 + w] = r[i * W + w];
        }
    }
};

// Register staging of a batch's trace blocks: six runs (one per face) of nel
// consecutive padded blocks, TR[f][e0 .. e0+nel), into LDS as [f][EMAX][CHP].
// All accesses are aligned 16-byte chunks.
template <int M, typename T, int EMAX, int NT>
struct TraceStage {
    using TL = TraceLayout<M, T>;
    using V = typename V16<T>::type;
    static constexpr int RUN = EMAX * TL::CHV;        // chunks per face run of a full batch
    static constexpr int NCH = 6 * RUN;
    static constexpr int PV = (NCH + NT - 1) / NT;
    V r[PV];

    __device__ __forceinline__ void load(const T *__restrict__ TR, int ne, int e0, int nel, int tid)
    {
        const V *src = reinterpret_cast<const V *>(TR);
        const unsigned run = (unsigned)nel * TL::CHV;
#pragma unroll
        for (int i = 0; i < PV; ++i) {
            const unsigned k = tid + i * NT;
            const unsigned f = k / RUN, o = k - f * RUN;
            if (((i + 1) * NT <= NCH || k < NCH) && (nel == EMAX || o < run))
                r[i] = __builtin_nontemporal_load(
                    src + ((int64_t)f * ne + e0) * TL::CHV + o);
        }
    }
    __device__ __forceinline__ void store(T *__restrict__ dst, int nel, int tid) const
    {
        V *d = reinterpret_cast<V *>(dst);
        const unsigned run = (unsigned)nel * TL::CHV;
#pragma unroll
        for (int i = 0; i < PV; ++i) {
            const unsigned k = tid + i * NT;
            const unsigned f = k / RUN, o = k - f * RUN;
            if (((i + 1) * NT <= NCH || k < NCH) && (nel == EMAX || o < run)) d[k] = r[i];
        }
    }
};

// The thread index, hidden from the optimiser so that index arithmetic derived
// from it is recomputed inside the batch loop instead of being hoisted out of
// it and kept live in registers for the whole kernel.
__device__ __forceinline__ int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Zero, hidden from the optimiser (a uniform value): an offset that keeps
// loads of loop-invariant data inside a loop.
__device__ __forceinline__ int opaque_zero()
{
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

// Neighbour element of every (element, face) of a batch, into an LDS table of
// 6 nel entries filled by the NT threads of the workgroup.
template <int NT>
__device__ __forceinline__ void neighbour_table(int *sNb, int e0, int nel, int nx, int ny, int nz)
{
    for (int t = threadIdx.x; t < 6 * nel; t += NT) {
        const int el = t / 6, f = t - el * 6;
        const int e = e0 + el;
        int ex = e % nx;
        const int r = e / nx;
        int ey = r % ny;
        int ez = r / ny;
        const int d = f >> 1, up = f & 1;
        if (d == 0) ex = up ? (ex + 1 == nx ? 0 : ex + 1) : (ex == 0 ? nx - 1 : ex - 1);
        else if (d == 1) ey = up ? (ey + 1 == ny ? 0 : ey + 1) : (ey == 0 ? ny - 1 : ey - 1);
        else ez = up ? (ez + 1 == nz ? 0 : ez + 1) : (ez == 0 ? nz - 1 : ez - 1);
        sNb[t] = ex + nx * (ey + ny * ez);
    }
}

// Common normal flux through a face of direction d, evaluated by the element
// on one side: own = its trace, oth = the neighbour's, own_minus = the element
// is on the minus side of the face (its + face).  Equal, bit for bit, to the
// same flux evaluated by the neighbour, because every asymmetric term is
// written as a signed difference oth - own whose sign is carried by an exact
// sign flip of lambda, and every symmetric term is a commutative sum.
//   out[0]     Rusanov dissipation on P, -|n| lambda (P_plus - P_minus) / 2
//   out[1..3]  momentum common flux (times |n_d|)
//   out[4..6]  mean velocity
template <typename T>
__device__ __forceinline__ void common_flux_sided(const T own[NTR], const T oth[NTR], bool own_minus,
                                                  const T nh[3], T nmag, T zeta, T nu, T out[NTR])
{
    T vo = own[1] * nh[0];
    vo = fma(own[2], nh[1], vo);
    vo = fma(own[3], nh[2], vo);
    T vt = oth[1] * nh[0];
    vt = fma(oth[2], nh[1], vt);
    vt = fma(oth[3], nh[2], vt);
    // lambda = max over both sides of |v| + sqrt(v^2 + zeta), evaluated once
    // at the larger |v| (the expression is monotone in |v| after rounding too)
    const T vm = fmax(fabs(vo), fabs(vt));
    const T lam = vm + sqrt(fma(vm, vm, zeta));
    const T hm = T(0.5) * nmag;
    // P_plus - P_minus = (own_minus ? 1 : -1) (P_oth - P_own)
    const T slam = own_minus ? lam : -lam;
    out[0] = (-hm * slam) * (oth[0] - own[0]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T fo = fma(own[1 + i], vo, fma(own[0], nh[i], -nu * own[4 + i]));
        const T ft = fma(oth[1 + i], vt, fma(oth[0], nh[i], -nu * oth[4 + i]));
        out[1 + i] = hm * fma(oth[1 + i] - own[1 + i], -slam, fo + ft);
        out[4 + i] = T(0.5) * (own[1 + i] + oth[1 + i]);
    }
}

// ---------------------------------------------------------------------------
// k_trace: per batch of consecutive elements staged in LDS, every face value
// an element's neighbours need, written to the neighbour's receiving block.
// ---------------------------------------------------------------------------
template <int P, typename T, bool DIAG>
__global__ void __launch_bounds__((TraceShape<P, T>::NT))
    k_trace(const T *__restrict__ U, T *__restrict__ TR, const T *__restrict__ ops, Consts<T> c,
            int nx, int ny, int nz, int E, int nbatch)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    using TL = TraceLayout<M, T>;
    constexpr int CH = TL::CH, CHV = TL::CHV, W = TL::W;
    constexpr int EMAX = TraceShape<P, T>::EMAX, NT = TraceShape<P, T>::NT;
    constexpr int MP = TracePad<M>::MP, NSP = TracePad<M>::NSP;
    using OL = OpsLayout<M>;
    using V = typename V16<T>::type;
    const int ne = nx * ny * nz;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sU = reinterpret_cast<T *>(smem_raw);
    T *sl = sU + EMAX * NV * NSP;  // lm[M], lp[M]
    int *sNb = reinterpret_cast<int *>(sl + 2 * M);
    if (threadIdx.x < 2 * M) sl[threadIdx.x] = ops[OL::lm + threadIdx.x];

    StateStage<T, EMAX * NV * NS, NT> st;
    int b = blockIdx.x;
    if (b < nbatch) {
        const int e0 = b * E;
        st.load(U + (int64_t)e0 * NV * NS, min(E, ne - e0) * NV * NS, threadIdx.x);
    }
    V *TRv = reinterpret_cast<V *>(TR);
    for (; b < nbatch; b += gridDim.x) {
        const int tid = opaque_tid();
        const int e0 = b * E;
        const int nel = min(E, ne - e0);
        __syncthreads();
        st.template store_padded<M>(sU, nel * NV * NS, tid);
        neighbour_table<NT>(sNb, e0, nel, nx, ny, nz);
        const int bn = b + gridDim.x;
        __syncthreads();
        if (bn < nbatch) {
            const int en = bn * E;
            st.load(U + (int64_t)en * NV * NS, min(E, ne - en) * NV * NS, tid);
        }
        // one 16-byte chunk of one (face, element) block per thread and step;
        // the block of own face f goes to the receiving block (f ^ 1, neighbour)
        for (unsigned t = tid; t < 6u * EMAX * CHV; t += NT) {
            const unsigned f = t / (EMAX * CHV), r = t - f * (EMAX * CHV);
            const unsigned el = r / CHV, k = r - el * CHV;
            if ((int)el >= nel) continue;
            const int d = f >> 1, s = f & 1;
            const T nh[3] = {c.nhat[d][0], c.nhat[d][1], c.nhat[d][2]};
            V x;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const unsigned o = k * W + w;
                const unsigned cc = o / NF, fp = o - cc * NF;
                const unsigned a = fp % M, bb = fp / M;
                const int stride = d == 0 ? 1 : (d == 1 ? MP : MP * M);
                const int base = d == 0 ? MP * fp : (d == 1 ? a + MP * M * bb : a + MP * bb);
                x[w] = o < (unsigned)CH
                           ? trace_value<M, T, NSP>(sU + el * NV * NSP, d, base, stride, sl + s * M, nh,
                                                    cc, DIAG)
                           : T(0);
            }
            const int nb = sNb[el * 6 + f];
            __builtin_nontemporal_store(x, TRv + ((int64_t)(f ^ 1) * ne + nb) * CHV + k);
        }
    }
}

// ---------------------------------------------------------------------------
// k_fused
// LDS: sU[EMAX][13][NS] | sF[EMAX][9][NS] | sFI[6][EMAX][CHP] | ops | geometry
// ---------------------------------------------------------------------------
template <int D> struct Dir { static constexpr int value = D; };

// Divergence as line tasks (diagonal Jacobian, p = 6, where it measured faster
// than the point-wise form; slower from p = 4 down): one thread per
// (element, field, line) reads the line once, applies the whole operator
// (uniform entries, scalar registers) and writes the line's corrected
// derivatives, instead of every point reading its whole line.
#ifndef FR_LDIV_PMIN
#define FR_LDIV_PMIN 6
#endif
template <int P, bool DIAG> struct LineDiv {
    static constexpr bool value = DIAG && P >= FR_LDIV_PMIN;
};

// Values per thread whose global operands the stage epilogue requests at once,
// per order and precision (a larger chunk overlaps more loads but can cost a
// wave of occupancy; measured).  FR_STG_CHUNK overrides the table.
template <int P, typename T>
constexpr int stage_chunk()
{
#ifdef FR_STG_CHUNK
    return FR_STG_CHUNK;
#else
    constexpr int d[PMAX + 1] = {0, 1, 1, 8, 1, 8, 4};
    constexpr int f[PMAX + 1] = {0, 8, 4, 1, 1, 8, 1};
    return sizeof(T) == 8 ? d[P] : f[P];
#endif
}

// Global loads and stores of the stage update: streams read or written once
// per stage, marked nontemporal (NTS) where that measured faster: always in
// the halo form's epilogue (2-7%), in the point form's except at p = 4 (where
// it measured 5-16% slower).
template <bool NTS, typename X>
__device__ __forceinline__ X stg_ld(const X *p)
{
    if constexpr (NTS) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NTS, typename X>
__device__ __forceinline__ void stg_st(X *p, X v)
{
    if constexpr (NTS) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// The RK stage update of one batch whose residual (working precision) is in
// LDS: tile(t) is the t-th of the batch's cnt values in global order
// ([element][variable][point], from element e0).  The double arithmetic of the
// stand-alone stage kernel (the residual went through LDS, so nothing is
// contracted into its last operation).  A thread (tid of nt) has at most J
// values, taken in chunks of C: the global operands of a chunk are requested
// before the first is used, so that the loads of a wave overlap, with a
// bounded register cost.  With tr_out the produced state replaces the
// residual in the tile; ss accumulates the squared velocity pseudo-residual.
template <int J, int C, int NS, typename T, bool NTS, typename Tile>
__device__ __forceinline__ void stage_update_batch(const StageSpec &sp, Tile &&tile, unsigned tid,
                                                   unsigned nt, unsigned cnt, int64_t e0, double &ss)
{
    const int64_t g0 = e0 * NV * NS;
#pragma unroll 1
    for (int j0 = 0; j0 < J; j0 += C) {
        double ou[C], oa[C], os[C], ob[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const unsigned t = tid + (j0 + j) * nt;
            if (t < cnt) {
                const int64_t gi = g0 + t;
                if (!sp.last) ou[j] = stg_ld<NTS>(sp.U + gi);
                if (!sp.first || sp.last) oa[j] = stg_ld<NTS>(sp.acc + gi);
                if (sp.B) {
                    const unsigned r = t / NS, q = t - r * NS;
                    const unsigned el = r / NV, v = r - el * NV;
                    if (v >= 1 && v <= 3) {
                        os[j] = sp.s_in ? stg_ld<NTS>(sp.s_in + gi) : stg_ld<NTS>(sp.U + gi);
                        ob[j] = stg_ld<NTS>(sp.B + ((int64_t)(e0 + el) * 3 + (v - 1)) * NS + q);
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const unsigned t = tid + (j0 + j) * nt;
            if (t < cnt) {
                const int64_t gi = g0 + t;
                const unsigned v = (t / NS) % NV;
                double kv = (double)tile(t);
                if (v >= 1 && v <= 3) {
                    if (sp.B) kv -= fma(sp.a, os[j], ob[j]);
                    if (sp.partial) ss = fma(kv, kv, ss);
                }
                if (sp.last) {
                    const double un = fma(sp.b, kv, oa[j]);
                    stg_st<NTS>(sp.U + gi, un);
                    if (sp.s_out) stg_st<NTS>(static_cast<T *>(sp.s_out) + gi, (T)un);
                    if (sp.tr_out) tile(t) = (T)un;
                } else {
                    stg_st<NTS>(sp.acc + gi, fma(sp.b, kv, sp.first ? ou[j] : oa[j]));
                    const double sn = fma(sp.cnext, kv, ou[j]);
                    if (sp.s_out64) stg_st<NTS>(sp.s_out64 + gi, sn);
                    stg_st<NTS>(static_cast<T *>(sp.s_out) + gi, (T)sn);
                    if (sp.tr_out) tile(t) = (T)sn;
                }
            }
        }
    }
}

// The stage epilogue needs the residual of a whole batch in the state tile:
// the line-task path leaves it there; the point-wise path holds it in
// registers, which is only done where a thread has a single point.
template <int P, typename T, bool DIAG> struct StageEpilogue {
    static constexpr int NS = (P + 1) * (P + 1) * (P + 1);
    static constexpr bool value =
        LineDiv<P, DIAG>::value || Shape<P, T>::EMAX * NS <= Shape<P, T>::NT;
};

// Face traces of one element line, written to the neighbours' receiving
// blocks (defined with the line form below).
template <int P, typename T, int D>
__device__ __forceinline__ void line_traces_out(const T *__restrict__ Ut, const T *__restrict__ lm,
                                                const T *__restrict__ lp, T *__restrict__ TR,
                                                int64_t e, int L, int nx, int ny, int nz, int64_t ne);

template <int P, typename T, bool DIAG, bool STG, bool MF = false>
__global__ void __launch_bounds__((Shape<P, T>::NT))
    k_fused(const T *__restrict__ U, const T *__restrict__ TR, T *__restrict__ R,
            const T *__restrict__ ops, Consts<T> c, int ne, int E, int nbatch, StageSpec sp)
{
    static_assert(!MF || (sizeof(T) == 4 && !STG), "matrix-core form: single precision residual");
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    using TL = TraceLayout<M, T>;
    constexpr int CHP = TL::CHP;
    constexpr int EMAX = Shape<P, T>::EMAX, NT = Shape<P, T>::NT;
    using OL = OpsLayout<M>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sU = reinterpret_cast<T *>(smem_raw);
    T *sF = sU + EMAX * NV * NS;
    T *sFI = sF + EMAX * 9 * NS;
    T *sop = sFI + 6 * EMAX * CHP;
    T *geo = sop + OL::size;  // n_d (row d), n_hat_d (row d), |n_d|
    for (int t = threadIdx.x; t < OL::size; t += NT) sop[t] = ops[t];
    if (threadIdx.x < 9) {
        geo[threadIdx.x] = c.nvec[threadIdx.x / 3][threadIdx.x % 3];
        geo[9 + threadIdx.x] = c.nhat[threadIdx.x / 3][threadIdx.x % 3];
    }
    if (threadIdx.x < 3) geo[18 + threadIdx.x] = c.nmag[threadIdx.x];

    StateStage<T, EMAX * NV * NS, NT> st;
    TraceStage<M, T, EMAX, NT> tt;
    int b = blockIdx.x;
    if (b < nbatch) {
        const int e0 = b * E, nel = min(E, ne - e0);
        st.load(U + (int64_t)e0 * NV * NS, nel * NV * NS, threadIdx.x);
        tt.load(TR, ne, e0, nel, threadIdx.x);
    }
    const T *Dt = sop + OL::Dt;
    const T *gl = sop + OL::gl;
    const T *gr = sop + OL::gr;
    // MF: this lane's A operands of [Dt | gl | gr] (rows i = lane % 16, K rows
    // 4 s + lane / 16; zero outside the m x (m + 2) block)
    constexpr int KS = (M + 2 + 3) / 4;
    T amf[MF ? KS : 1];
    if constexpr (MF) {
        const int i = threadIdx.x & 15, kq = (threadIdx.x & 63) >> 4;
#pragma unroll
        for (int st2 = 0; st2 < KS; ++st2) {
            const int kap = 4 * st2 + kq;
            amf[st2] = i >= M ? T(0)
                              : (kap < M ? ops[OL::Dt + i * M + kap]
                                         : (kap == M ? ops[OL::gl + i]
                                                     : (kap == M + 1 ? ops[OL::gr + i] : T(0))));
        }
    }
    // STG: sum of (k*_V)^2 over this workgroup's stage updates
    double ss = 0.0;
    for (; b < nbatch; b += gridDim.x) {
        const int tid = opaque_tid();
        const int e0 = b * E;
        const int nel = min(E, ne - e0);
        __syncthreads();
        st.store(sU, nel * NV * NS, tid);
        tt.store(sFI, nel, tid);
        const int bn = b + gridDim.x;
        __syncthreads();
        if (bn < nbatch) {
            const int en = bn * E, neln = min(E, ne - en);
            st.load(U + (int64_t)en * NV * NS, neln * NV * NS, tid);
            tt.load(TR, ne, en, neln, tid);
        }

        // ---- stage 2: transformed momentum flux at every point,
        //      Fhat_{d,i} = u_i (n_d . V) + P n_d,i - nu sum_j n_d,j S_ij
        for (unsigned t = tid; t < (unsigned)nel * NS; t += NT) {
            const unsigned el = t / NS, q = t - el * NS;
            const T *Ue = sU + el * NV * NS;
            const T u[3] = {Ue[1 * NS + q], Ue[2 * NS + q], Ue[3 * NS + q]};
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
        // ---- stages 1 + 4 on chip: own trace, common flux with the neighbour
        //      trace, result in place of the neighbour trace.  Face points are
        //      ordered (d, el, side, fp) so that the lanes of a wave mostly
        //      share a direction.
        for (unsigned t = tid; t < 3u * EMAX * 2 * NF; t += NT) {
            const unsigned d = t / (EMAX * 2 * NF), r = t - d * (EMAX * 2 * NF);
            const unsigned el = r / (2 * NF), r2 = r - el * (2 * NF);
            if ((int)el >= nel) continue;
            const unsigned s = r2 / NF, fp = r2 - s * NF;
            const unsigned a = fp % M, bb = fp / M;
            const int stride = d == 0 ? 1 : (d == 1 ? M : M * M);
            const int base = d == 0 ? M * fp : (d == 1 ? a + M * M * bb : fp);
            const T nh[3] = {geo[9 + 3 * d], geo[10 + 3 * d], geo[11 + 3 * d]};
            const T *lf = sop + (s ? OL::lp : OL::lm);
            T own[NTR], oth[NTR], out[NTR];
#pragma unroll
            for (int cc = 0; cc < NTR; ++cc) {
                if (cc >= 4) __builtin_amdgcn_sched_barrier(0);
                own[cc] = trace_value<M, T>(sU + el * NV * NS, d, base, stride, lf, nh, cc, DIAG);
            }
            T *slot = sFI + ((2 * d + s) * EMAX + el) * CHP + fp;
#pragma unroll
            for (int cc = 0; cc < NTR; ++cc) oth[cc] = slot[cc * NF];
            common_flux_sided<T>(own, oth, s != 0, nh, geo[18 + d], c.zeta, c.nu, out);
#pragma unroll
            for (int cc = 0; cc < NTR; ++cc) slot[cc * NF] = out[cc];
        }
        __syncthreads();

        // ---- stages 3, 5, 6 as line tasks (diagonal Jacobian).  Per direction:
        //      task (element, field, line) with field u_a or Fhat_{d,a}; the
        //      corrected derivative along the line, in the same fma order as the
        //      point-wise form.  Velocity derivatives give the auxiliary residual
        //      at once (stored over S, which is no longer needed) and the
        //      divergence (accumulated over P); flux derivatives are stored over
        //      the consumed flux values.  A final pass writes R.
        if constexpr (MF) {
            // ---- stages 3, 5, 6 on the matrix cores (FP32 operands, FP32
            //      accumulation).  Per direction the corrected derivative of a
            //      line is [Dt | gl | gr] (m x (m + 2)) times the line's m values
            //      followed by its two common-flux values; 16 lines (element,
            //      face point) are the 16 columns of one v_mfma_f32_16x16x4f32
            //      chain over K = m + 2 (padded to a multiple of 4), one chain per
            //      field (the three velocities and the direction's three
            //      transformed momentum fluxes).  Lane l owns column l % 16: it
            //      supplies that line's K rows 4 s + l / 16 and receives output
            //      rows 4 (l / 16) + t.  Velocity derivatives update the auxiliary
            //      slots (S - (1/det J) sum_d n_d,k du_a/dxi_d, over S) and the
            //      velocity divergence (over P); flux derivatives replace the
            //      consumed flux values; a final pass writes R.
            constexpr int NGMAX = (EMAX * NF + 15) / 16;
            constexpr int NW = NT / 64;
            constexpr int GPW = (NGMAX + NW - 1) / NW;
            typedef float v4f __attribute__((ext_vector_type(4)));
            const int lane = tid & 63, wv = tid >> 6, qt = lane >> 4, cl = lane & 15;
            const int ncol = nel * NF;
            auto direction = [&](auto dc) {
                constexpr int d = decltype(dc)::value;
                constexpr int str = d == 0 ? 1 : (d == 1 ? M : M * M);
                v4f out[GPW][6];
#pragma unroll
                for (int u = 0; u < GPW; ++u) {
                    const int col = (wv + u * NW) * 16 + cl;
                    const bool ok = col < ncol;
                    const int el = ok ? col / NF : 0, L = ok ? col - el * NF : 0;
                    const int a = L % M, bb = L / M;
                    const int base = d == 0 ? M * L : (d == 1 ? a + M * M * bb : L);
                    const T *FIm = sFI + ((2 * d) * EMAX + el) * CHP + L;
#pragma unroll
                    for (int f = 0; f < 6; ++f) {
                        const T *fld = f < 3 ? sU + (el * NV + 1 + f) * NS
                                             : sF + (el * 9 + 3 * d + f - 3) * NS;
                        const int comp = f < 3 ? 4 + f : f - 2;
                        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int st2 = 0; st2 < KS; ++st2) {
                            const int kap = 4 * st2 + qt;
                            T bv = T(0);
                            if (ok) {
                                if (kap < M) bv = fld[base + kap * str];
                                else if (kap == M) bv = FIm[comp * NF];
                                else if (kap == M + 1) bv = FIm[EMAX * CHP + comp * NF];
                            }
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(amf[st2], bv, acc, 0, 0, 0);
                        }
                        out[u][f] = acc;
                    }
                }
                __syncthreads();  // every read of this direction's flux values is done
                const T nv[3] = {c.nvec[d][0], c.nvec[d][1], c.nvec[d][2]};
#pragma unroll
                for (int u = 0; u < GPW; ++u) {
                    const int col = (wv + u * NW) * 16 + cl;
                    if (col >= ncol) continue;
                    const int el = col / NF, L = col - el * NF;
                    const int a = L % M, bb = L / M;
                    const int base = d == 0 ? M * L : (d == 1 ? a + M * M * bb : L);
                    T *Ue = sU + el * NV * NS;
                    T *Fe = sF + el * 9 * NS;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int i = 4 * qt + t;
                        if (i < M) {
                            const int q = base + i * str;
                            T dv = T(0);
#pragma unroll
                            for (int f = 0; f < 3; ++f) {
                                const T cd = out[u][f][t];
#pragma unroll
                                for (int k = 0; k < 3; ++k) {
                                    if (DIAG && k != d) continue;
                                    T *slot = Ue + (4 + 3 * f + k) * NS + q;
                                    *slot = fma(-c.inv_det * nv[k], cd, *slot);
                                }
                                if (!DIAG || f == d) dv = fma(nv[f], cd, dv);
                            }
                            Ue[q] = d == 0 ? dv : Ue[q] + dv;
#pragma unroll
                            for (int a2 = 0; a2 < 3; ++a2) Fe[(3 * d + a2) * NS + q] = out[u][3 + a2][t];
                        }
                    }
                }
            };
            direction(Dir<0>{});
            direction(Dir<1>{});
            direction(Dir<2>{});
            __syncthreads();
            for (unsigned t = tid; t < (unsigned)nel * NS; t += NT) {
                const unsigned el = t / NS, q = t - el * NS;
                const unsigned qi = q % M, qj = (q / M) % M, qk = q / (M * M);
                const T *Ue = sU + el * NV * NS;
                const T *Fe = sF + el * 9 * NS;
                T dissP = T(0);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const unsigned id = d == 0 ? qi : (d == 1 ? qj : qk);
                    const unsigned fp = d == 0 ? qj + M * qk : (d == 1 ? qi + M * qk : qi + M * qj);
                    const T *FIm = sFI + ((2 * d) * EMAX + el) * CHP + fp;
                    dissP = fma(gl[id], FIm[0], fma(gr[id], FIm[EMAX * CHP], dissP));
                }
                T *Re = R + ((int64_t)(e0 + el) * NV) * NS + q;
                __builtin_nontemporal_store(-c.inv_det * fma(c.zeta, Ue[q], dissP), Re);
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    __builtin_nontemporal_store(
                        -c.inv_det * ((Fe[a * NS + q] + Fe[(3 + a) * NS + q]) + Fe[(6 + a) * NS + q]),
                        Re + (1 + a) * NS);
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    __builtin_nontemporal_store(-c.invT * Ue[(4 + k) * NS + q], Re + (4 + k) * NS);
            }
        } else if constexpr (LineDiv<P, DIAG>::value) {
            // The three directions' tasks (direction, element, field, line) are
            // read in one phase (882 tasks on 256 threads at p = 6: four passes
            // instead of two per direction) and written after one barrier: flux
            // derivatives over the consumed flux values, auxiliary residuals over
            // S, and each direction's velocity-divergence term n_dd du_d/dxi_d
            // over the velocity u_d, which no task reads any more; the final pass
            // sums the three terms in direction order.
            constexpr int NTD = EMAX * 6 * NF;
            constexpr int TPT = (3 * NTD + NT - 1) / NT;
            const int ntd = nel * 6 * NF;
            const T *gD = ops + OL::Dt;   // uniform operator entries
            const T *gL = ops + OL::gl;
            const T *gR = ops + OL::gr;
            // task t -> direction, element, field, line; first point and stride of the line
            auto decode = [&](unsigned t, unsigned &d, unsigned &el, unsigned &f, unsigned &L,
                              unsigned &base, unsigned &str) {
                d = t / ntd;
                const unsigned r0 = t - d * ntd;
                el = r0 / (6 * NF);
                const unsigned r = r0 - el * (6 * NF);
                f = r / NF;
                L = r - f * NF;
                const unsigned a = L % M, bb = L / M;
                str = d == 0 ? 1u : (d == 1 ? (unsigned)M : (unsigned)(M * M));
                base = d == 0 ? M * L : (d == 1 ? a + M * M * bb : L);
            };
            T outv[TPT][M];
#pragma unroll
            for (int u = 0; u < TPT; ++u) {
                const unsigned t = tid + u * NT;
                if ((int)t < 3 * ntd) {
                    unsigned d, el, f, L, base, str;
                    decode(t, d, el, f, L, base, str);
                    const T *fld = f < 3 ? sU + (el * NV + 1 + f) * NS
                                         : sF + (el * 9 + 3 * d + f - 3) * NS;
                    const unsigned comp = f < 3 ? 4 + f : f - 2;
                    const T *FIm = sFI + ((2 * d) * EMAX + el) * CHP + comp * NF + L;
                    const T fm = FIm[0], fpl = FIm[EMAX * CHP];
                    T in[M];
#pragma unroll
                    for (int l = 0; l < M; ++l) in[l] = fld[base + l * str];
#pragma unroll
                    for (int i = 0; i < M; ++i) {
                        T v = T(0);
#pragma unroll
                        for (int l = 0; l < M; ++l) v = fma(gD[i * M + l], in[l], v);
                        outv[u][i] = fma(gL[i], fm, fma(gR[i], fpl, v));
                    }
                }
            }
            __syncthreads();  // every read of the velocities and flux values is done
#pragma unroll
            for (int u = 0; u < TPT; ++u) {
                const unsigned t = tid + u * NT;
                if ((int)t < 3 * ntd) {
                    unsigned d, el, f, L, base, str;
                    decode(t, d, el, f, L, base, str);
                    T *Ue = sU + el * NV * NS;
                    if (f < 3) {
                        // g[3f+d] = n_dd (corrected d u_f / d xi_d); aux residual (f, d)
                        const T ndd = d == 0 ? c.nvec[0][0] : (d == 1 ? c.nvec[1][1] : c.nvec[2][2]);
#pragma unroll
                        for (int i = 0; i < M; ++i) {
                            const unsigned q = base + i * str;
                            const T gv = outv[u][i] * ndd;
                            T *sq = Ue + (4 + 3 * f + d) * NS + q;
                            *sq = c.invT * fma(c.inv_det, gv, -*sq);
                            if (f == d) Ue[(1 + d) * NS + q] = gv;
                        }
                    } else {
                        T *Fq = sF + (el * 9 + 3 * d + f - 3) * NS + base;
#pragma unroll
                        for (int i = 0; i < M; ++i) Fq[i * str] = outv[u][i];
                    }
                }
            }
            __syncthreads();
            for (unsigned t = tid; t < (unsigned)nel * NS; t += NT) {
                const unsigned el = t / NS, q = t - el * NS;
                const unsigned qi = q % M, qj = (q / M) % M, qk = q / (M * M);
                const T *Ue = sU + el * NV * NS;
                const T *Fe = sF + el * 9 * NS;
                T dissP = T(0);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const unsigned id = d == 0 ? qi : (d == 1 ? qj : qk);
                    const unsigned fp = d == 0 ? qj + M * qk : (d == 1 ? qi + M * qk : qi + M * qj);
                    const T *FIm = sFI + ((2 * d) * EMAX + el) * CHP + fp;
                    dissP = fma(gl[id], FIm[0], fma(gr[id], FIm[EMAX * CHP], dissP));
                }
                const T divV = (Ue[NS + q] + Ue[2 * NS + q]) + Ue[3 * NS + q];
                const T rP = -c.inv_det * fma(c.zeta, divV, dissP);
                T rm[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    rm[a] = -c.inv_det * ((Fe[a * NS + q] + Fe[(3 + a) * NS + q]) + Fe[(6 + a) * NS + q]);
                if constexpr (STG) {
                    // only this thread touches point q's slots in this pass
                    T *Uw = sU + el * NV * NS + q;
                    Uw[0] = rP;
#pragma unroll
                    for (int a = 0; a < 3; ++a) Uw[(1 + a) * NS] = rm[a];
                } else {
                    T *Re = R + ((int64_t)(e0 + el) * NV) * NS + q;
                    __builtin_nontemporal_store(rP, Re);
#pragma unroll
                    for (int a = 0; a < 3; ++a) __builtin_nontemporal_store(rm[a], Re + (1 + a) * NS);
#pragma unroll
                    for (int k = 0; k < 9; ++k)
                        __builtin_nontemporal_store(Ue[(4 + k) * NS + q], Re + (4 + k) * NS);
                }
            }
        } else {
            // ---- stages 3, 5, 6: partially corrected divergence along the three
            //      line families (compile-time strides), correction with the common
            //      fluxes, negate, source.  A thread handles at most KP points.
            //      With STG the residual of each point is held in registers until
            //      every thread has read the tile, then written over the state tile.
            constexpr int KP = (EMAX * NS + NT - 1) / NT;
            T rhold[STG ? KP : 1][NV];
            // residual of point q of element el, each value handed to put(v, value)
            // as soon as it is formed (keeps few values live in the plain path)
            auto point = [&](unsigned el, unsigned q, auto &&put) {
                const unsigned qi = q % M, qj = (q / M) % M, qk = q / (M * M);
                const T *Ue = sU + el * NV * NS;
                const T *Fe = sF + el * 9 * NS;
                // g[3a+k] = sum_d n_d,k (corrected d u_a / d xi_d) = det J d u_a / d x_k
                T g[9], mom[3] = {T(0), T(0), T(0)}, dissP = T(0);
#pragma unroll
                for (int k = 0; k < 9; ++k) g[k] = T(0);
                auto direction = [&](auto dc) {
                    constexpr int d = decltype(dc)::value;
                    constexpr int str = d == 0 ? 1 : (d == 1 ? M : M * M);
                    const unsigned id = d == 0 ? qi : (d == 1 ? qj : qk);
                    const unsigned base = q - id * str;
                    const unsigned fp = d == 0 ? qj + M * qk : (d == 1 ? qi + M * qk : qi + M * qj);
                    const T *FIm = sFI + ((2 * d) * EMAX + el) * CHP + fp;
                    const T *FIp = FIm + EMAX * CHP;
                    const T gld = gl[id], grd = gr[id];
                    const T *Fd = Fe + 3 * d * NS;
                    const T *Drow = Dt + id * M;
                    T du[3] = {T(0), T(0), T(0)}, df[3] = {T(0), T(0), T(0)};
#pragma unroll
                    for (int l = 0; l < M; ++l) {
                        const unsigned ql = base + l * str;
                        const T w = Drow[l];
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            du[a] = fma(w, Ue[(1 + a) * NS + ql], du[a]);
                            df[a] = fma(w, Fd[a * NS + ql], df[a]);
                        }
                    }
                    const T n0 = geo[3 * d], n1 = geo[3 * d + 1], n2 = geo[3 * d + 2];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const T cd = fma(gld, FIm[(4 + a) * NF], fma(grd, FIp[(4 + a) * NF], du[a]));
                        mom[a] += fma(gld, FIm[(1 + a) * NF], fma(grd, FIp[(1 + a) * NF], df[a]));
                        g[3 * a] = fma(cd, n0, g[3 * a]);
                        g[3 * a + 1] = fma(cd, n1, g[3 * a + 1]);
                        g[3 * a + 2] = fma(cd, n2, g[3 * a + 2]);
                    }
                    dissP = fma(gld, FIm[0], fma(grd, FIp[0], dissP));
                };
                direction(Dir<0>{});
                __builtin_amdgcn_sched_barrier(0);
                direction(Dir<1>{});
                __builtin_amdgcn_sched_barrier(0);
                direction(Dir<2>{});
                // P: -(1/detJ) [ zeta (det J div V) + dissipation ]
                const T divV = g[0] + g[4] + g[8];
                put(0, -c.inv_det * fma(c.zeta, divV, dissP));
#pragma unroll
                for (int a = 0; a < 3; ++a) put(1 + a, -c.inv_det * mom[a]);
                // aux (a, k): (1/T) [ d u_a / d x_k - S_ak ]
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    put(4 + k, c.invT * fma(c.inv_det, g[k], -Ue[(4 + k) * NS + q]));
            };
            if constexpr (STG) {
#pragma unroll
                for (int u = 0; u < KP; ++u) {
                    const unsigned t = tid + u * NT;
                    if (t >= (unsigned)nel * NS) break;
                    point(t / NS, t % NS, [&](int v, T val) { rhold[u][v] = val; });
                }
            } else {
                for (unsigned t = tid; t < (unsigned)nel * NS; t += NT) {
                    const unsigned el = t / NS, q = t - el * NS;
                    T *Re = R + ((int64_t)(e0 + el) * NV) * NS + q;
                    point(el, q, [&](int v, T val) { __builtin_nontemporal_store(val, Re + v * NS); });
                }
            }
            if constexpr (STG) {
                __syncthreads();  // every read of the state tile is done
#pragma unroll
                for (int u = 0; u < KP; ++u) {
                    const unsigned t = tid + u * NT;
                    if (t < (unsigned)nel * NS) {
                        const unsigned el = t / NS, q = t - el * NS;
#pragma unroll
                        for (int v = 0; v < NV; ++v) sU[(el * NV + v) * NS + q] = rhold[u][v];
                    }
                }
            }
        }
        if constexpr (STG) {
            // ---- RK stage update over the batch's contiguous [element][variable]
            //      [point] range, the same double arithmetic as the stand-alone
            //      stage kernel (the residual went through LDS, so nothing is
            //      contracted into its last operation).  A thread has at most J
            //      values, taken in chunks of C: the global operands of a chunk
            //      are requested before the first is used, so that the loads of a
            //      wave overlap, with a bounded register cost.
            constexpr int J = (EMAX * NV * NS + NT - 1) / NT;
            constexpr int C = stage_chunk<P, T>() < J ? stage_chunk<P, T>() : J;
            __syncthreads();
            stage_update_batch<J, C, NS, T, P != 4>(sp, [&](unsigned t) -> T & { return sU[t]; }, tid, NT,
                                           (unsigned)nel * NV * NS, e0, ss);
            if (sp.tr_out) {
                // ---- stage 1 of the next residual: the produced state's face
                //      traces (k_trace's values and layout) from the tile, written
                //      to the neighbours' receiving blocks
                using V = typename V16<T>::type;
                constexpr int CH = TL::CH, CHV = TL::CHV, W = TL::W;
                __syncthreads();
                if constexpr (DIAG) {
                    // one task per (direction, element, line)
                    T lmr[M], lpr[M];
#pragma unroll
                    for (int l = 0; l < M; ++l) {
                        lmr[l] = sop[OL::lm + l];
                        lpr[l] = sop[OL::lp + l];
                    }
                    T *TRs = static_cast<T *>(sp.tr_out);
                    for (unsigned t = tid; t < 3u * EMAX * NF; t += NT) {
                        const unsigned dd = t / (EMAX * NF), r = t - dd * (EMAX * NF);
                        const unsigned el = r / NF, L = r - el * NF;
                        if ((int)el >= nel) continue;
                        const T *Ut = sU + el * NV * NS;
                        if (dd == 0)
                            line_traces_out<P, T, 0>(Ut, lmr, lpr, TRs, e0 + el, L, sp.nx, sp.ny, sp.nz, ne);
                        else if (dd == 1)
                            line_traces_out<P, T, 1>(Ut, lmr, lpr, TRs, e0 + el, L, sp.nx, sp.ny, sp.nz, ne);
                        else
                            line_traces_out<P, T, 2>(Ut, lmr, lpr, TRs, e0 + el, L, sp.nx, sp.ny, sp.nz, ne);
                    }
                } else {
                V *TRo = static_cast<V *>(sp.tr_out);
                for (unsigned t = tid; t < 6u * EMAX * CHV; t += NT) {
                    const unsigned f = t / (EMAX * CHV), r = t - f * (EMAX * CHV);
                    const unsigned el = r / CHV, k = r - el * CHV;
                    if ((int)el >= nel) continue;
                    const int d = f >> 1, s = f & 1;
                    const T nh[3] = {geo[9 + 3 * d], geo[10 + 3 * d], geo[11 + 3 * d]};
                    const T *lf = sop + (s ? OL::lp : OL::lm);
                    V x;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const unsigned o = k * W + w;
                        const unsigned cc = o / NF, fp = o - cc * NF;
                        const unsigned a = fp % M, bb = fp / M;
                        const int stride = d == 0 ? 1 : (d == 1 ? M : M * M);
                        const int base = d == 0 ? M * fp : (d == 1 ? a + M * M * bb : fp);
                        x[w] = o < (unsigned)CH
                                   ? trace_value<M, T>(sU + el * NV * NS, d, base, stride, lf, nh, cc, DIAG)
                                   : T(0);
                    }
                    const int64_t nb = neighbour(e0 + el, (int)f, sp.nx, sp.ny, sp.nz);
                    __builtin_nontemporal_store(x, TRo + ((int64_t)(f ^ 1) * ne + nb) * CHV + k);
                }
                }
            }
        }
    }
    if constexpr (STG) {
        if (sp.partial) {
            // fixed-order workgroup sum: wave butterfly, then the waves in order
            __shared__ double red[NT / 64];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int w = 0; w < NT / 64; ++w) t += red[w];
                sp.partial[blockIdx.x] = t;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// k_lines: stages 2-6 as line tasks (diagonal Jacobian).
//
// A workgroup takes LE consecutive elements: it copies their contiguous state
// block into LDS (16-byte vectors where the element size allows), then runs
// three groups of LW waves, one group per direction d.  A lane owns one line
// of direction d of one element (face point L = a + m b of the faces 2d and
// 2d+1).  It reads the m values of the seven variables the direction needs
// (P, u, v, w and S_0d, S_1d, S_2d: with a diagonal Jacobian the transformed
// flux along d involves no other), projects them to both ends of the line (the
// element's own traces, with k_trace's fma chain, so both sides of a face see
// the same bits), reads the neighbours' traces, forms the two common fluxes,
// the transformed flux at the m points and the six partially corrected
// derivatives (three velocities, three momentum fluxes; Table 1 stages 3 and 5
// with the operator Dt and the correction derivatives g_L', g_R').  The
// auxiliary residuals (a, d) are complete at that point and replace S_ad in the
// tile.  The P and momentum parts of the three directions are summed in the
// order x, y, z; where they wait for the sum is a per-shape choice (XR):
//   0  each direction's parts in LDS slots of their own ([3][E][4][m^3]); the
//      final pass sums them while it writes R
//   1  the x direction's in its lanes' registers, y and z in LDS; the x lanes
//      sum and write P and momentum, the auxiliary residuals are copied
//   2  all in registers; after a barrier (the state's P and velocity values are
//      dead by then) the x lanes store theirs over those values, the y lanes
//      add theirs, the z lanes add and scale, and the finished tile is R
//   3  as 2, but the momentum parts are summed between the line task's two
//      halves (after every lane has read the tile's P and velocities for the
//      last time) and the P parts after the second, so that the flux half's
//      and the velocity half's results are never held in registers together
// Modes 2 and 3 need no LDS beyond the tile (more workgroups per CU), at the
// cost of registers and more barriers; mode 3 holds about as many registers
// as mode 0 and is the default.  All four give the same bits.
// ---------------------------------------------------------------------------
#ifndef FR_LE1_D
#define FR_LE1_D 16
#endif
#ifndef FR_LW1_D
#define FR_LW1_D 1
#endif
#ifndef FR_LE2_D
#define FR_LE2_D 7
#endif
#ifndef FR_LW2_D
#define FR_LW2_D 1
#endif
#ifndef FR_LE3_D
#define FR_LE3_D 4
#endif
#ifndef FR_LW3_D
#define FR_LW3_D 1
#endif
#ifndef FR_LE4_D
#define FR_LE4_D 2
#endif
#ifndef FR_LW4_D
#define FR_LW4_D 1
#endif
#ifndef FR_LE5_D
#define FR_LE5_D 1
#endif
#ifndef FR_LW5_D
#define FR_LW5_D 1
#endif
#ifndef FR_LE6_D
#define FR_LE6_D 1
#endif
#ifndef FR_LW6_D
#define FR_LW6_D 1
#endif
#ifndef FR_LE1_F
#define FR_LE1_F 16
#endif
#ifndef FR_LW1_F
#define FR_LW1_F 1
#endif
#ifndef FR_LE2_F
#define FR_LE2_F 7
#endif
#ifndef FR_LW2_F
#define FR_LW2_F 1
#endif
#ifndef FR_LE3_F
#define FR_LE3_F 4
#endif
#ifndef FR_LW3_F
#define FR_LW3_F 1
#endif
#ifndef FR_LE4_F
#define FR_LE4_F 5
#endif
#ifndef FR_LW4_F
#define FR_LW4_F 2
#endif
#ifndef FR_LE5_F
#define FR_LE5_F 3
#endif
#ifndef FR_LW5_F
#define FR_LW5_F 2
#endif
#ifndef FR_LE6_F
#define FR_LE6_F 1
#endif
#ifndef FR_LW6_F
#define FR_LW6_F 1
#endif

#ifndef FR_LX1_D
#define FR_LX1_D 3
#endif
#ifndef FR_LX2_D
#define FR_LX2_D 3
#endif
#ifndef FR_LX3_D
#define FR_LX3_D 3
#endif
#ifndef FR_LX4_D
#define FR_LX4_D 3
#endif
#ifndef FR_LX5_D
#define FR_LX5_D 3
#endif
#ifndef FR_LX6_D
#define FR_LX6_D 3
#endif
#ifndef FR_LX1_F
#define FR_LX1_F 3
#endif
#ifndef FR_LX2_F
#define FR_LX2_F 3
#endif
#ifndef FR_LX3_F
#define FR_LX3_F 0
#endif
#ifndef FR_LX4_F
#define FR_LX4_F 3
#endif
#ifndef FR_LX5_F
#define FR_LX5_F 3
#endif
#ifndef FR_LX6_F
#define FR_LX6_F 3
#endif
// FR_FORM_AUTO's choice per order and precision (0: point form with the trace
// kernel, 1: line form with the trace kernel, 2: halo form, no trace kernel),
// from the measured whole-residual times on the order-sweep lattices (periodic
// box, about 16.6-22.0 M points): the halo form is the fastest everywhere
// (at p = 5 in single precision the line form is within 3%).
#ifndef FR_LA1_D
#define FR_LA1_D 2
#endif
#ifndef FR_LA2_D
#define FR_LA2_D 2
#endif
#ifndef FR_LA3_D
#define FR_LA3_D 2
#endif
#ifndef FR_LA4_D
#define FR_LA4_D 2
#endif
#ifndef FR_LA5_D
#define FR_LA5_D 2
#endif
#ifndef FR_LA6_D
#define FR_LA6_D 2
#endif
#ifndef FR_LA1_F
#define FR_LA1_F 2
#endif
#ifndef FR_LA2_F
#define FR_LA2_F 2
#endif
#ifndef FR_LA3_F
#define FR_LA3_F 2
#endif
#ifndef FR_LA4_F
#define FR_LA4_F 2
#endif
#ifndef FR_LA5_F
#define FR_LA5_F 2
#endif
#ifndef FR_LA6_F
#define FR_LA6_F 2
#endif
// Waves per SIMD the register allocation of the line-form residual kernels aims
// for (at least): 3 at p = 6 in double precision (168 VGPRs with a few values
// spilled, against 171 VGPRs and two waves without the hint: 1.63 against
// 2.13 ms per halo residual on 40^3 hexes); the stage-epilogue kernels take no
// hint (three waves spill there and measured 15-58% slower in double precision).
#ifndef FR_LV_DEFAULT
#define FR_LV_DEFAULT 1
#endif
#ifndef FR_LV1_D
#define FR_LV1_D FR_LV_DEFAULT
#endif
#ifndef FR_LV2_D
#define FR_LV2_D FR_LV_DEFAULT
#endif
#ifndef FR_LV3_D
#define FR_LV3_D FR_LV_DEFAULT
#endif
#ifndef FR_LV4_D
#define FR_LV4_D FR_LV_DEFAULT
#endif
#ifndef FR_LV5_D
#define FR_LV5_D FR_LV_DEFAULT
#endif
#ifndef FR_LV6_D
#define FR_LV6_D 3
#endif
#ifndef FR_LV1_F
#define FR_LV1_F FR_LV_DEFAULT
#endif
#ifndef FR_LV2_F
#define FR_LV2_F FR_LV_DEFAULT
#endif
#ifndef FR_LV3_F
#define FR_LV3_F FR_LV_DEFAULT
#endif
#ifndef FR_LV4_F
#define FR_LV4_F FR_LV_DEFAULT
#endif
#ifndef FR_LV5_F
#define FR_LV5_F FR_LV_DEFAULT
#endif
#ifndef FR_LV6_F
#define FR_LV6_F FR_LV_DEFAULT
#endif
// How fr_rk_step and fr_dual_step apply the RK stage update when the plan's
// residual is the halo form by the automatic choice, per order and precision
// (FR_STAGE_SEPARATE: the halo-form residual, then the separate stage kernel;
// FR_STAGE_POINT: the point form's kernel with the epilogue; FR_STAGE_HALO: the
// halo form's kernel with the epilogue), from the measured RK4 step and dual
// pseudo-step times on Taylor-Green lattices of 1.8-33.6 M points (the dual
// pseudo-step decides).
#ifndef FR_SA1_D
#define FR_SA1_D FR_STAGE_HALO
#endif
#ifndef FR_SA2_D
#define FR_SA2_D FR_STAGE_HALO
#endif
#ifndef FR_SA3_D
#define FR_SA3_D FR_STAGE_HALO
#endif
#ifndef FR_SA4_D
#define FR_SA4_D FR_STAGE_POINT
#endif
#ifndef FR_SA5_D
#define FR_SA5_D FR_STAGE_HALO
#endif
#ifndef FR_SA6_D
#define FR_SA6_D FR_STAGE_HALO
#endif
#ifndef FR_SA1_F
#define FR_SA1_F FR_STAGE_HALO
#endif
#ifndef FR_SA2_F
#define FR_SA2_F FR_STAGE_HALO
#endif
#ifndef FR_SA3_F
#define FR_SA3_F FR_STAGE_HALO
#endif
#ifndef FR_SA4_F
#define FR_SA4_F FR_STAGE_HALO
#endif
#ifndef FR_SA5_F
#define FR_SA5_F FR_STAGE_POINT
#endif
#ifndef FR_SA6_F
#define FR_SA6_F FR_STAGE_HALO
#endif
template <int P, typename T> struct StageAuto;
#define FR_SAUTO(PP, TT, S) \
    template <> struct StageAuto<PP, TT> { static constexpr int value = FR_SA##PP##_##S; };
FR_SAUTO(1, double, D)
FR_SAUTO(2, double, D)
FR_SAUTO(3, double, D)
FR_SAUTO(4, double, D)
FR_SAUTO(5, double, D)
FR_SAUTO(6, double, D)
FR_SAUTO(1, float, F)
FR_SAUTO(2, float, F)
FR_SAUTO(3, float, F)
FR_SAUTO(4, float, F)
FR_SAUTO(5, float, F)
FR_SAUTO(6, float, F)
#undef FR_SAUTO

template <int P, typename T> struct LinesShape;
#define FR_LSHAPE(PP, TT, S)                                                        \
    template <> struct LinesShape<PP, TT> {                                         \
        static constexpr int E = FR_LE##PP##_##S, W = FR_LW##PP##_##S, NT = 192 * W; \
        static_assert(E * (PP + 1) * (PP + 1) <= 64 * W, "one lane per line");       \
        static constexpr int XR = FR_LX##PP##_##S;                                   \
        static constexpr int AUTO = FR_LA##PP##_##S;                                 \
        static constexpr int WPE = FR_LV##PP##_##S;                                  \
        static_assert(LinesLds<PP, TT>::values(E, XR) * sizeof(TT) <= 160 * 1024, "LDS"); \
    };
FR_LSHAPE(1, double, D)
FR_LSHAPE(2, double, D)
FR_LSHAPE(3, double, D)
FR_LSHAPE(4, double, D)
FR_LSHAPE(5, double, D)
FR_LSHAPE(6, double, D)
FR_LSHAPE(1, float, F)
FR_LSHAPE(2, float, F)
FR_LSHAPE(3, float, F)
FR_LSHAPE(4, float, F)
FR_LSHAPE(5, float, F)
FR_LSHAPE(6, float, F)
#undef FR_LSHAPE

// The m values of one line (first value p, stride STR) into registers; an
// x-line (STR = 1) is contiguous and is read in 16- or 8-byte vectors where
// its length and the element size keep them aligned.
template <int M, int STR, typename T>
__device__ __forceinline__ void line_load(const T *__restrict__ p, T (&x)[M])
{
    if constexpr (STR == 1 && (M * sizeof(T)) % 16 == 0) {
        using V = typename V16<T>::type;
        constexpr int W = 16 / sizeof(T);
#pragma unroll
        for (int k = 0; k < M / W; ++k) {
            const V v = reinterpret_cast<const V *>(p)[k];
#pragma unroll
            for (int w = 0; w < W; ++w) x[k * W + w] = v[w];
        }
    } else if constexpr (STR == 1 && sizeof(T) == 4 && M % 2 == 0) {
        typedef float f2v __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int k = 0; k < M / 2; ++k) {
            const f2v v = reinterpret_cast<const f2v *>(p)[k];
            x[2 * k] = v[0];
            x[2 * k + 1] = v[1];
        }
    } else {
#pragma unroll
        for (int l = 0; l < M; ++l) x[l] = p[l * STR];
    }
}

template <int M, int STR, typename T>
__device__ __forceinline__ void line_store(T *__restrict__ p, const T (&x)[M])
{
    if constexpr (STR == 1 && (M * sizeof(T)) % 16 == 0) {
        using V = typename V16<T>::type;
        constexpr int W = 16 / sizeof(T);
#pragma unroll
        for (int k = 0; k < M / W; ++k) {
            V v;
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] = x[k * W + w];
            __builtin_nontemporal_store(v, reinterpret_cast<V *>(p) + k);
        }
    } else if constexpr (STR == 1 && sizeof(T) == 4 && M % 2 == 0) {
        typedef float f2v __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int k = 0; k < M / 2; ++k) {
            f2v v;
            v[0] = x[2 * k];
            v[1] = x[2 * k + 1];
            __builtin_nontemporal_store(v, reinterpret_cast<f2v *>(p) + k);
        }
    } else {
#pragma unroll
        for (int l = 0; l < M; ++l) __builtin_nontemporal_store(x[l], p + l * STR);
    }
}



// The m values of one line into LDS (the layout of line_load).
template <int M, int STR, typename T>
__device__ __forceinline__ void line_put(T *__restrict__ p, const T (&x)[M])
{
    if constexpr (STR == 1 && (M * sizeof(T)) % 16 == 0) {
        using V = typename V16<T>::type;
        constexpr int W = 16 / sizeof(T);
#pragma unroll
        for (int k = 0; k < M / W; ++k) {
            V v;
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] = x[k * W + w];
            reinterpret_cast<V *>(p)[k] = v;
        }
    } else {
#pragma unroll
        for (int l = 0; l < M; ++l) p[l * STR] = x[l];
    }
}

// Whether the line task's row loop stays rolled (per order and precision;
// fewer live registers against loop overhead).
#ifndef FR_LROLL
#define FR_LROLL 1
#endif
template <int P, typename T> struct LinesRolled {
    static constexpr bool value = FR_LROLL != 0;
};

// One direction's line task on the element tile Ut (LDS, updated in place),
// in three phases that a caller may separate by barriers:
//   lt_fluxes      the line's own traces (k_trace's chain), the two common
//                  fluxes FIm / FIp, the transformed momentum fluxes and their
//                  corrected derivatives (momentum parts)
//   lt_velocities  the line's velocities (read from the tile)
//   lt_derivs      their corrected derivatives: the auxiliary residuals (a, D)
//                  replace S_aD in the tile (only this lane touches those
//                  values) and the P part zeta n_DD du_D/dxi_D + dissipation
// sop: the operator block in LDS; oth{m,p}: the neighbours' traces on the
// line's two face points.  The P and momentum parts go to sCd (this
// direction's [4][m^3] slots of the element) or, with XR, to ctb[0..3][r] in
// registers.
template <int P, typename T, int D>
__device__ __forceinline__ int lt_base(int L)
{
    constexpr int M = P + 1;
    const int a = L % M, b = L / M;
    return D == 0 ? M * L : (D == 1 ? a + M * M * b : L);
}

template <int P, typename T, int D, bool XR>
__device__ __forceinline__ void lt_fluxes(T *__restrict__ Ut, const T *__restrict__ sop,
                                          const T (&othm)[NTR], const T (&othp)[NTR],
                                          const Consts<T> &c, int L, T *__restrict__ sCd,
                                          T (&ctb)[4][P + 1], T (&FIm)[NTR], T (&FIp)[NTR])
{
    constexpr int M = P + 1, NS = M * M * M;
    constexpr int STR = D == 0 ? 1 : (D == 1 ? M : M * M);
    using OL = OpsLayout<M>;
    const int base = lt_base<P, T, D>(L);
    T *Ue = Ut + base;
    {
        T lm[M], lp[M];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            lm[l] = sop[OL::lm + l];
            lp[l] = sop[OL::lp + l];
        }
        T ownm[NTR], ownp[NTR];
#pragma unroll
        for (int cc = 0; cc < NTR; ++cc) {
            T x[M];
            line_load<M, STR>(Ue + (cc < 4 ? cc : 4 + 3 * (cc - 4) + D) * NS, x);
            T am = T(0), ap = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) {
                am = fma(lm[l], x[l], am);
                ap = fma(lp[l], x[l], ap);
            }
            ownm[cc] = am;
            ownp[cc] = ap;
        }
        const T nh[3] = {c.nhat[D][0], c.nhat[D][1], c.nhat[D][2]};
        common_flux_sided<T>(ownm, othm, false, nh, c.nmag[D], c.zeta, c.nu, FIm);
        common_flux_sided<T>(ownp, othp, true, nh, c.nmag[D], c.zeta, c.nu, FIp);
    }
    // the lines are read again below rather than kept live through the
    // common-flux arithmetic (the barrier stops the compiler from reusing the
    // first reads)
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    const T ndd = c.nvec[D][D];
    // the transformed momentum fluxes F_D,i = n_DD (u_i u_D + P delta_iD -
    // nu S_iD) along the line (S is still the state's here)
    T F[3][M];
    {
        T X[3][M], Pl[M];
#pragma unroll
        for (int ia = 0; ia < 3; ++ia) line_load<M, STR>(Ue + (1 + ia) * NS, X[ia]);
        line_load<M, STR>(Ue, Pl);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T Sl[M];
            line_load<M, STR>(Ue + (4 + 3 * i + D) * NS, Sl);
#pragma unroll
            for (int l = 0; l < M; ++l) {
                const T vn = X[D][l] * ndd;
                const T sn = Sl[l] * ndd;
                F[i][l] = i == D ? fma(X[i][l], vn, fma(Pl[l], ndd, -c.nu * sn))
                                 : fma(X[i][l], vn, -c.nu * sn);
            }
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    // the corrected derivatives of the three fluxes, row by row (the fluxes
    // and the velocities are never live at once)
    auto rowF = [&](int r) {
        // one row's operator values at a time (bounds the live registers)
        __builtin_amdgcn_sched_barrier(0);
        T Dr[M];
#pragma unroll
        for (int l = 0; l < M; ++l) Dr[l] = sop[OL::Dt + r * M + l];
        const T glr = sop[OL::gl + r], grr = sop[OL::gr + r];
        const int q = r * STR;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T s = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) s = fma(Dr[l], F[i][l], s);
            const T cf = fma(glr, FIm[1 + i], fma(grr, FIp[1 + i], s));
            if constexpr (XR) ctb[1 + i][r] = cf;
            else sCd[(1 + i) * NS + base + q] = cf;
        }
    };
    // with XR the row index selects registers, so the loop is unrolled;
    // otherwise it stays rolled (fewer live registers)
    if constexpr (XR || !LinesRolled<P, T>::value) {
#pragma unroll
        for (int r = 0; r < M; ++r) rowF(r);
    } else {
#pragma unroll 1
        for (int r = 0; r < M; ++r) rowF(r);
    }
}

template <int P, typename T, int D>
__device__ __forceinline__ void lt_velocities(const T *__restrict__ Ut, int L, T (&X)[3][P + 1])
{
    constexpr int M = P + 1, NS = M * M * M;
    constexpr int STR = D == 0 ? 1 : (D == 1 ? M : M * M);
    __asm__ volatile("" ::: "memory");  // read the velocities again
    __builtin_amdgcn_sched_barrier(0);
    const T *Ue = Ut + lt_base<P, T, D>(L);
#pragma unroll
    for (int ia = 0; ia < 3; ++ia) line_load<M, STR>(Ue + (1 + ia) * NS, X[ia]);
}

template <int P, typename T, int D, bool XR>
__device__ __forceinline__ void lt_derivs(T *__restrict__ Ut, const T *__restrict__ sop,
                                          const T (&X)[3][P + 1], const T (&FIm)[NTR],
                                          const T (&FIp)[NTR], const Consts<T> &c, int L,
                                          T *__restrict__ sCd, T (&ctb)[4][P + 1])
{
    constexpr int M = P + 1, NS = M * M * M;
    constexpr int STR = D == 0 ? 1 : (D == 1 ? M : M * M);
    using OL = OpsLayout<M>;
    const int base = lt_base<P, T, D>(L);
    T *Ue = Ut + base;
    const T ndd = c.nvec[D][D];
    auto rowV = [&](int r) {
        __builtin_amdgcn_sched_barrier(0);
        T Dr[M];
#pragma unroll
        for (int l = 0; l < M; ++l) Dr[l] = sop[OL::Dt + r * M + l];
        const T glr = sop[OL::gl + r], grr = sop[OL::gr + r];
        const int q = r * STR;
        T pc = T(0);
#pragma unroll
        for (int va = 0; va < 3; ++va) {
            T s = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) s = fma(Dr[l], X[va][l], s);
            const T cd = fma(glr, FIm[4 + va], fma(grr, FIp[4 + va], s));
            const T gv = cd * ndd;
            // S_aD at this point is replaced by the auxiliary residual (only
            // this lane reads or writes it from here on)
            T *sq = Ue + (4 + 3 * va + D) * NS + q;
            *sq = c.invT * fma(c.inv_det, gv, -*sq);
            if (va == D) pc = fma(c.zeta, gv, fma(glr, FIm[0], grr * FIp[0]));
        }
        if constexpr (XR) ctb[0][r] = pc;
        else sCd[base + q] = pc;
    };
    if constexpr (XR || !LinesRolled<P, T>::value) {
#pragma unroll
        for (int r = 0; r < M; ++r) rowV(r);
    } else {
#pragma unroll 1
        for (int r = 0; r < M; ++r) rowV(r);
    }
}

// The three phases in a row.
template <int P, typename T, int D, bool XR>
__device__ __forceinline__ void line_task(T *__restrict__ Ut, const T *__restrict__ sop,
                                          const T (&othm)[NTR], const T (&othp)[NTR],
                                          const Consts<T> &c, int L, T *__restrict__ sCd,
                                          T (&ctb)[4][P + 1])
{
    T FIm[NTR], FIp[NTR], X[3][P + 1];
    lt_fluxes<P, T, D, XR>(Ut, sop, othm, othp, c, L, sCd, ctb, FIm, FIp);
    lt_velocities<P, T, D>(Ut, L, X);
    lt_derivs<P, T, D, XR>(Ut, sop, X, FIm, FIp, c, L, sCd, ctb);
}

// The face trace of a neighbour element, from its state Un (global memory or
// the tile): its end lf (l(+1) for the minus neighbour, l(-1) for the plus
// neighbour) of the direction-D line through face point L, for the seven trace
// variables, with k_trace's fma chain (so the values have the bits k_trace
// would write).
template <int P, typename T, int D>
__device__ __forceinline__ void nbr_trace(const T *__restrict__ Un, int L, const T *__restrict__ lf,
                                          T (&out)[NTR])
{
    constexpr int M = P + 1, NS = M * M * M;
    constexpr int STR = D == 0 ? 1 : (D == 1 ? M : M * M);
    const int a = L % M, b = L / M;
    const T *X = Un + (D == 0 ? M * L : (D == 1 ? a + M * M * b : L));
#pragma unroll
    for (int cc = 0; cc < NTR; ++cc) {
        const T *Xc = X + (cc < 4 ? cc : 4 + 3 * (cc - 4) + D) * NS;
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < M; ++l) acc = fma(lf[l], Xc[l * STR], acc);
        out[cc] = acc;
    }
}

// Whether the halo form's stage-epilogue kernel loops over batches with a grid
// bounded by the partial sums or takes one batch per workgroup.  The loop
// holds 20-50 more VGPRs (a wave of occupancy at p = 2-5) but saves workgroup
// launches where batches are small; measured per order and precision on the
// dual pseudo-step.
#ifndef FR_SL1_D
#define FR_SL1_D 1
#endif
#ifndef FR_SL2_D
#define FR_SL2_D 0
#endif
#ifndef FR_SL3_D
#define FR_SL3_D 0
#endif
#ifndef FR_SL4_D
#define FR_SL4_D 0
#endif
#ifndef FR_SL5_D
#define FR_SL5_D 0
#endif
#ifndef FR_SL6_D
#define FR_SL6_D 1
#endif
#ifndef FR_SL1_F
#define FR_SL1_F 1
#endif
#ifndef FR_SL2_F
#define FR_SL2_F 0
#endif
#ifndef FR_SL3_F
#define FR_SL3_F 0
#endif
#ifndef FR_SL4_F
#define FR_SL4_F 0
#endif
#ifndef FR_SL5_F
#define FR_SL5_F 1
#endif
#ifndef FR_SL6_F
#define FR_SL6_F 1
#endif
template <int P, typename T> struct StageLoop;
#define FR_SLOOP(PP, TT, S) \
    template <> struct StageLoop<PP, TT> { static constexpr bool value = FR_SL##PP##_##S != 0; };
FR_SLOOP(1, double, D)
FR_SLOOP(2, double, D)
FR_SLOOP(3, double, D)
FR_SLOOP(4, double, D)
FR_SLOOP(5, double, D)
FR_SLOOP(6, double, D)
FR_SLOOP(1, float, F)
FR_SLOOP(2, float, F)
FR_SLOOP(3, float, F)
FR_SLOOP(4, float, F)
FR_SLOOP(5, float, F)
FR_SLOOP(6, float, F)
#undef FR_SLOOP

// Values per thread whose global operands the halo form's stage epilogue
// requests at once, per order and precision (as stage_chunk for the point
// form; measured: 16 spills, 1 leaves too few loads in flight).
// FR_LSTG_CHUNK overrides the table.
template <int P, typename T>
constexpr int line_stage_chunk()
{
#ifdef FR_LSTG_CHUNK
    return FR_LSTG_CHUNK;
#else
    constexpr int d[PMAX + 1] = {0, 8, 8, 8, 8, 8, 8};
    constexpr int f[PMAX + 1] = {0, 8, 8, 4, 4, 8, 8};
    return sizeof(T) == 8 ? d[P] : f[P];
#endif
}

template <int P, typename T, bool HALO, bool STG>
__global__ void __launch_bounds__((LinesShape<P, T>::NT))
    __attribute__((amdgpu_waves_per_eu(STG ? 1 : LinesShape<P, T>::WPE, 8)))
    k_lines(const T *__restrict__ U, const T *__restrict__ TR, T *__restrict__ R,
            const T *__restrict__ ops0, Consts<T> c, int nx, int ny, int nz, StageSpec sp)
{
    const int ne = nx * ny * nz;
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    constexpr int E = LinesShape<P, T>::E, W = LinesShape<P, T>::W, NT = LinesShape<P, T>::NT;
    constexpr int XR = LinesShape<P, T>::XR;
    using LL = LinesLds<P, T>;
    using TL = TraceLayout<M, T>;
    using OL = OpsLayout<M>;
    constexpr int EP = LL::EP, RAW = LL::raw;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sop0 = reinterpret_cast<T *>(smem_raw);  // operators
    T *sU = sop0 + LL::OPS;                      // [E][EP] state tile
    // P and momentum parts per direction, [3][E][4][NS] (XR = 1: the x
    // direction's stay in its lanes' registers and only y and z are here;
    // XR = 2, 3: none here)
    T *sC = sU + E * EP - (XR == 1 ? 4 * E * NS : 0);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int d = wave / W;
    const int t = (wave - d * W) * 64 + (threadIdx.x & 63);
    const int el = t / NF, L = t - el * NF;
    const int64_t nbt = ((int64_t)ne + E - 1) / E;
    if (threadIdx.x < OL::size) sop0[threadIdx.x] = ops0[threadIdx.x];
    // with STG: sum of (k*_V)^2 over this workgroup's stage updates
    double ss = 0.0;
    auto run_batch = [&](int64_t e0, int nel) {
        // the operator blocks through an offset the compiler cannot see, so that
        // a loop over batches reloads them instead of holding them in registers
        const int oz = opaque_zero();
        const T *sop = sop0 + oz;
        const T *ops = ops0 + oz;
        const bool act = el < nel;
        const int64_t e = e0 + el;
        // the neighbours' traces on this lane's line, requested before the state:
        // from the trace array, or with HALO from the neighbours' own states (from
        // global memory for a neighbour outside the batch, from the tile after it
        // is loaded otherwise)
        T othm[NTR], othp[NTR];
        int64_t nbm = 0, nbp = 0;
        bool inm = false, inp = false;
        if (act) {
            if constexpr (HALO) {
                nbm = neighbour(e, 2 * d, nx, ny, nz);
                nbp = neighbour(e, 2 * d + 1, nx, ny, nz);
                inm = nbm >= e0 && nbm < e0 + nel;
                inp = nbp >= e0 && nbp < e0 + nel;
                auto from_global = [&](auto dc) {
                    constexpr int DD = decltype(dc)::value;
                    if (!inm) nbr_trace<P, T, DD>(U + nbm * RAW, L, ops + OL::lp, othm);
                    if (!inp) nbr_trace<P, T, DD>(U + nbp * RAW, L, ops + OL::lm, othp);
                };
                if (d == 0) from_global(Dir<0>{});
                else if (d == 1) from_global(Dir<1>{});
                else from_global(Dir<2>{});
            } else {
                const T *tm = TR + ((int64_t)(2 * d) * ne + e) * TL::CHP + L;
                const T *tp = TR + ((int64_t)(2 * d + 1) * ne + e) * TL::CHP + L;
#pragma unroll
                for (int cc = 0; cc < NTR; ++cc) {
                    othm[cc] = __builtin_nontemporal_load(tm + cc * NF);
                    othp[cc] = __builtin_nontemporal_load(tp + cc * NF);
                }
            }
        }
        // the batch's state block into LDS
        tile_load<P, T, NT>(U + e0 * RAW, sU, nel);
        __syncthreads();
        if constexpr (HALO) {
            if (act && (inm || inp)) {
                auto from_tile = [&](auto dc) {
                    constexpr int DD = decltype(dc)::value;
                    if (inm) nbr_trace<P, T, DD>(sU + (nbm - e0) * EP, L, sop + OL::lp, othm);
                    if (inp) nbr_trace<P, T, DD>(sU + (nbp - e0) * EP, L, sop + OL::lm, othp);
                };
                if (d == 0) from_tile(Dir<0>{});
                else if (d == 1) from_tile(Dir<1>{});
                else from_tile(Dir<2>{});
            }
            // a neighbour's S_ad is replaced by its auxiliary residual in the line
            // task; with several waves per direction that lane may be in another
            // wave, so every wave finishes these reads first
            if constexpr (W > 1) __syncthreads();
        }
        T ctb[4][M];
        const T mid = -c.inv_det;
        // the parts ctb[k0..k1) of this lane's line added over the tile's P and
        // velocity values (x stores, y adds, z adds and scales by -1/det J)
        auto add_lines = [&](auto dc, auto k0c, auto k1c) {
            constexpr int DD = decltype(dc)::value;
            constexpr int K0 = decltype(k0c)::value, K1 = decltype(k1c)::value;
            constexpr int STR = DD == 0 ? 1 : (DD == 1 ? M : M * M);
            T *Ue = sU + el * EP + lt_base<P, T, DD>(L);
#pragma unroll
            for (int k = K0; k < K1; ++k) {
                T o[M];
                if constexpr (DD == 0) {
#pragma unroll
                    for (int r = 0; r < M; ++r) o[r] = ctb[k][r];
                } else {
                    line_load<M, STR>(Ue + k * NS, o);
#pragma unroll
                    for (int r = 0; r < M; ++r) o[r] = o[r] + ctb[k][r];
                    if constexpr (DD == 2) {
#pragma unroll
                        for (int r = 0; r < M; ++r) o[r] = mid * o[r];
                    }
                }
                line_put<M, STR>(Ue + k * NS, o);
            }
        };
        if constexpr (XR == 3) {
            // the momentum parts are summed between the two halves of the line
            // task, once every lane has read the tile's P and velocities, and the
            // P parts after it: the fluxes' and the velocities' parts are never
            // held in registers together
            T FIm[NTR], FIp[NTR], X[3][M];
            T *Ut = sU + el * EP;
            if (act) {
                auto ph1 = [&](auto dc) {
                    constexpr int DD = decltype(dc)::value;
                    lt_fluxes<P, T, DD, true>(Ut, sop, othm, othp, c, L, nullptr, ctb, FIm, FIp);
                    lt_velocities<P, T, DD>(Ut, L, X);
                };
                if (d == 0) ph1(Dir<0>{});
                else if (d == 1) ph1(Dir<1>{});
                else ph1(Dir<2>{});
            }
            __syncthreads();
            if (act && d == 0) add_lines(Dir<0>{}, Dir<1>{}, Dir<4>{});
            __syncthreads();
            if (act && d == 1) add_lines(Dir<1>{}, Dir<1>{}, Dir<4>{});
            __syncthreads();
            if (act && d == 2) add_lines(Dir<2>{}, Dir<1>{}, Dir<4>{});
            if (act) {
                if (d == 0) lt_derivs<P, T, 0, true>(Ut, sop, X, FIm, FIp, c, L, nullptr, ctb);
                else if (d == 1) lt_derivs<P, T, 1, true>(Ut, sop, X, FIm, FIp, c, L, nullptr, ctb);
                else lt_derivs<P, T, 2, true>(Ut, sop, X, FIm, FIp, c, L, nullptr, ctb);
            }
            if (act && d == 0) add_lines(Dir<0>{}, Dir<0>{}, Dir<1>{});
            __syncthreads();
            if (act && d == 1) add_lines(Dir<1>{}, Dir<0>{}, Dir<1>{});
            __syncthreads();
            if (act && d == 2) add_lines(Dir<2>{}, Dir<0>{}, Dir<1>{});
        } else {
            if (act) {
                T *Ut = sU + el * EP;
                T *sCd = sC + ((d * E + el) * 4) * NS;
                if (d == 0) line_task<P, T, 0, (XR >= 1)>(Ut, sop, othm, othp, c, L, sCd, ctb);
                else if (d == 1) line_task<P, T, 1, (XR == 2)>(Ut, sop, othm, othp, c, L, sCd, ctb);
                else line_task<P, T, 2, (XR == 2)>(Ut, sop, othm, othp, c, L, sCd, ctb);
            }
            __syncthreads();
        }
        // R of the batch: P and momentum summed over the three directions in the
        // order x, y, z and scaled by -1/det J, the auxiliary residuals from the
        // tile.  Without STG it goes to R; with STG it stays in the tile for the
        // stage update.
        if constexpr (XR == 3) {
            if constexpr (!STG) {
                __syncthreads();
                tile_store<P, T, NT>(sU, R + e0 * RAW, nel);
            }
        } else if constexpr (XR == 2) {
            // summed over the tile's P and velocity values, one direction after
            // the other
            if (act && d == 0) add_lines(Dir<0>{}, Dir<0>{}, Dir<4>{});
            __syncthreads();
            if (act && d == 1) add_lines(Dir<1>{}, Dir<0>{}, Dir<4>{});
            __syncthreads();
            if (act && d == 2) add_lines(Dir<2>{}, Dir<0>{}, Dir<4>{});
            if constexpr (!STG) {
                __syncthreads();
                tile_store<P, T, NT>(sU, R + e0 * RAW, nel);
            }
        } else if constexpr (XR == 1) {
            // x lanes: their own parts plus those of y and z at the x-line's points
            if (act && d == 0) {
                const T *cy = sC + ((E + el) * 4) * NS + M * L;
                const T *cz = sC + ((2 * E + el) * 4) * NS + M * L;
                T *Re = R + e * (NV * NS) + M * L;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    T o[M];
#pragma unroll
                    for (int r = 0; r < M; ++r) o[r] = mid * ((ctb[k][r] + cy[k * NS + r]) + cz[k * NS + r]);
                    if constexpr (STG) line_put<M, 1>(sU + el * EP + M * L + k * NS, o);
                    else line_store<M, 1>(Re + k * NS, o);
                }
            }
            if constexpr (!STG) {
                // every thread: the auxiliary residuals from the tile
                T *dst = R + e0 * RAW;
                constexpr int A0 = 4 * NS, NA = 9 * NS;
                if constexpr (LL::VEC && (A0 * sizeof(T)) % 16 == 0) {
                    using V = typename V16<T>::type;
                    constexpr int VW = 16 / sizeof(T), CPE = NA / VW;
                    const int nch = nel * CPE;
#pragma unroll 4
                    for (int k = threadIdx.x; k < nch; k += NT) {
                        const int ek = k / CPE, o = k - ek * CPE;
                        __builtin_nontemporal_store(reinterpret_cast<const V *>(sU + ek * EP + A0)[o],
                                                    reinterpret_cast<V *>(dst + ek * RAW + A0) + o);
                    }
                } else {
                    const int nv = nel * NA;
#pragma unroll 4
                    for (int k = threadIdx.x; k < nv; k += NT) {
                        const int ek = k / NA, o = k - ek * NA;
                        __builtin_nontemporal_store(sU[ek * EP + A0 + o], dst + ek * RAW + A0 + o);
                    }
                }
            }
        } else {
            // one pass over the batch: the three directions' parts from their
            // slots, the auxiliary residuals from the tile
            T *dst = R + e0 * RAW;
            if constexpr (LL::VEC) {
                using V = typename V16<T>::type;
                constexpr int VW = 16 / sizeof(T), CPE = RAW / VW, C4 = 4 * NS / VW;
                static_assert((4 * NS) % VW == 0, "P and momentum in whole chunks");
                const int nch = nel * CPE;
#pragma unroll 4
                for (int k = threadIdx.x; k < nch; k += NT) {
                    const int ek = k / CPE, o = k - ek * CPE;
                    V x;
                    if (o < C4) {
                        const V *cx = reinterpret_cast<const V *>(sC + (ek * 4) * NS) + o;
                        const V *cy = reinterpret_cast<const V *>(sC + ((E + ek) * 4) * NS) + o;
                        const V *cz = reinterpret_cast<const V *>(sC + ((2 * E + ek) * 4) * NS) + o;
                        const V vx = *cx, vy = *cy, vz = *cz;
#pragma unroll
                        for (int w = 0; w < VW; ++w) x[w] = mid * ((vx[w] + vy[w]) + vz[w]);
                        if constexpr (STG) reinterpret_cast<V *>(sU + ek * EP)[o] = x;
                    } else {
                        x = reinterpret_cast<const V *>(sU + ek * EP)[o];
                    }
                    if constexpr (!STG) __builtin_nontemporal_store(x, reinterpret_cast<V *>(dst) + k);
                }
            } else {
                const int nv = nel * RAW;
#pragma unroll 4
                for (int k = threadIdx.x; k < nv; k += NT) {
                    const int ek = k / RAW, o = k - ek * RAW;
                    T x;
                    if (o < 4 * NS) {
                        const T *cx = sC + (ek * 4) * NS + o;
                        x = mid * ((cx[0] + cx[E * 4 * NS]) + cx[2 * E * 4 * NS]);
                        if constexpr (STG) sU[ek * EP + o] = x;
                    } else {
                        x = sU[ek * EP + o];
                    }
                    if constexpr (!STG) __builtin_nontemporal_store(x, dst + k);
                }
            }
        }
        if constexpr (STG) {
            // ---- the RK stage update of the batch from its residual in the tile
            constexpr int J = (E * RAW + NT - 1) / NT;
            constexpr int C = line_stage_chunk<P, T>() < J ? line_stage_chunk<P, T>() : J;
            __syncthreads();
            stage_update_batch<J, C, NS, T, true>(
                sp, [&](unsigned q) -> T & { return sU[(q / RAW) * EP + q % RAW]; }, threadIdx.x, NT,
                (unsigned)nel * RAW, e0, ss);
        }
    };
    auto batch_at = [&](int64_t bt) {
        const int64_t e0 = bt * E;
        run_batch(e0, (int)min((int64_t)E, (int64_t)ne - e0));
    };
    if constexpr (STG && StageLoop<P, T>::value) {
        // the stage epilogue's grid bounded by its partial sums: a workgroup
        // may take several batches
        for (int64_t bt = blockIdx.x; bt < nbt; bt += gridDim.x) {
            if (bt != (int64_t)blockIdx.x) __syncthreads();  // the tile is free again
            batch_at(bt);
        }
    } else {
        // one batch per workgroup (the partial sums take one slot per batch)
        batch_at(blockIdx.x);
    }
    if constexpr (STG) {
        if (sp.partial) {
            // fixed-order workgroup sum: wave butterfly, then the waves in order
            __shared__ double red[NT / 64];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
            __syncthreads();
            if (threadIdx.x == 0) {
                double tsum = 0.0;
                for (int w = 0; w < NT / 64; ++w) tsum += red[w];
                sp.partial[blockIdx.x] = tsum;
            }
        }
    }
}

// The two face traces (7 values each) of the direction-D line through face
// point L of the element tile Ut (element pitch of the line form), written to
// the receiving blocks of the neighbours across faces 2D and 2D+1.
template <int P, typename T, int D>
__device__ __forceinline__ void line_traces_out(const T *__restrict__ Ut, const T *__restrict__ lm,
                                                const T *__restrict__ lp, T *__restrict__ TR,
                                                int64_t e, int L, int nx, int ny, int nz, int64_t ne)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    constexpr int STR = D == 0 ? 1 : (D == 1 ? M : M * M);
    using TL = TraceLayout<M, T>;
    const int a = L % M, b = L / M;
    const int base = D == 0 ? M * L : (D == 1 ? a + M * M * b : L);
    const T *Ue = Ut + base;
    T tm[NTR], tp[NTR];
#pragma unroll
    for (int cc = 0; cc < NTR; ++cc) {
        T x[M];
        line_load<M, STR>(Ue + (cc < 4 ? cc : 4 + 3 * (cc - 4) + D) * NS, x);
        T am = T(0), ap = T(0);
#pragma unroll
        for (int l = 0; l < M; ++l) {
            am = fma(lm[l], x[l], am);
            ap = fma(lp[l], x[l], ap);
        }
        tm[cc] = am;
        tp[cc] = ap;
    }
    // the minus face's values go to the minus neighbour's plus-face block and
    // the plus face's to the plus neighbour's minus-face block
    const int64_t nbm = neighbour(e, 2 * D, nx, ny, nz), nbp = neighbour(e, 2 * D + 1, nx, ny, nz);
    T *dm = TR + ((int64_t)(2 * D + 1) * ne + nbm) * TL::CHP + L;
    T *dp = TR + ((int64_t)(2 * D) * ne + nbp) * TL::CHP + L;
#pragma unroll
    for (int cc = 0; cc < NTR; ++cc) {
        __builtin_nontemporal_store(tm[cc], dm + cc * NF);
        __builtin_nontemporal_store(tp[cc], dp + cc * NF);
    }
}

// ---------------------------------------------------------------------------
// k_trace_lines: stage 1 for a diagonal Jacobian.  A workgroup copies a batch
// of TLE consecutive elements into LDS (the line form's tile); one task per
// (direction d, element, line) projects the seven trace variables (P, u, v, w,
// S_0d, S_1d, S_2d) to both ends of its line with k_trace's fma chain and puts
// them in an LDS copy of the batch's outgoing blocks; the workgroup then writes
// every block to its receiving slot (the neighbour across the face) in
// 16-byte vectors, as k_trace does.
// ---------------------------------------------------------------------------
#ifndef FR_TLE1_D
#define FR_TLE1_D 16
#endif
#ifndef FR_TLE2_D
#define FR_TLE2_D 7
#endif
#ifndef FR_TLE3_D
#define FR_TLE3_D 4
#endif
#ifndef FR_TLE4_D
#define FR_TLE4_D 2
#endif
#ifndef FR_TLE5_D
#define FR_TLE5_D 1
#endif
#ifndef FR_TLE6_D
#define FR_TLE6_D 1
#endif
#ifndef FR_TLE1_F
#define FR_TLE1_F 32
#endif
#ifndef FR_TLE2_F
#define FR_TLE2_F 14
#endif
#ifndef FR_TLE3_F
#define FR_TLE3_F 8
#endif
#ifndef FR_TLE4_F
#define FR_TLE4_F 4
#endif
#ifndef FR_TLE5_F
#define FR_TLE5_F 2
#endif
#ifndef FR_TLE6_F
#define FR_TLE6_F 1
#endif
#ifndef FR_TLNT
#define FR_TLNT 256
#endif
#ifndef FR_TLU1_D
#define FR_TLU1_D 0
#endif
#ifndef FR_TLU2_D
#define FR_TLU2_D 0
#endif
#ifndef FR_TLU3_D
#define FR_TLU3_D 0
#endif
#ifndef FR_TLU4_D
#define FR_TLU4_D 0
#endif
#ifndef FR_TLU5_D
#define FR_TLU5_D 1
#endif
#ifndef FR_TLU6_D
#define FR_TLU6_D 0
#endif
#ifndef FR_TLU1_F
#define FR_TLU1_F 0
#endif
#ifndef FR_TLU2_F
#define FR_TLU2_F 0
#endif
#ifndef FR_TLU3_F
#define FR_TLU3_F 0
#endif
#ifndef FR_TLU4_F
#define FR_TLU4_F 0
#endif
#ifndef FR_TLU5_F
#define FR_TLU5_F 1
#endif
#ifndef FR_TLU6_F
#define FR_TLU6_F 1
#endif
// Whether stage 1 runs as k_trace_lines (1) or k_trace (0) for a diagonal
// Jacobian, per order and precision, from the measured times of both on the
// order-sweep lattices (both write the same bits).
template <int P, typename T> struct TraceLinesShape;
#define FR_TLSHAPE(PP, TT, S)                                                                  \
    template <> struct TraceLinesShape<PP, TT> {                                               \
        static constexpr int E = FR_TLE##PP##_##S, NT = FR_TLNT;                               \
        static constexpr bool USE = FR_TLU##PP##_##S;                                          \
        static constexpr int OUT = 6 * E * TraceLayout<PP + 1, TT>::CHP;                       \
        static constexpr int values = LinesLds<PP, TT>::OPS + E * LinesLds<PP, TT>::EP + OUT;  \
        static_assert(values * sizeof(TT) <= 160 * 1024, "LDS");                               \
    };
FR_TLSHAPE(1, double, D)
FR_TLSHAPE(2, double, D)
FR_TLSHAPE(3, double, D)
FR_TLSHAPE(4, double, D)
FR_TLSHAPE(5, double, D)
FR_TLSHAPE(6, double, D)
FR_TLSHAPE(1, float, F)
FR_TLSHAPE(2, float, F)
FR_TLSHAPE(3, float, F)
FR_TLSHAPE(4, float, F)
FR_TLSHAPE(5, float, F)
FR_TLSHAPE(6, float, F)
#undef FR_TLSHAPE

template <int P, typename T>
__global__ void __launch_bounds__(FR_TLNT)
    k_trace_lines(const T *__restrict__ U, T *__restrict__ TR, const T *__restrict__ ops, int nx,
                  int ny, int nz)
{
    constexpr int M = P + 1, NS = M * M * M, NF = M * M;
    constexpr int E = TraceLinesShape<P, T>::E, NT = TraceLinesShape<P, T>::NT;
    using LL = LinesLds<P, T>;
    using OL = OpsLayout<M>;
    using TL = TraceLayout<M, T>;
    using V = typename V16<T>::type;
    constexpr int EP = LL::EP, RAW = LL::raw, CH = TL::CH, CHP = TL::CHP, CHV = TL::CHV;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sop = reinterpret_cast<T *>(smem_raw);
    T *sU = sop + LL::OPS;       // [E][EP]
    T *sO = sU + E * EP;         // [6][E][CHP] outgoing blocks, by own face
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t e0 = (int64_t)blockIdx.x * E;
    const int nel = (int)min((int64_t)E, ne - e0);
    if (threadIdx.x < 2 * M) sop[OL::lm + threadIdx.x] = ops[OL::lm + threadIdx.x];
    // the padding of every outgoing block is written as zeros
    if constexpr (CHP > CH)
        for (int k = threadIdx.x; k < 6 * E * (CHP - CH); k += NT)
            sO[(k / (CHP - CH)) * CHP + CH + k % (CHP - CH)] = T(0);
    tile_load<P, T, NT>(U + e0 * RAW, sU, nel);
    __syncthreads();
    T lm[M], lp[M];
#pragma unroll
    for (int l = 0; l < M; ++l) {
        lm[l] = sop[OL::lm + l];
        lp[l] = sop[OL::lp + l];
    }
    for (int t = threadIdx.x; t < 3 * E * NF; t += NT) {
        const int d = t / (E * NF), r = t - d * (E * NF);
        const int el = r / NF, L = r - el * NF;
        if (el >= nel) continue;
        const int a = L % M, b = L / M;
        const int str = d == 0 ? 1 : (d == 1 ? M : M * M);
        const int base = d == 0 ? M * L : (d == 1 ? a + M * M * b : L);
        const T *Ue = sU + el * EP + base;
        T *om = sO + ((2 * d) * E + el) * CHP + L;
        T *op = om + E * CHP;
#pragma unroll
        for (int cc = 0; cc < NTR; ++cc) {
            const T *X = Ue + (cc < 4 ? cc : 4 + 3 * (cc - 4) + d) * NS;
            T am = T(0), ap = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) {
                const T x = X[l * str];
                am = fma(lm[l], x, am);
                ap = fma(lp[l], x, ap);
            }
            om[cc * NF] = am;
            op[cc * NF] = ap;
        }
    }
    __syncthreads();
    // block (f, el) goes to the receiving block (f ^ 1, neighbour across f)
    V *TRv = reinterpret_cast<V *>(TR);
    const V *sOv = reinterpret_cast<const V *>(sO);
    for (int t = threadIdx.x; t < 6 * E * CHV; t += NT) {
        const int fe = t / CHV, k = t - fe * CHV;
        const int f = fe / E, el = fe - f * E;
        if (el >= nel) continue;
        const int64_t nb = neighbour(e0 + el, f, nx, ny, nz);
        __builtin_nontemporal_store(sOv[t], TRv + ((int64_t)(f ^ 1) * ne + nb) * CHV + k);
    }
}

// ---------------------------------------------------------------------------
// launch
// ---------------------------------------------------------------------------
template <int P, typename T, bool DIAG, bool MF>
int fused_impl(fr_plan *pl, const T *U, T *R, const StageSpec *sp, int *nparts, T *TR,
               const T *ops, const Consts<T> &c, hipStream_t s, bool prof)
{
    constexpr int M = P + 1, NS = M * M * M;
    constexpr int CHP = TraceLayout<M, T>::CHP;
    constexpr int EMAX = Shape<P, T>::EMAX, NT = Shape<P, T>::NT;
    constexpr int TEMAX = TraceShape<P, T>::EMAX, TNT = TraceShape<P, T>::NT;
    const int ne = (int)pl->ne;
    int E = pl->block ? pl->block : EMAX;
    if (E > EMAX)
        return set_error(FR_EINVAL, "fused kernel: block %d exceeds %d elements at p=%d", E, EMAX, P);
    if (E > ne) E = ne;
    const int nbatch = (ne + E - 1) / E;
    const int TE = TEMAX < ne ? TEMAX : ne;
    const int nbatch_tr = (ne + TE - 1) / TE;
    const size_t lds_tr =
        ((size_t)TEMAX * NV * TracePad<M>::NSP + 2 * M) * sizeof(T) + 6 * TEMAX * sizeof(int);
    const size_t lds_fu =
        ((size_t)EMAX * (NV + 9) * NS + (size_t)6 * EMAX * CHP + OpsLayout<M>::size + 24) * sizeof(T);
    const void *ktr = (const void *)k_trace<P, T, DIAG>;
    constexpr bool STG_OK = StageEpilogue<P, T, DIAG>::value;
    // the halo form (line tasks that form the neighbours' traces from their
    // states: no trace kernel), for the residual and for the stage epilogue
    const bool halo = !MF && DIAG &&
                      (sp ? stage_path(pl) == FR_STAGE_HALO
                          : (pl->form == FR_FORM_HALO ||
                             (pl->form == FR_FORM_AUTO && LinesShape<P, T>::AUTO == 2)));
    if (sp && !STG_OK && !halo)
        return set_error(FR_EUNSUPPORTED, "stage epilogue not available at p=%d", P);
    if (sp && halo && (sp->tr_in || sp->tr_out))
        return set_error(FR_EINVAL, "halo-form stage epilogue: no face-trace arrays");
    const void *kfu = (const void *)k_fused<P, T, DIAG, false>;
    if constexpr (STG_OK)
        if (sp) kfu = (const void *)k_fused<P, T, DIAG, true>;
    if constexpr (MF) {
        if (sp) return set_error(FR_EUNSUPPORTED, "matrix-core variant: no stage epilogue");
        kfu = (const void *)k_fused<P, T, DIAG, false, true>;
    }
    // line-task forms (diagonal Jacobian); the plain line form's stage
    // epilogue is the point form's
    const bool lines = halo || (!MF && !sp && DIAG &&
                                (pl->form == FR_FORM_LINES ||
                                 (pl->form == FR_FORM_AUTO && LinesShape<P, T>::AUTO == 1)));
    if (!MF && !sp && !DIAG && (pl->form == FR_FORM_LINES || pl->form == FR_FORM_HALO))
        return set_error(FR_EUNSUPPORTED, "line-task forms: diagonal Jacobians only");
    // persistent grid: every workgroup that fits on the device at once
    auto persistent_grid = [&](const void *fn, int nt, size_t lds, int &grid) -> int {
        if (grid) return FR_OK;
        int dev = 0, ncu = 0, occ = 0;
        if (int rc = check_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
        if (int rc = check_hip(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev),
                               "hipDeviceGetAttribute"))
            return rc;
        if (int rc = check_hip(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)lds),
                               "hipFuncSetAttribute"))
            return rc;
        if (int rc = check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, nt, lds),
                               "hipOccupancyMaxActiveBlocksPerMultiprocessor"))
            return rc;
        if (occ < 1) return set_error(FR_EUNSUPPORTED, "fused kernels do not fit on a CU at p=%d", P);
        grid = ncu * occ;
        return FR_OK;
    };
    int &grid_tr = pl->fused_grid[0][P][sizeof(T) == 8][DIAG];
    int &grid_fu = pl->fused_grid[MF ? 3 : (sp ? 2 : 1)][P][sizeof(T) == 8][DIAG];
    if (int rc = persistent_grid(ktr, TNT, lds_tr, grid_tr)) return rc;
    if (!lines && !halo)
        if (int rc = persistent_grid(kfu, NT, lds_fu, grid_fu)) return rc;
    const unsigned gtr = (unsigned)min(nbatch_tr, grid_tr);
    const unsigned gfu = (unsigned)min(min(nbatch, grid_fu), sp ? MAX_PARTIALS : grid_fu);
    if (!halo && !TR && !(sp && sp->tr_in))
        return set_error(FR_EINVAL, "fused residual: no face-trace array");
    if (halo) {
        // no trace kernel: the line tasks form the neighbours' traces themselves
    } else if (sp && sp->tr_in) {
        TR = static_cast<T *>(const_cast<void *>(sp->tr_in));
    } else if (DIAG && TraceLinesShape<P, T>::USE) {
        using TLS = TraceLinesShape<P, T>;
        const size_t lds_tl = (size_t)TLS::values * sizeof(T);
        int &set = pl->lines_attr[1][P][sizeof(T) == 8];
        if (!set) {
            if (int rc = check_hip(hipFuncSetAttribute((const void *)k_trace_lines<P, T>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)lds_tl),
                                   "hipFuncSetAttribute"))
                return rc;
            set = 1;
        }
        ProfScope ps(prof ? pl : nullptr, FR_K_TRACE, s);
        hipLaunchKernelGGL((k_trace_lines<P, T>), dim3((unsigned)((ne + TLS::E - 1) / TLS::E)),
                           dim3(TLS::NT), lds_tl, s, U, TR, ops, pl->nx, pl->ny, pl->nz);
    } else {
        ProfScope ps(prof ? pl : nullptr, FR_K_TRACE, s);
        hipLaunchKernelGGL((k_trace<P, T, DIAG>), dim3(gtr), dim3(TNT), lds_tr, s, U, TR, ops, c,
                           pl->nx, pl->ny, pl->nz, TE, nbatch_tr);
    }
    if (lines) {
        constexpr int LE = LinesShape<P, T>::E, LNT = LinesShape<P, T>::NT;
        const size_t lds_li = (size_t)LinesLds<P, T>::values(LE, LinesShape<P, T>::XR) * sizeof(T);
        const int64_t nb = ((int64_t)ne + LE - 1) / LE;
        int &set = pl->lines_attr[0][P][sizeof(T) == 8];
        if (!set) {
            for (const void *fn : {(const void *)k_lines<P, T, false, false>,
                                   (const void *)k_lines<P, T, true, false>,
                                   (const void *)k_lines<P, T, true, true>})
                if (int rc = check_hip(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                           (int)lds_li),
                                       "hipFuncSetAttribute"))
                    return rc;
            set = 1;
        }
        ProfScope ps(prof ? pl : nullptr, FR_K_FUSED, s);
        if constexpr (DIAG) {
            if (sp) {
                // one partial norm sum per workgroup (the caller sizes the
                // partial sums by stage_partials)
                const unsigned g =
                    (unsigned)(StageLoop<P, T>::value ? std::min<int64_t>(nb, MAX_PARTIALS) : nb);
                if (nparts) *nparts = (int)g;
                hipLaunchKernelGGL((k_lines<P, T, true, true>), dim3(g), dim3(LNT), lds_li, s, U,
                                   (const T *)nullptr, (T *)nullptr, ops, c, pl->nx, pl->ny, pl->nz,
                                   *sp);
            } else if (halo) {
                hipLaunchKernelGGL((k_lines<P, T, true, false>), dim3((unsigned)nb), dim3(LNT), lds_li,
                                   s, U, TR, R, ops, c, pl->nx, pl->ny, pl->nz, StageSpec{});
            } else {
                hipLaunchKernelGGL((k_lines<P, T, false, false>), dim3((unsigned)nb), dim3(LNT), lds_li,
                                   s, U, TR, R, ops, c, pl->nx, pl->ny, pl->nz, StageSpec{});
            }
        }
        return check_hip(hipGetLastError(), "fused residual launch");
    }
    {
        ProfScope ps(prof ? pl : nullptr, FR_K_FUSED, s);
        if (sp) {
            if constexpr (STG_OK) {
                if (nparts) *nparts = (int)gfu;
                hipLaunchKernelGGL((k_fused<P, T, DIAG, true>), dim3(gfu), dim3(NT), lds_fu, s, U,
                                   TR, (T *)nullptr, ops, c, ne, E, nbatch, *sp);
            }
        } else if constexpr (MF) {
            hipLaunchKernelGGL((k_fused<P, T, DIAG, false, true>), dim3(gfu), dim3(NT), lds_fu, s, U,
                               TR, R, ops, c, ne, E, nbatch, StageSpec{});
        } else {
            hipLaunchKernelGGL((k_fused<P, T, DIAG, false>), dim3(gfu), dim3(NT), lds_fu, s, U, TR,
                               R, ops, c, ne, E, nbatch, StageSpec{});
        }
    }
    return check_hip(hipGetLastError(), "fused residual launch");
}

template <typename T, bool MF = false>
int dispatch_fused(fr_plan *pl, const T *U, T *R, const StageSpec *sp, int *nparts, T *TR,
                   const T *ops, const Consts<T> &c, hipStream_t s, bool prof)
{
    const bool dg = c.diag != 0;
#define FR_CASE(PP)                                                                        \
    case PP:                                                                               \
        return dg ? fused_impl<PP, T, true, MF>(pl, U, R, sp, nparts, TR, ops, c, s, prof) \
                  : fused_impl<PP, T, false, MF>(pl, U, R, sp, nparts, TR, ops, c, s, prof);
    switch (pl->p) {
        FR_CASE(1)
        FR_CASE(2)
        FR_CASE(3)
        FR_CASE(4)
        FR_CASE(5)
        FR_CASE(6)
    }
#undef FR_CASE
    return set_error(FR_EINVAL, "order %d", pl->p);
}

// Bytes of the face-trace array of the fused path.
size_t trace_bytes(const fr_plan *pl)
{
    const int m = pl->m;
    const size_t esz = pl->precision == FR_F64 ? 8 : 4;
    const size_t w = 16 / esz;
    const size_t chp = (NTR * m * m + w - 1) / w * w;
    return (size_t)6 * pl->ne * chp * esz;
}

// The fused residual (or stage) with its face traces in TR: the plan's own
// scratch (allocated on first use) when TR is null.  prof = false skips the
// per-kernel event timing.
int fused_any(fr_plan *pl, const void *U, void *R, const StageSpec *sp, int *nparts,
              hipStream_t s, void *TR = nullptr, bool prof = true, bool mf = false)
{
    // the halo form needs no trace array (for a stage, the stage path decides
    // the form: the point form's epilogue may follow a halo-form residual)
    const bool halo = !mf && (sp ? stage_path(pl) == FR_STAGE_HALO : residual_form(pl) == FR_FORM_HALO);
    if (!TR && !halo) {
        if (int rc = ensure_scratch(pl->traces, trace_bytes(pl))) return rc;
        TR = pl->traces.ptr;
    }
    if (mf) {
        if (pl->precision != FR_F32)
            return set_error(FR_EUNSUPPORTED,
                             "the matrix-core variant computes in single precision (FR_F32)");
        return dispatch_fused<float, true>(pl, (const float *)U, (float *)R, sp, nparts, (float *)TR,
                                           (const float *)pl->ops32, pl->c32, s, prof);
    }
    if (pl->precision == FR_F64)
        return dispatch_fused<double>(pl, (const double *)U, (double *)R, sp, nparts,
                                      (double *)TR, (const double *)pl->ops64, pl->c64, s, prof);
    return dispatch_fused<float>(pl, (const float *)U, (float *)R, sp, nparts, (float *)TR,
                                 (const float *)pl->ops32, pl->c32, s, prof);
}


}  // namespace

int launch_residual_fused(fr_plan *pl, const void *U, void *R, hipStream_t s)
{
    return fused_any(pl, U, R, nullptr, nullptr, s);
}

int launch_residual_mfma(fr_plan *pl, const void *U, void *R, hipStream_t s)
{
    return fused_any(pl, U, R, nullptr, nullptr, s, nullptr, true, true);
}

// ---------------------------------------------------------------------------
// Allocation-free residual: the face traces go to a fixed device array of
// SCRATCH_BYTES instead of the plan's scratch.  Every device holds its own
// copy of the array; host code never uses the array's name (a host-side
// stand-in), only the device address looked up once per device.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
constexpr int SCRATCH_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static std::mutex scratch_mu;
static void *scratch_ptr[SCRATCH_MAX_DEVICES] = {};

int scratch_setup(int dev)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return set_error(FR_EUNSUPPORTED, "device %d: at most %d devices", dev, SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptr[dev]) return FR_OK;
    void *ptr = nullptr;
    if (int rc = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))
        return rc;
    scratch_ptr[dev] = ptr;
    return FR_OK;
}

int launch_residual_noalloc(fr_plan *pl, const void *U, void *R, hipStream_t s)
{
    if (pl->variant != FR_FUSED && pl->variant != FR_MFMA)
        return set_error(FR_EUNSUPPORTED, "fr_residual_noalloc: fused or matrix-core variant only");
    // the halo form forms the neighbours' traces itself and uses no array
    const size_t need = residual_form(pl) == FR_FORM_HALO ? 0 : trace_bytes(pl);
    if (need > SCRATCH_BYTES)
        return set_error(FR_EINVAL,
                         "fr_residual_noalloc: the face traces need %zu bytes, the fixed array holds "
                         "%zu (at most about %zu elements at this order and precision)",
                         need, SCRATCH_BYTES, (size_t)(SCRATCH_BYTES / (need / pl->ne)));
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mu);
        if (pl->device >= 0 && pl->device < SCRATCH_MAX_DEVICES) ptr = scratch_ptr[pl->device];
    }
    if (!ptr) return set_error(FR_EHIP, "fr_residual_noalloc: no trace array on device %d", pl->device);
    return fused_any(pl, U, R, nullptr, nullptr, s, ptr, false, pl->variant == FR_MFMA);
}


int residual_form(const fr_plan *pl)
{
    if (pl->variant != FR_FUSED) return 0;
    if (pl->c64.diag == 0 || pl->form == FR_FORM_POINT) return FR_FORM_POINT;
    if (pl->form == FR_FORM_LINES || pl->form == FR_FORM_HALO) return pl->form;
    const bool f64 = pl->precision == FR_F64;
    auto pick = [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        const int a = f64 ? LinesShape<P, double>::AUTO : LinesShape<P, float>::AUTO;
        return a == 2 ? FR_FORM_HALO : (a == 1 ? FR_FORM_LINES : FR_FORM_POINT);
    };
    switch (pl->p) {
        case 1: return pick(Dir<1>{});
        case 2: return pick(Dir<2>{});
        case 3: return pick(Dir<3>{});
        case 4: return pick(Dir<4>{});
        case 5: return pick(Dir<5>{});
        case 6: return pick(Dir<6>{});
    }
    return FR_FORM_POINT;
}

// Whether the point form's kernel has a stage epilogue for this plan.
static bool point_stage_available(const fr_plan *pl)
{
    const bool dg = pl->c64.diag != 0, f64 = pl->precision == FR_F64;
    auto pick = [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        return f64 ? (dg ? StageEpilogue<P, double, true>::value : StageEpilogue<P, double, false>::value)
                   : (dg ? StageEpilogue<P, float, true>::value : StageEpilogue<P, float, false>::value);
    };
    switch (pl->p) {
        case 1: return pick(Dir<1>{});
        case 2: return pick(Dir<2>{});
        case 3: return pick(Dir<3>{});
        case 4: return pick(Dir<4>{});
        case 5: return pick(Dir<5>{});
        case 6: return pick(Dir<6>{});
    }
    return false;
}

int stage_path(const fr_plan *pl)
{
    if (pl->variant != FR_FUSED || !pl->fuse_stage) return FR_STAGE_SEPARATE;
    const int point = point_stage_available(pl) ? FR_STAGE_POINT : FR_STAGE_SEPARATE;
    if (residual_form(pl) != FR_FORM_HALO) return point;
    if (pl->form == FR_FORM_HALO) return FR_STAGE_HALO;
    const bool f64 = pl->precision == FR_F64;
    auto pick = [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        return f64 ? StageAuto<P, double>::value : StageAuto<P, float>::value;
    };
    int a = FR_STAGE_HALO;
    switch (pl->p) {
        case 1: a = pick(Dir<1>{}); break;
        case 2: a = pick(Dir<2>{}); break;
        case 3: a = pick(Dir<3>{}); break;
        case 4: a = pick(Dir<4>{}); break;
        case 5: a = pick(Dir<5>{}); break;
        case 6: a = pick(Dir<6>{}); break;
    }
    return a == FR_STAGE_POINT ? point : a;
}

int stage_partials(const fr_plan *pl)
{
    if (stage_path(pl) != FR_STAGE_HALO) return 0;
    const bool f64 = pl->precision == FR_F64;
    auto pick = [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        const int E = f64 ? LinesShape<P, double>::E : LinesShape<P, float>::E;
        const bool loop = f64 ? StageLoop<P, double>::value : StageLoop<P, float>::value;
        const int64_t nb = (pl->ne + E - 1) / E;
        return (int)(loop ? std::min<int64_t>(nb, MAX_PARTIALS) : nb);
    };
    switch (pl->p) {
        case 1: return pick(Dir<1>{});
        case 2: return pick(Dir<2>{});
        case 3: return pick(Dir<3>{});
        case 4: return pick(Dir<4>{});
        case 5: return pick(Dir<5>{});
        case 6: return pick(Dir<6>{});
    }
    return 0;
}

int launch_residual_stage(fr_plan *pl, const void *U, const StageSpec &sp, int *nparts,
                          hipStream_t s)
{
    return fused_any(pl, U, nullptr, &sp, nparts, s);
}

int stage_trace_buffers(fr_plan *pl, void *&a, void *&b)
{
    if (int rc = ensure_scratch(pl->traces, trace_bytes(pl))) return rc;
    if (int rc = ensure_scratch(pl->traces2, trace_bytes(pl))) return rc;
    a = pl->traces.ptr;
    b = pl->traces2.ptr;
    return FR_OK;
}

// Launch shape of the fused path's kernels (host only): elements per batch,
// threads per workgroup and dynamic LDS bytes, as fused_impl launches them.
template <int P, typename T>
void shape_of(int kernel, int out[3])
{
    constexpr int M = P + 1, NS = M * M * M;
    if (kernel == FR_K_TRACE) {
        constexpr int E = TraceShape<P, T>::EMAX;
        out[0] = E;
        out[1] = TraceShape<P, T>::NT;
        out[2] = (int)(((size_t)E * NV * TracePad<M>::NSP + 2 * M) * sizeof(T) + 6 * E * sizeof(int));
    } else {
        constexpr int E = Shape<P, T>::EMAX;
        out[0] = E;
        out[1] = Shape<P, T>::NT;
        out[2] = (int)(((size_t)E * (NV + 9) * NS + (size_t)6 * E * TraceLayout<M, T>::CHP +
                        OpsLayout<M>::size + 24) * sizeof(T));
    }
}

}  // namespace fr

extern "C" int fr_launch_shape(int p, int precision, int kernel, int out[3])
{
    using namespace fr;
    if (p < 1 || p > PMAX || !out || (precision != FR_F64 && precision != FR_F32) ||
        (kernel != FR_K_TRACE && kernel != FR_K_FUSED))
        return set_error(FR_EINVAL, "fr_launch_shape: p=%d precision=%d kernel=%d", p, precision,
                         kernel);
    const bool f64 = precision == FR_F64;
    switch (p) {
#define FR_SHAPE_CASE(PP)                                                  \
    case PP:                                                               \
        f64 ? shape_of<PP, double>(kernel, out) : shape_of<PP, float>(kernel, out); \
        break;
        FR_SHAPE_CASE(1)
        FR_SHAPE_CASE(2)
        FR_SHAPE_CASE(3)
        FR_SHAPE_CASE(4)
        FR_SHAPE_CASE(5)
        FR_SHAPE_CASE(6)
#undef FR_SHAPE_CASE
    }
    return FR_OK;
}

namespace fr {

}  // namespace fr
