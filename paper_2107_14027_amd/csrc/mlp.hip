// Pointwise multilayer perceptron that predicts the initial guess of a
// physical time step (P, u, v, w at n+1 from the three previous states), on
// gfx950 BF16 matrix cores with FP32 accumulation.  Not part of the paper: the
// pseudo-time iteration still decides the answer; only its starting point
// changes.  The plain quadratic extrapolation is the network's zero: the
// network predicts a correction to it.
//
// Network, per point:  x (12) -> h1 = tanh(W1 x + b1) (64) -> h2 = tanh(W2 h1 + b2) (64)
//                      -> y = W3 h2 + b3 (4)
// Features (normalised in FP32, x = ((float) raw - mu) * inv_sd):
//   raw = [U^n_c,  U^n_c - U^{n-1}_c,  U^n_c - 2 U^{n-1}_c + U^{n-2}_c]  for c = P, u, v, w
// Guess:  G_c = E_c + y_sd_c * y_c        (c = P, u, v, w)
//         G_v = E_v                         (auxiliary v)
// with E the quadratic (3 U^n - 3 U^{n-1} + U^{n-2}) or linear (2 U^n - U^{n-1})
// extrapolation, written exactly as the plain extrapolation kernel writes it.
//
// Matrix-core mapping (v_mfma_f32_16x16x16_bf16, one wave = 16 points): the
// weights are the A operand and the activations, transposed (units x points),
// the B operand.  Then the FP32 output registers of one layer, after bias and
// tanh, are exactly the B operand of the next layer's K-block:
//   A[i][k] in lane l: i = l%16, k = 4(l/16)+j ;  B[k][n]: n = l%16, k = 4(l/16)+j ;
//   D[i][n]: n = l%16, i = 4(l/16)+t.
// Training transposes activations through LDS for the weight gradients.
#include <cmath>
#include <new>

#include "fr_internal.h"

namespace fr {
namespace mlp {

constexpr int NI = 12, NH = 64, NO = 4;
constexpr int OW1 = 0, OB1 = 768, OW2 = 832, OB2 = 4928, OW3 = 4992, OB3 = 5248, NPAR = 5252;
constexpr int ONORM = NPAR;                  // mu[12], inv_sd[12], y_sd[4]
constexpr int OADAM_M = NPAR + 28, OADAM_V = OADAM_M + NPAR, NSTATE = OADAM_V + NPAR;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (the hardware conversion, two values
// per instruction on gfx950).
__device__ __forceinline__ short bf16_rne(float x)
{
    return __builtin_bit_cast(short, (__bf16)x);
}

__device__ __forceinline__ v4s pack4(float a, float b, float c, float d)
{
    v4s r;
    r[0] = bf16_rne(a);
    r[1] = bf16_rne(b);
    r[2] = bf16_rne(c);
    r[3] = bf16_rne(d);
    return r;
}

// Orders one wave's LDS writes before its later LDS reads of other lanes' data.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Hyperbolic tangent from the exponential identity tanh x = 1 - 2 / (1 + e^{2x}),
// e^{2x} = 2^{2 log2(e) x}, on the hardware exp2 and reciprocal: four
// instructions, no branch.  It saturates by itself (e^{2x} = inf gives 1, 0
// gives -1).  The absolute error is a few units in the last place of 1 (below
// 5e-7), against the BF16 rounding (2^-9 relative) the activations get next;
// near x = 0 that is an absolute, not a relative, error, which is what the next
// layer's sum sees.
__device__ __forceinline__ float tanh_exp(float x)
{
    const float t = __builtin_amdgcn_exp2f(2.88539008177792681f * x);
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + t), 1.0f);
}

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weights of one wave, packed as MFMA A operands (bf16).
struct Weights {
    v4s w1[4];      // block r: W1[16r + l%16][4(l/16)+j]   (inputs >= 12 are zero)
    v4s w2[4][4];   // [r2][r]: W2[16r2 + l%16][16r + 4(l/16)+j]
    v4s w3[4];      // [r]: W3[l%16][16r + 4(l/16)+j]       (outputs >= 4 are zero)
    float b1[4][4], b2[4][4], b3[4];  // bias of D rows 16r + 4(l/16) + t
};

// A operand k of lane l (k = r: W1 block r; k = 4 + 4 r2 + r: W2 block [r2][r];
// k = 20 + r: W3 block r), packed to bf16.
constexpr int NBLK = 24;

__device__ __forceinline__ v4s weight_block(const float *__restrict__ P, int k, int lane)
{
    const int i = lane & 15, g = lane >> 4;
    float v[4];
    if (k < 4) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int f = 4 * g + j;
            v[j] = f < NI ? P[OW1 + (16 * k + i) * NI + f] : 0.0f;
        }
    } else if (k < 20) {
        const int r2 = (k - 4) >> 2, r = (k - 4) & 3;
        const float *row = P + OW2 + (16 * r2 + i) * NH + 16 * r + 4 * g;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = row[j];
    } else {
        const int r = k - 20;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = i < NO ? P[OW3 + i * NH + 16 * r + 4 * g + j] : 0.0f;
    }
    return pack4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ void load_weights(const float *__restrict__ P, Weights &w, int lane)
{
    const int g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        w.w1[r] = weight_block(P, r, lane);
#pragma unroll
        for (int r2 = 0; r2 < 4; ++r2) w.w2[r2][r] = weight_block(P, 4 + 4 * r2 + r, lane);
        w.w3[r] = weight_block(P, 20 + r, lane);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            w.b1[r][t] = P[OB1 + 16 * r + 4 * g + t];
            w.b2[r][t] = P[OB2 + 16 * r + 4 * g + t];
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) w.b3[t] = (g == 0) ? P[OB3 + t] : 0.0f;
}

// Forward pass of one 16-point tile.  xb: this lane's B operand of the input
// (features 4(l/16)..+3 of point l%16).  Returns the output D (rows 4(l/16)+t:
// lanes 0..15 hold the 4 outputs of point l%16) and, if wanted, the FP32
// activations h1, h2 in D layout.
struct Acts {
    v4f h1[4], h2[4];
};

__device__ __forceinline__ v4f forward(const Weights &w, v4s xb, Acts &a)
{
    v4s hb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        // the FP32 bias seeds the accumulator
        v4f z = {w.b1[r][0], w.b1[r][1], w.b1[r][2], w.b1[r][3]};
        z = mfma(w.w1[r], xb, z);
#pragma unroll
        for (int t = 0; t < 4; ++t) a.h1[r][t] = tanh_exp(z[t]);
        hb[r] = pack4(a.h1[r][0], a.h1[r][1], a.h1[r][2], a.h1[r][3]);
    }
    v4s h2b[4];
#pragma unroll
    for (int r2 = 0; r2 < 4; ++r2) {
        v4f z = {w.b2[r2][0], w.b2[r2][1], w.b2[r2][2], w.b2[r2][3]};
#pragma unroll
        for (int r = 0; r < 4; ++r) z = mfma(w.w2[r2][r], hb[r], z);
#pragma unroll
        for (int t = 0; t < 4; ++t) a.h2[r2][t] = tanh_exp(z[t]);
        h2b[r2] = pack4(a.h2[r2][0], a.h2[r2][1], a.h2[r2][2], a.h2[r2][3]);
    }
    v4f y = {w.b3[0], w.b3[1], w.b3[2], w.b3[3]};
#pragma unroll
    for (int r = 0; r < 4; ++r) y = mfma(w.w3[r], h2b[r], y);
    return y;
}

// ---------------------------------------------------------------------------
// Raw features and extrapolation at one point
// ---------------------------------------------------------------------------
__device__ __forceinline__ void raw_features(const double *Un, const double *Unm1,
                                             const double *Unm2, int64_t base, int ns, double f[12])
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t i = base + (int64_t)c * ns;
        const double a = Un[i], b = Unm1[i], d = Unm2[i];
        f[c] = a;
        f[4 + c] = a - b;
        f[8 + c] = (a - b) - (b - d);
    }
}

// Polynomial extrapolation, the same expressions as the plain extrapolation kernel.
__device__ __forceinline__ double extrap(double a, double b, double d, int order)
{
    return order == 1 ? 2.0 * a - b : 3.0 * (a - b) + d;
}

// Guess kernel.  One lane per point, so every global load and store of a wave
// covers 64 consecutive points (512 contiguous bytes of one variable); waves
// loop over 64-point groups of the flat point index (e, q).  The weights sit in
// LDS in A-operand order (read once per block), which keeps the registers to
// the streaming state; each lane's normalised features go through LDS into the
// B-operand layout of the four 16-point tiles, and the network outputs back to
// the lane of their point.  Same operands and products as forward(), hence the
// same bits.
constexpr int GUESS_WAVES = 4;

struct GuessLds {
    v4s a[NBLK][64];            // weight_block(k, lane)
    float b1[NH], b2[NH], b3[4];
    v4s xs[GUESS_WAVES][4][64]; // per wave: features 4g..4g+3 of point pt at [g][pt]
    v4f ys[GUESS_WAVES][64];    // per wave: network outputs of point pt
};

__device__ __forceinline__ v4f forward_lds(const GuessLds &L, int lane, v4s xb)
{
    const int g4 = 4 * (lane >> 4);
    v4s hb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        v4f z = *(const v4f *)&L.b1[16 * r + g4];
        z = mfma(L.a[r][lane], xb, z);
        hb[r] = pack4(tanh_exp(z[0]), tanh_exp(z[1]), tanh_exp(z[2]), tanh_exp(z[3]));
    }
    v4s h2b[4];
#pragma unroll
    for (int r2 = 0; r2 < 4; ++r2) {
        v4f z = *(const v4f *)&L.b2[16 * r2 + g4];
#pragma unroll
        for (int r = 0; r < 4; ++r) z = mfma(L.a[4 + 4 * r2 + r][lane], hb[r], z);
        h2b[r2] = pack4(tanh_exp(z[0]), tanh_exp(z[1]), tanh_exp(z[2]), tanh_exp(z[3]));
    }
    v4f y = g4 == 0 ? *(const v4f *)&L.b3[0] : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 4; ++r) y = mfma(L.a[20 + r][lane], h2b[r], y);
    return y;
}

__global__ void __launch_bounds__(64 * GUESS_WAVES) k_mlp_guess(const float *__restrict__ S,
                                                                const double *__restrict__ Un,
                                                                const double *__restrict__ Unm1,
                                                                const double *__restrict__ Unm2,
                                                                double *__restrict__ G,
                                                                int64_t npts, int ns, int order)
{
    __shared__ __align__(16) GuessLds L;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, pi = lane & 15;
    for (int i = threadIdx.x; i < NBLK * 64; i += 64 * GUESS_WAVES)
        L.a[i >> 6][i & 63] = weight_block(S, i >> 6, i & 63);
    if (threadIdx.x < NH) {
        L.b1[threadIdx.x] = S[OB1 + threadIdx.x];
        L.b2[threadIdx.x] = S[OB2 + threadIdx.x];
    }
    if (threadIdx.x < 4) L.b3[threadIdx.x] = S[OB3 + threadIdx.x];
    L.xs[wv][3][lane] = pack4(0.f, 0.f, 0.f, 0.f);   // features 12..15: zero
    __syncthreads();
    const int64_t ngrp = (npts + 63) / 64;
    const int64_t step = (int64_t)gridDim.x * GUESS_WAVES * 64;   // points per sweep of the grid
    const int64_t de = step / ns;
    const int dq = (int)(step - de * ns);
    int64_t pt = ((int64_t)blockIdx.x * GUESS_WAVES + wv) * 64 + lane;
    int64_t e = pt / ns;         // (e, q) of pt, advanced by step below
    int q = (int)(pt - e * ns);
    for (int64_t grp = pt >> 6; grp < ngrp; grp += step >> 6) {
        const bool ok = pt < npts;
        // lanes past the end read point 0 and write nothing
        const int64_t base = ok ? e * NV * ns + q : 0;
        // P, u, v, w: features (kind k: U^n, first, second difference) and extrapolation
        float x[3][4];
        double ex[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t i = base + (int64_t)c * ns;
            const double a = Un[i], b = Unm1[i], d = Unm2[i];
            const double raw[3] = {a, a - b, (a - b) - (b - d)};
            // normalised in FP32 from the raw feature rounded to FP32, as the
            // training samples are (fr_mlp_sample, then k_mlp_forward / k_mlp_grad)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                x[k][c] = ok ? ((float)raw[k] - S[ONORM + 4 * k + c]) * S[ONORM + NI + 4 * k + c] : 0.0f;
            ex[c] = extrap(a, b, d, order);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) L.xs[wv][k][lane] = pack4(x[k][0], x[k][1], x[k][2], x[k][3]);
        wave_sync();
        // the four 16-point tiles through the network; the nine auxiliary
        // variables (the extrapolation alone) stream between them, their loads
        // issued ahead of each tile's products
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int v0 = t == 0 ? 4 : 5 + 2 * t, v1 = 7 + 2 * t;   // 4-6, 7-8, 9-10, 11-12
            double av[3], bv[3], dv[3];
#pragma unroll
            for (int v = v0; v < v1; ++v) {
                const int64_t i = base + (int64_t)v * ns;
                av[v - v0] = Un[i];
                bv[v - v0] = Unm1[i];
                dv[v - v0] = Unm2[i];
            }
            const v4f y = forward_lds(L, lane, L.xs[wv][g][16 * t + pi]);
            if (g == 0) L.ys[wv][16 * t + pi] = y;
            if (ok) {
#pragma unroll
                for (int v = v0; v < v1; ++v)
                    G[base + (int64_t)v * ns] = extrap(av[v - v0], bv[v - v0], dv[v - v0], order);
            }
        }
        wave_sync();
        if (ok) {
            const v4f y = L.ys[wv][lane];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                G[base + (int64_t)c * ns] = ex[c] + (double)(S[ONORM + 2 * NI + c] * y[c]);
        }
        pt += step;
        e += de;
        q += dq;
        if (q >= ns) {
            q -= ns;
            ++e;
        }
    }
}

// Training samples: raw features and raw targets (U^{n+1} - extrapolation E) of
// every point p = offset + s * stride, s < n.
__global__ void __launch_bounds__(256) k_mlp_sample(const double *__restrict__ Un,
                                                    const double *__restrict__ Unm1,
                                                    const double *__restrict__ Unm2,
                                                    const double *__restrict__ Unp1, int64_t offset,
                                                    int64_t stride, int64_t n, int ns, int order,
                                                    float *__restrict__ X, float *__restrict__ Y)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pt = offset + s * stride;
        const int64_t e = pt / ns;
        const int q = (int)(pt - e * ns);
        const int64_t base = e * NV * ns + q;
        double f[12];
        raw_features(Un, Unm1, Unm2, base, ns, f);
#pragma unroll
        for (int k = 0; k < 12; ++k) X[s * NI + k] = (float)f[k];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t i = base + (int64_t)c * ns;
            Y[s * NO + c] = Unp1 ? (float)(Unp1[i] - extrap(Un[i], Unm1[i], Unm2[i], order)) : 0.0f;
        }
    }
}

// Column moments (sum, sum of squares) of X [n][12] and Y [n][4] in double,
// per block into part[block][32]; fixed-order two-level reduction.
__global__ void __launch_bounds__(256) k_mlp_moments(const float *__restrict__ X,
                                                     const float *__restrict__ Y, int64_t n,
                                                     double *__restrict__ part)
{
    __shared__ double sh[256][17];
    const int tid = threadIdx.x;
    double acc[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[k] = 0.0;
    for (int64_t s = (int64_t)blockIdx.x * 256 + tid; s < n; s += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double v = X[s * NI + k];
            acc[k] += v;
            acc[16 + k] += v * v;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double v = Y[s * NO + k];
            acc[12 + k] += v;
            acc[28 + k] += v * v;
        }
    }
    for (int half = 0; half < 2; ++half) {
#pragma unroll
        for (int k = 0; k < 16; ++k) sh[tid][k] = acc[16 * half + k];
        __syncthreads();
        if (tid < 16) {
            double s = 0.0;
            for (int t = 0; t < 256; ++t) s += sh[t][tid];
            part[(int64_t)blockIdx.x * 32 + 16 * half + tid] = s;
        }
        __syncthreads();
    }
}

__global__ void k_mlp_norm(const double *__restrict__ part, int nb, int64_t n, float *__restrict__ S)
{
    const int k = threadIdx.x;  // 16 threads: 12 features, 4 targets
    if (k >= 16) return;
    double s = 0.0, s2 = 0.0;
    for (int b = 0; b < nb; ++b) {
        s += part[(int64_t)b * 32 + k];
        s2 += part[(int64_t)b * 32 + 16 + k];
    }
    const double mean = s / (double)n;
    double var = s2 / (double)n - mean * mean;
    if (!(var > 0.0)) var = 0.0;
    const double sd = sqrt(var);
    if (k < NI) {
        S[ONORM + k] = (float)mean;
        S[ONORM + NI + k] = (float)(sd > 0.0 ? 1.0 / sd : 1.0);
    } else {
        S[ONORM + 2 * NI + (k - NI)] = (float)(sd > 0.0 ? sd : 1.0);
    }
}

// ---------------------------------------------------------------------------
// Training: forward, MSE, backward for a batch; per-wave FP32 gradient
// partials grad[wave][NPAR] (weights in the layout of the master parameters).
// ---------------------------------------------------------------------------
constexpr int TW = 4;  // waves per block

__global__ void __launch_bounds__(64 * TW) k_mlp_grad(const float *__restrict__ S,
                                                       const float *__restrict__ X,
                                                       const float *__restrict__ Y, int64_t n,
                                                       float *__restrict__ part,
                                                       double *__restrict__ loss_part)
{
    // per wave LDS: transposes of the 16-point tile, float [64][17] each
    __shared__ float sT[TW][3][64][17];
    __shared__ float sX[TW][16][17];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, pi = lane & 15;
    Weights w;
    load_weights(S, w, lane);
    // transposed copies as A operands for the backward products:
    //   w2t[r1][r2] : W2^T[16r1 + l%16][16r2 + 4(l/16)+j] = W2[16r2 + 4g + j][16r1 + i]
    //   w3t[r]      : W3^T[16r + l%16][4g + j]            = W3[4g + j][16r + i]  (g = 0 only)
    v4s w2t[4][4], w3t[4];
#pragma unroll
    for (int r1 = 0; r1 < 4; ++r1) {
#pragma unroll
        for (int r2 = 0; r2 < 4; ++r2) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = S[OW2 + (16 * r2 + 4 * g + j) * NH + 16 * r1 + pi];
            w2t[r1][r2] = pack4(v[0], v[1], v[2], v[3]);
        }
        float v3[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v3[j] = (g == 0) ? S[OW3 + j * NH + 16 * r1 + pi] : 0.f;
        w3t[r1] = pack4(v3[0], v3[1], v3[2], v3[3]);
    }
    float mu[4], isd[4], ysd_inv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * g + j;
        mu[j] = k < NI ? S[ONORM + k] : 0.f;
        isd[j] = k < NI ? S[ONORM + NI + k] : 0.f;
        ysd_inv[j] = 1.0f / S[ONORM + 2 * NI + j];
    }
    // gradient accumulators in D layout
    v4f gw1[4], gw2[4][4], gw3[4];
    float gb1[4][4], gb2[4][4], gb3[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        gw1[r] = v4f{0.f, 0.f, 0.f, 0.f};
        gw3[r] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r2 = 0; r2 < 4; ++r2) gw2[r][r2] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 4; ++t) gb1[r][t] = gb2[r][t] = 0.f;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) gb3[t] = 0.f;
    double lsum = 0.0;
    const float scale = 2.0f / (4.0f * (float)n);   // d/dy of mean over n points x 4 outputs

    const int64_t ntile = (n + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * TW + wv;
    const int64_t nwaves = (int64_t)gridDim.x * TW;
    float(*T1)[17] = sT[wv][0];
    float(*T2)[17] = sT[wv][1];
    float(*TD)[17] = sT[wv][2];
    float(*XS)[17] = sX[wv];
    for (int64_t tile = wave; tile < ntile; tile += nwaves) {
        const int64_t s = tile * 16 + pi;
        const bool ok = s < n;
        float xv[4] = {0.f, 0.f, 0.f, 0.f};
        if (ok && g < 3) {
#pragma unroll
            for (int j = 0; j < 4; ++j) xv[j] = (X[s * NI + 4 * g + j] - mu[j]) * isd[j];
        }
        const v4s xb = pack4(xv[0], xv[1], xv[2], xv[3]);
        Acts a;
        const v4f y = forward(w, xb, a);
        // dL/dy (rows 0..3 live in lanes 0..15); padded rows and points are zero
        float dy[4] = {0.f, 0.f, 0.f, 0.f};
        if (ok && g == 0) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float r = y[t] - Y[s * NO + t] * ysd_inv[t];
                lsum += (double)r * (double)r;
                dy[t] = scale * r;
                gb3[t] += dy[t];
            }
        }
        const v4s dyb = pack4(dy[0], dy[1], dy[2], dy[3]);
        // dZ2^T = (W3^T dY^T) * (1 - h2^2)
        v4f dz2[4];
        v4s dz2b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            v4f z = {0.f, 0.f, 0.f, 0.f};
            z = mfma(w3t[r], dyb, z);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                dz2[r][t] = ok ? z[t] * (1.0f - a.h2[r][t] * a.h2[r][t]) : 0.f;
                gb2[r][t] += dz2[r][t];
            }
            dz2b[r] = pack4(dz2[r][0], dz2[r][1], dz2[r][2], dz2[r][3]);
        }
        // dZ1^T = (W2^T dZ2^T) * (1 - h1^2)
        v4f dz1[4];
#pragma unroll
        for (int r1 = 0; r1 < 4; ++r1) {
            v4f z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r2 = 0; r2 < 4; ++r2) z = mfma(w2t[r1][r2], dz2b[r2], z);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                dz1[r1][t] = ok ? z[t] * (1.0f - a.h1[r1][t] * a.h1[r1][t]) : 0.f;
                gb1[r1][t] += dz1[r1][t];
            }
        }
        // transposes through LDS: T1 = h1 (points x units), T2 = h2, TD = dz1,
        // XS = x (points x features); then the weight gradients
        //   gW2 += dZ2^T h1, gW3 += dY^T h2, gW1 += dZ1^T x   (K = the 16 points)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                T1[16 * r + 4 * g + t][pi] = ok ? a.h1[r][t] : 0.f;
                T2[16 * r + 4 * g + t][pi] = ok ? a.h2[r][t] : 0.f;
                TD[16 * r + 4 * g + t][pi] = dz1[r][t];
            }
#pragma unroll
        for (int j = 0; j < 4; ++j) XS[pi][4 * g + j] = xv[j];
        wave_sync();
        // B operands [point][unit] of h1, h2 and the input; the A operands
        // [unit][point] of dZ1, dZ2 and dY are read from TD in turn
        v4s hb1[4], hb2[4], xtb;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // B operand [point][unit]: lane l holds H[4g + j][16r + i]
            hb1[r] = pack4(T1[16 * r + pi][4 * g + 0], T1[16 * r + pi][4 * g + 1],
                           T1[16 * r + pi][4 * g + 2], T1[16 * r + pi][4 * g + 3]);
            hb2[r] = pack4(T2[16 * r + pi][4 * g + 0], T2[16 * r + pi][4 * g + 1],
                           T2[16 * r + pi][4 * g + 2], T2[16 * r + pi][4 * g + 3]);
        }
        xtb = pack4(XS[4 * g + 0][pi], XS[4 * g + 1][pi], XS[4 * g + 2][pi], XS[4 * g + 3][pi]);
        // gW1 (units x features): A = dZ1^T [unit][point], B = X [point][feature]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const v4s ab = pack4(TD[16 * r + pi][4 * g + 0], TD[16 * r + pi][4 * g + 1],
                                 TD[16 * r + pi][4 * g + 2], TD[16 * r + pi][4 * g + 3]);
            gw1[r] = mfma(ab, xtb, gw1[r]);
        }
        wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < 4; ++t) TD[16 * r + 4 * g + t][pi] = dz2[r][t];
        wave_sync();
#pragma unroll
        for (int r2 = 0; r2 < 4; ++r2) {
            const v4s ab = pack4(TD[16 * r2 + pi][4 * g + 0], TD[16 * r2 + pi][4 * g + 1],
                                 TD[16 * r2 + pi][4 * g + 2], TD[16 * r2 + pi][4 * g + 3]);
#pragma unroll
            for (int r1 = 0; r1 < 4; ++r1) gw2[r2][r1] = mfma(ab, hb1[r1], gw2[r2][r1]);
        }
        // gW3 (outputs x units): A = dY^T [output][point]: lane l holds dY[4g+j][pi] ->
        // outputs live in lanes 0..15 of the D layout; stage through LDS row block 0
        wave_sync();
        if (g == 0) {
#pragma unroll
            for (int t = 0; t < 4; ++t) TD[t][pi] = dy[t];
        }
        wave_sync();
        {
            const v4s ab = (pi < NO) ? pack4(TD[pi][4 * g + 0], TD[pi][4 * g + 1],
                                             TD[pi][4 * g + 2], TD[pi][4 * g + 3])
                                     : pack4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int r = 0; r < 4; ++r) gw3[r] = mfma(ab, hb2[r], gw3[r]);
        }
        wave_sync();
    }
    // write this wave's partial gradients in the master layout
    float *pg = part + wave * NPAR;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = 16 * r + 4 * g + t;  // D row
            // gW1[row][feature pi] (features >= 12 dropped)
            if (pi < NI) pg[OW1 + row * NI + pi] = gw1[r][t];
#pragma unroll
            for (int r1 = 0; r1 < 4; ++r1) pg[OW2 + row * NH + 16 * r1 + pi] = gw2[r][r1][t];
            // gW3 rows are outputs (4g + t < 4 only for g = 0, r = ... ) see below
        }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (g == 0) pg[OW3 + t * NH + 16 * r + pi] = gw3[r][t];
    // biases: sum the 16 points held by lanes with the same g
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float s1 = gb1[r][t], s2 = gb2[r][t];
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                s1 += __shfl_xor(s1, o, 64);
                s2 += __shfl_xor(s2, o, 64);
            }
            if (pi == 0) {
                pg[OB1 + 16 * r + 4 * g + t] = s1;
                pg[OB2 + 16 * r + 4 * g + t] = s2;
            }
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float s3 = gb3[t];
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) s3 += __shfl_xor(s3, o, 64);
        if (lane == 0) pg[OB3 + t] = s3;
    }
    // loss partial (sum of squared normalised residuals) per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
    if (lane == 0) loss_part[wave] = lsum;
}

// The per-wave gradient partials part[nwaves][NPAR] are summed in a fixed
// order in two levels: chunks of RCH consecutive waves (one thread per
// parameter and chunk, so the loads of many chunks are in flight at once),
// then the chunks in order.
constexpr int RCH = 32;

__global__ void __launch_bounds__(256) k_mlp_chunks(const float *__restrict__ part, int nwaves,
                                                    float *__restrict__ chunks)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPAR) return;
    const int c = blockIdx.y;
    const int w0 = c * RCH, w1 = min(w0 + RCH, nwaves);
    float s = 0.f;
    for (int wv = w0; wv < w1; ++wv) s += part[(int64_t)wv * NPAR + k];
    chunks[(int64_t)c * NPAR + k] = s;
}

// Sum the chunk partials in order and apply Adam to the master.
__global__ void __launch_bounds__(256) k_mlp_adam(const float *__restrict__ chunks, int nchunk,
                                                  float *__restrict__ S, float lr, float b1,
                                                  float b2, float eps, int step)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPAR) return;
    float gsum = 0.f;
    for (int c = 0; c < nchunk; ++c) gsum += chunks[(int64_t)c * NPAR + k];
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    float m = S[OADAM_M + k] = b1 * S[OADAM_M + k] + (1.0f - b1) * gsum;
    float v = S[OADAM_V + k] = b2 * S[OADAM_V + k] + (1.0f - b2) * gsum * gsum;
    S[k] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

__global__ void __launch_bounds__(256) k_mlp_sum_partials(const float *__restrict__ chunks,
                                                           int nchunk, float *__restrict__ grad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPAR) return;
    float gsum = 0.f;
    for (int c = 0; c < nchunk; ++c) gsum += chunks[(int64_t)c * NPAR + k];
    grad[k] = gsum;
}

// Network outputs (normalised units) for raw feature rows X[n][12] -> Yo[n][4].
__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ S,
                                                     const float *__restrict__ X, int64_t n,
                                                     float *__restrict__ Yo)
{
    const int lane = threadIdx.x & 63, g = lane >> 4, pi = lane & 15;
    Weights w;
    load_weights(S, w, lane);
    float mu[4], isd[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * g + j;
        mu[j] = k < NI ? S[ONORM + k] : 0.f;
        isd[j] = k < NI ? S[ONORM + NI + k] : 0.f;
    }
    const int64_t ntile = (n + 15) / 16;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t tile = wave; tile < ntile; tile += nwaves) {
        const int64_t s = tile * 16 + pi;
        const bool ok = s < n;
        float xv[4] = {0.f, 0.f, 0.f, 0.f};
        if (ok && g < 3) {
#pragma unroll
            for (int j = 0; j < 4; ++j) xv[j] = (X[s * NI + 4 * g + j] - mu[j]) * isd[j];
        }
        Acts a;
        const v4f y = forward(w, pack4(xv[0], xv[1], xv[2], xv[3]), a);
        if (ok && g == 0) {
#pragma unroll
            for (int t = 0; t < 4; ++t) Yo[s * NO + t] = y[t];
        }
    }
}

// Mean squared error from the per-wave sums: one block, fixed order (strided
// per-thread sums, then a butterfly within each wave, then the waves in order).
__global__ void __launch_bounds__(256) k_loss_sum(const double *__restrict__ lp, int nwaves,
                                                  int64_t n, float *__restrict__ out)
{
    __shared__ double sh[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < nwaves; i += 256) s += lp[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (float)((((sh[0] + sh[1]) + sh[2]) + sh[3]) / (4.0 * (double)n));
}

}  // namespace mlp
}  // namespace fr

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {
using namespace fr;
using namespace fr::mlp;

constexpr int GRAD_BLOCKS = 256;  // k_mlp_grad grid: 1024 waves of gradient partials
constexpr int MOM_BLOCKS = 256;

int check_dev(const void *p, const char *name)
{
    if (!p) return set_error(FR_EINVAL, "%s is NULL", name);
    if (((uintptr_t)p) & 15) return set_error(FR_EINVAL, "%s is not 16-byte aligned", name);
    return FR_OK;
}

// splitmix64: deterministic host random numbers for the initial weights
uint64_t mix(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

constexpr int NWAVES_GRAD = GRAD_BLOCKS * TW;
constexpr int NCHUNK = (NWAVES_GRAD + RCH - 1) / RCH;

// Gradient partials per wave, then their chunk sums; *chunks_out holds NCHUNK
// rows of NPAR floats, *loss_out the per-wave squared-error sums.
int grad_impl(fr_plan *pl, const float *S, const float *X, const float *Y, int64_t n,
              float **chunks_out, double **loss_out, hipStream_t s)
{
    const size_t bytes = (size_t)NWAVES_GRAD * NPAR * sizeof(float) +
                         (size_t)NWAVES_GRAD * sizeof(double) +
                         (size_t)NCHUNK * NPAR * sizeof(float) + 64 * sizeof(float);
    if (int rc = ensure_scratch(pl->mlp, bytes)) return rc;
    float *part = (float *)pl->mlp.ptr;
    double *lp = (double *)(part + (size_t)NWAVES_GRAD * NPAR);
    float *chunks = (float *)(lp + NWAVES_GRAD);
    hipLaunchKernelGGL(k_mlp_grad, dim3(GRAD_BLOCKS), dim3(64 * TW), 0, s, S, X, Y, n, part, lp);
    if (int rc = check_hip(hipGetLastError(), "k_mlp_grad launch")) return rc;
    hipLaunchKernelGGL(k_mlp_chunks, dim3((NPAR + 255) / 256, NCHUNK), dim3(256), 0, s, part,
                       NWAVES_GRAD, chunks);
    *chunks_out = chunks;
    *loss_out = lp;
    return check_hip(hipGetLastError(), "k_mlp_chunks launch");
}

}  // namespace

extern "C" {

size_t fr_mlp_state_floats(void) { return (size_t)NSTATE; }

int fr_mlp_init(float *state, uint64_t seed, fr_stream_t s)
{
    if (int rc = check_dev(state, "state")) return rc;
    float *h = new (std::nothrow) float[NSTATE];
    if (!h) return set_error(FR_ENOMEM, "fr_mlp_init: host allocation");
    for (int i = 0; i < NSTATE; ++i) h[i] = 0.0f;
    uint64_t st = seed;
    auto uni = [&](float a) {  // uniform in [-a, a]
        const double u = (double)(mix(st) >> 11) * (1.0 / 9007199254740992.0);
        return (float)((2.0 * u - 1.0) * a);
    };
    const float a1 = std::sqrt(6.0f / (NI + NH)), a2 = std::sqrt(6.0f / (NH + NH));
    for (int i = 0; i < NH * NI; ++i) h[OW1 + i] = uni(a1);
    for (int i = 0; i < NH * NH; ++i) h[OW2 + i] = uni(a2);
    // W3 = b3 = 0: the initial network adds nothing to the extrapolation
    for (int k = 0; k < NI; ++k) h[ONORM + NI + k] = 1.0f;
    for (int k = 0; k < NO; ++k) h[ONORM + 2 * NI + k] = 1.0f;
    int rc = check_hip(hipMemcpyAsync(state, h, sizeof(float) * NSTATE, hipMemcpyHostToDevice,
                                      (hipStream_t)s),
                       "hipMemcpyAsync(mlp state)");
    if (!rc) rc = check_hip(hipStreamSynchronize((hipStream_t)s), "hipStreamSynchronize");
    delete[] h;
    return rc;
}

int fr_mlp_sample(fr_plan *pl, const double *Un, const double *Unm1, const double *Unm2,
                  const double *Unp1, int64_t offset, int64_t stride, int64_t n, float *X,
                  float *Y, fr_stream_t s)
{
    if (!pl) return set_error(FR_EINVAL, "fr_mlp_sample: NULL plan");
    if (int rc = check_dev(Un, "Un")) return rc;
    if (int rc = check_dev(Unm1, "Unm1")) return rc;
    if (int rc = check_dev(Unm2, "Unm2")) return rc;
    if (int rc = check_dev(X, "X")) return rc;
    if (int rc = check_dev(Y, "Y")) return rc;
    const int ns = pl->m * pl->m * pl->m;
    const int64_t npts = pl->ne * ns;
    if (n < 0 || stride < 1 || offset < 0 || (n > 0 && offset + (n - 1) * stride >= npts))
        return set_error(FR_EINVAL, "fr_mlp_sample: samples outside the %lld points",
                         (long long)npts);
    if (n == 0) return FR_OK;
    const int64_t g = (n + 255) / 256;
    hipLaunchKernelGGL(k_mlp_sample, dim3((unsigned)(g > 4096 ? 4096 : g)), dim3(256), 0,
                       (hipStream_t)s, Un, Unm1, Unm2, Unp1, offset, stride, n, ns, pl->guess_base,
                       X, Y);
    return check_hip(hipGetLastError(), "k_mlp_sample launch");
}

int fr_mlp_fit_norm(fr_plan *pl, float *state, const float *X, const float *Y, int64_t n,
                    fr_stream_t sv)
{
    if (!pl) return set_error(FR_EINVAL, "fr_mlp_fit_norm: NULL plan");
    if (int rc = check_dev(state, "state")) return rc;
    if (int rc = check_dev(X, "X")) return rc;
    if (int rc = check_dev(Y, "Y")) return rc;
    if (n < 2) return set_error(FR_EINVAL, "fr_mlp_fit_norm: need at least 2 samples");
    hipStream_t s = (hipStream_t)sv;
    if (int rc = ensure_scratch(pl->mlp, (size_t)MOM_BLOCKS * 32 * sizeof(double))) return rc;
    double *part = (double *)pl->mlp.ptr;
    hipLaunchKernelGGL(k_mlp_moments, dim3(MOM_BLOCKS), dim3(256), 0, s, X, Y, n, part);
    hipLaunchKernelGGL(k_mlp_norm, dim3(1), dim3(64), 0, s, part, MOM_BLOCKS, n, state);
    return check_hip(hipGetLastError(), "k_mlp_moments launch");
}

int fr_mlp_forward(fr_plan *pl, const float *state, const float *X, int64_t n, float *Yout,
                   fr_stream_t s)
{
    if (!pl) return set_error(FR_EINVAL, "fr_mlp_forward: NULL plan");
    if (int rc = check_dev(state, "state")) return rc;
    if (int rc = check_dev(X, "X")) return rc;
    if (int rc = check_dev(Yout, "Yout")) return rc;
    if (n < 1) return set_error(FR_EINVAL, "fr_mlp_forward: n = %lld", (long long)n);
    int64_t blocks = ((n + 15) / 16 + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)s, state,
                       X, n, Yout);
    return check_hip(hipGetLastError(), "k_mlp_forward launch");
}

int fr_mlp_grad(fr_plan *pl, const float *state, const float *X, const float *Y, int64_t n,
                float *grad, float *loss, fr_stream_t sv)
{
    if (!pl) return set_error(FR_EINVAL, "fr_mlp_grad: NULL plan");
    if (int rc = check_dev(state, "state")) return rc;
    if (int rc = check_dev(X, "X")) return rc;
    if (int rc = check_dev(Y, "Y")) return rc;
    if (int rc = check_dev(grad, "grad")) return rc;
    if (n < 1) return set_error(FR_EINVAL, "fr_mlp_grad: n = %lld", (long long)n);
    hipStream_t s = (hipStream_t)sv;
    float *chunks;
    double *lp;
    if (int rc = grad_impl(pl, state, X, Y, n, &chunks, &lp, s)) return rc;
    // fixed-order sum of the chunk partials, no update
    hipLaunchKernelGGL(k_mlp_sum_partials, dim3((NPAR + 255) / 256), dim3(256), 0, s, chunks,
                       NCHUNK, grad);
    if (loss) hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, s, lp, NWAVES_GRAD, n, loss);
    return check_hip(hipGetLastError(), "fr_mlp_grad launch");
}

int fr_mlp_train_step(fr_plan *pl, float *state, const float *X, const float *Y, int64_t n,
                      float lr, int step, float *loss, fr_stream_t sv)
{
    if (!pl) return set_error(FR_EINVAL, "fr_mlp_train_step: NULL plan");
    if (int rc = check_dev(state, "state")) return rc;
    if (int rc = check_dev(X, "X")) return rc;
    if (int rc = check_dev(Y, "Y")) return rc;
    if (n < 1 || step < 1 || !(lr >= 0.0f))
        return set_error(FR_EINVAL, "fr_mlp_train_step: n=%lld step=%d lr=%g", (long long)n, step,
                         (double)lr);
    hipStream_t s = (hipStream_t)sv;
    float *chunks;
    double *lp;
    if (int rc = grad_impl(pl, state, X, Y, n, &chunks, &lp, s)) return rc;
    if (loss) hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, s, lp, NWAVES_GRAD, n, loss);
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPAR + 255) / 256), dim3(256), 0, s, chunks, NCHUNK,
                       state, lr, 0.9f, 0.999f, 1e-8f, step);
    return check_hip(hipGetLastError(), "fr_mlp_train_step launch");
}

int fr_mlp_guess(fr_plan *pl, const float *state, const double *Un, const double *Unm1,
                 const double *Unm2, double *G, fr_stream_t s)
{
    if (!pl) return set_error(FR_EINVAL, "fr_mlp_guess: NULL plan");
    if (int rc = check_dev(state, "state")) return rc;
    if (int rc = check_dev(Un, "Un")) return rc;
    if (int rc = check_dev(Unm1, "Unm1")) return rc;
    if (int rc = check_dev(Unm2, "Unm2")) return rc;
    if (int rc = check_dev(G, "G")) return rc;
    const int ns = pl->m * pl->m * pl->m;
    const int64_t npts = pl->ne * ns;
    const int64_t groups = (npts + 63) / 64;   // 64 points per wave
    int64_t blocks = (groups + GUESS_WAVES - 1) / GUESS_WAVES;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_mlp_guess, dim3((unsigned)blocks), dim3(64 * GUESS_WAVES), 0,
                       (hipStream_t)s, state,
                       Un, Unm1, Unm2, G, npts, ns, pl->guess_base);
    return check_hip(hipGetLastError(), "k_mlp_guess launch");
}

}  // extern "C"
