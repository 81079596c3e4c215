/*
 * mlp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain double-precision reference for the pointwise multilayer perceptron
 * that supplies the initial guess of each physical step's pseudo-time
 * iteration (not part of the paper; the method is unchanged by it, because
 * the converged pseudo-residual decides the answer).  Textbook forward pass,
 * back-propagation of the mean-squared error, and Adam, written out with
 * loops.  Shares no code with the GPU library.
 *
 * Network (per point, 12 -> 64 -> 64 -> 4):
 *   h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3,
 * W1[64][12], W2[64][64], W3[4][64] row-major (output index first).
 * Loss: L = (1/(4n)) sum_{points, outputs} (y - t)^2.
 *
 * Operand rounding (rnd != 0): the matrix products then take their operands
 * in bfloat16, as matrix cores with bfloat16 inputs and wide accumulation do.
 * Every operand of every product is rounded -- in the forward pass the layer
 * inputs x, h1, h2 and the weights W1, W2, W3; in the backward pass the
 * back-propagated gradients dL/dy, dL/dz2, dL/dz1 together with the weights
 * they are multiplied by and the activations (x, h1, h2) they meet in the
 * weight gradients -- while the sums accumulate in double, and biases, tanh,
 * its derivative 1 - h^2 and the bias gradients use the unrounded values.
 * bf16() rounds a value first to binary32 and then to the bfloat16 format (the
 * upper 16 bits of binary32: 8 significant bits), round to nearest, ties to
 * even, from the formats' definitions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NI 12
#define NH 64
#define NO 4

/* binary64 -> binary32 (the C conversion rounds to nearest even) -> bfloat16:
 * keep the upper 16 bits of the binary32 pattern, adding half a unit of the
 * kept part plus the kept part's lowest bit (ties to even).  Finite inputs. */
static double bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

static double rd(double x, int rnd) { return rnd ? bf16(x) : x; }

/* y[i] = bf16(x[i]) (exposed so that the rounding itself can be checked). */
void orc_bf16(int64_t n, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) y[i] = bf16(x[i]);
}

static void forward_one(const double *x, const double *W1, const double *b1,
                        const double *W2, const double *b2, const double *W3,
                        const double *b3, double *h1, double *h2, double *y, int rnd)
{
    for (int o = 0; o < NH; ++o) {
        double s = b1[o];
        for (int i = 0; i < NI; ++i) s += rd(W1[o * NI + i], rnd) * rd(x[i], rnd);
        h1[o] = tanh(s);
    }
    for (int o = 0; o < NH; ++o) {
        double s = b2[o];
        for (int i = 0; i < NH; ++i) s += rd(W2[o * NH + i], rnd) * rd(h1[i], rnd);
        h2[o] = tanh(s);
    }
    for (int o = 0; o < NO; ++o) {
        double s = b3[o];
        for (int i = 0; i < NH; ++i) s += rd(W3[o * NH + i], rnd) * rd(h2[i], rnd);
        y[o] = s;
    }
}

/* Y[n][4] = network(X[n][12]); H (nullable) receives [n][h1(64), h2(64)]. */
void orc_mlp_forward(int64_t n, const double *X, const double *W1, const double *b1,
                     const double *W2, const double *b2, const double *W3, const double *b3,
                     double *Y, double *H, int rnd)
{
    double h1[NH], h2[NH];
    for (int64_t s = 0; s < n; ++s) {
        forward_one(X + s * NI, W1, b1, W2, b2, W3, b3, h1, h2, Y + s * NO, rnd);
        if (H) {
            memcpy(H + s * 2 * NH, h1, sizeof h1);
            memcpy(H + s * 2 * NH + NH, h2, sizeof h2);
        }
    }
}

/* Mean-squared-error loss and its gradient with respect to every parameter
 * (gradients overwritten, not accumulated).  Returns the loss. */
double orc_mlp_loss_grad(int64_t n, const double *X, const double *Tg, const double *W1,
                         const double *b1, const double *W2, const double *b2,
                         const double *W3, const double *b3, double *gW1, double *gb1,
                         double *gW2, double *gb2, double *gW3, double *gb3, int rnd)
{
    memset(gW1, 0, sizeof(double) * NH * NI);
    memset(gb1, 0, sizeof(double) * NH);
    memset(gW2, 0, sizeof(double) * NH * NH);
    memset(gb2, 0, sizeof(double) * NH);
    memset(gW3, 0, sizeof(double) * NO * NH);
    memset(gb3, 0, sizeof(double) * NO);
    double h1[NH], h2[NH], y[NO], dy[NO], d2[NH], d1[NH];
    double loss = 0.0;
    const double scale = 1.0 / (4.0 * (double)n);
    for (int64_t s = 0; s < n; ++s) {
        const double *x = X + s * NI;
        forward_one(x, W1, b1, W2, b2, W3, b3, h1, h2, y, rnd);
        for (int o = 0; o < NO; ++o) {
            double r = y[o] - Tg[s * NO + o];
            loss += r * r;
            dy[o] = 2.0 * r * scale;        /* dL/dy */
        }
        for (int o = 0; o < NO; ++o) {
            gb3[o] += dy[o];
            for (int i = 0; i < NH; ++i) gW3[o * NH + i] += rd(dy[o], rnd) * rd(h2[i], rnd);
        }
        for (int i = 0; i < NH; ++i) {      /* through tanh: 1 - h^2 */
            double g = 0.0;
            for (int o = 0; o < NO; ++o) g += rd(W3[o * NH + i], rnd) * rd(dy[o], rnd);
            d2[i] = g * (1.0 - h2[i] * h2[i]);
        }
        for (int o = 0; o < NH; ++o) {
            gb2[o] += d2[o];
            for (int i = 0; i < NH; ++i) gW2[o * NH + i] += rd(d2[o], rnd) * rd(h1[i], rnd);
        }
        for (int i = 0; i < NH; ++i) {
            double g = 0.0;
            for (int o = 0; o < NH; ++o) g += rd(W2[o * NH + i], rnd) * rd(d2[o], rnd);
            d1[i] = g * (1.0 - h1[i] * h1[i]);
        }
        for (int o = 0; o < NH; ++o) {
            gb1[o] += d1[o];
            for (int i = 0; i < NI; ++i) gW1[o * NI + i] += rd(d1[o], rnd) * rd(x[i], rnd);
        }
    }
    return loss * scale;
}

/* Adam (Kingma & Ba) with bias correction; step counts from 1. */
void orc_adam(int64_t n, double *param, const double *grad, double *m, double *v, double lr,
              double beta1, double beta2, double eps, int step)
{
    double c1 = 1.0 - pow(beta1, step), c2 = 1.0 - pow(beta2, step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        param[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
