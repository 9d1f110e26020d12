/*
 * mlp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain f64 reference of the surrogate network (a multilayer perceptron d_in -> H -> H -> d_out
 * with SiLU hidden activations) that the GPU's bfloat16 matrix-core kernels are checked against.  The
 * surrogate is not in the paper; it maps agent-population parameters to ensemble statistics
 * for calibration sweeps (the paper's parameter-sweep use case, section IV-J).
 *
 * Mixed precision is reproduced by rounding to bfloat16 (round to nearest, ties to even, on the
 * value first rounded to binary32) at exactly the points where the GPU stores bfloat16:
 * the input x, the weights, the hidden activations h1 and h2, the output gradient dy and the
 * hidden gradients dz2 and dz1.  Everything else is f64 here (f32 on the GPU).  With
 * round_bf16 = 0 no rounding happens, and backward() is the exact gradient of sum(dy * y),
 * which the tests check by central differences.
 *
 * Parameter layout (row-major, "in" index first):
 *   W1[d_in][H], b1[H], W2[H][H], b2[H], W3[H][d_out], b3[d_out].
 * Adam follows Kingma and Ba (2015), algorithm 1, with bias-corrected moments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* bfloat16 keeps the top 16 bits of a binary32; round to nearest even on the dropped 16 bits. */
double orm_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (double)f; /* inf / nan unchanged */
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double rb(double x, int on) { return on ? orm_bf16(x) : x; }

static double silu(double z) { return z / (1.0 + exp(-z)); }

static double dsilu(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

uint64_t orm_param_count(uint32_t d_in, uint32_t H, uint32_t d_out)
{
    return (uint64_t)d_in * H + H + (uint64_t)H * H + H + (uint64_t)H * d_out + d_out;
}

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3;
} orm_view;

static orm_view view(const double *p, uint32_t d_in, uint32_t H, uint32_t d_out)
{
    orm_view v;
    v.W1 = p;
    v.b1 = v.W1 + (size_t)d_in * H;
    v.W2 = v.b1 + H;
    v.b2 = v.W2 + (size_t)H * H;
    v.W3 = v.b2 + H;
    v.b3 = v.W3 + (size_t)H * d_out;
    return v;
}

/* Forward pass for N samples.  x[N][d_in] -> y[N][d_out].  If z1, h1, z2, h2 are non-NULL
 * ([N][H] each) the pre-activations and (rounded) activations are returned for backward(). */
void orm_forward(const double *params, uint32_t d_in, uint32_t H, uint32_t d_out, const double *x,
                 uint32_t N, int round_bf16, double *y, double *z1, double *h1, double *z2, double *h2)
{
    orm_view v = view(params, d_in, H, d_out);
    double *a1 = (double *)malloc(sizeof(double) * H);
    double *a2 = (double *)malloc(sizeof(double) * H);
    double *xr = (double *)malloc(sizeof(double) * d_in);
    for (uint32_t n = 0; n < N; ++n) {
        for (uint32_t i = 0; i < d_in; ++i) xr[i] = rb(x[(size_t)n * d_in + i], round_bf16);
        for (uint32_t j = 0; j < H; ++j) {
            double s = 0.0;
            for (uint32_t i = 0; i < d_in; ++i) s += xr[i] * rb(v.W1[(size_t)i * H + j], round_bf16);
            s += v.b1[j];
            if (z1) z1[(size_t)n * H + j] = s;
            a1[j] = rb(silu(s), round_bf16);
            if (h1) h1[(size_t)n * H + j] = a1[j];
        }
        for (uint32_t j = 0; j < H; ++j) {
            double s = 0.0;
            for (uint32_t i = 0; i < H; ++i) s += a1[i] * rb(v.W2[(size_t)i * H + j], round_bf16);
            s += v.b2[j];
            if (z2) z2[(size_t)n * H + j] = s;
            a2[j] = rb(silu(s), round_bf16);
            if (h2) h2[(size_t)n * H + j] = a2[j];
        }
        for (uint32_t k = 0; k < d_out; ++k) {
            double s = 0.0;
            for (uint32_t i = 0; i < H; ++i) s += a2[i] * rb(v.W3[(size_t)i * d_out + k], round_bf16);
            y[(size_t)n * d_out + k] = s + v.b3[k];
        }
    }
    free(a1);
    free(a2);
    free(xr);
}

/* Gradient of sum_{n,k} dy[n][k] * y[n][k] with respect to every parameter (layout of params),
 * summed over the N samples, written to grads.  Recomputes the forward pass itself. */
void orm_backward(const double *params, uint32_t d_in, uint32_t H, uint32_t d_out, const double *x,
                  const double *dy, uint32_t N, int round_bf16, double *grads)
{
    orm_view v = view(params, d_in, H, d_out);
    size_t NH = (size_t)N * H;
    double *z1 = (double *)malloc(sizeof(double) * NH);
    double *h1 = (double *)malloc(sizeof(double) * NH);
    double *z2 = (double *)malloc(sizeof(double) * NH);
    double *h2 = (double *)malloc(sizeof(double) * NH);
    double *y = (double *)malloc(sizeof(double) * (size_t)N * d_out);
    orm_forward(params, d_in, H, d_out, x, N, round_bf16, y, z1, h1, z2, h2);

    uint64_t P = orm_param_count(d_in, H, d_out);
    memset(grads, 0, sizeof(double) * P);
    double *gW1 = grads;
    double *gb1 = gW1 + (size_t)d_in * H;
    double *gW2 = gb1 + H;
    double *gb2 = gW2 + (size_t)H * H;
    double *gW3 = gb2 + H;
    double *gb3 = gW3 + (size_t)H * d_out;

    double *g = (double *)malloc(sizeof(double) * d_out);
    double *dz2 = (double *)malloc(sizeof(double) * H);
    double *dz1 = (double *)malloc(sizeof(double) * H);
    for (uint32_t n = 0; n < N; ++n) {
        const double *hn1 = h1 + (size_t)n * H, *hn2 = h2 + (size_t)n * H;
        for (uint32_t k = 0; k < d_out; ++k) g[k] = rb(dy[(size_t)n * d_out + k], round_bf16);
        /* output layer */
        for (uint32_t i = 0; i < H; ++i)
            for (uint32_t k = 0; k < d_out; ++k) gW3[(size_t)i * d_out + k] += hn2[i] * g[k];
        for (uint32_t k = 0; k < d_out; ++k) gb3[k] += g[k];
        /* second hidden layer */
        for (uint32_t i = 0; i < H; ++i) {
            double s = 0.0;
            for (uint32_t k = 0; k < d_out; ++k) s += g[k] * rb(v.W3[(size_t)i * d_out + k], round_bf16);
            dz2[i] = rb(s * dsilu(z2[(size_t)n * H + i]), round_bf16);
        }
        for (uint32_t i = 0; i < H; ++i)
            for (uint32_t j = 0; j < H; ++j) gW2[(size_t)i * H + j] += hn1[i] * dz2[j];
        for (uint32_t j = 0; j < H; ++j) gb2[j] += dz2[j];
        /* first hidden layer */
        for (uint32_t i = 0; i < H; ++i) {
            double s = 0.0;
            for (uint32_t j = 0; j < H; ++j) s += dz2[j] * rb(v.W2[(size_t)i * H + j], round_bf16);
            dz1[i] = rb(s * dsilu(z1[(size_t)n * H + i]), round_bf16);
        }
        for (uint32_t i = 0; i < d_in; ++i) {
            double xi = rb(x[(size_t)n * d_in + i], round_bf16);
            for (uint32_t j = 0; j < H; ++j) gW1[(size_t)i * H + j] += xi * dz1[j];
        }
        for (uint32_t j = 0; j < H; ++j) gb1[j] += dz1[j];
    }
    free(g);
    free(dz2);
    free(dz1);
    free(z1);
    free(h1);
    free(z2);
    free(h2);
    free(y);
}

/* One Adam step (t >= 1) on n parameters, in place. */
void orm_adam(double *p, const double *g, double *m, double *v, uint64_t n, uint32_t t, double lr,
              double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (uint64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
