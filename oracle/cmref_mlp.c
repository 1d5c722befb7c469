/*
 * Learned SGS closure: reference network (TEST INFRASTRUCTURE ONLY).
 *
 * A 12-64-64-64-2 multilayer perceptron with SiLU hidden activations maps
 * standardised local inputs (resolved velocity gradient, buoyancy frequency
 * N^2, filter width, a TKE estimate) to an eddy viscosity and a turbulent
 * Prandtl number.  The paper's closures (Sect. 4: Smagorinsky-Lilly,
 * Richardson factor) give the fallback and the feature set; the network is
 * the learned replacement.
 *
 * Parameter vector (FP64 here, FP32 on the GPU), layer by layer, each weight
 * matrix row-major [out][in] followed by its bias:
 *   W1[64][12] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2]
 * = 9282 values.  Output mapping: nu_t = Delta^2 |S| softplus(o1),
 * Pr_t = 0.1 + softplus(o2).
 *
 * Provided: FP64 forward; forward with bfloat16 rounding of every matrix
 * operand (round to nearest even) at the points where the GPU kernels round;
 * FP64 gradient of the mean squared error of the raw outputs; one Adam step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NI 12
#define NH 64
#define NO 2
#define NPARAM (NH * NI + NH + NH * NH + NH + NH * NH + NH + NO * NH + NO)

static const int OFF_W1 = 0;
static const int OFF_B1 = NH * NI;
static const int OFF_W2 = NH * NI + NH;
static const int OFF_B2 = NH * NI + NH + NH * NH;
static const int OFF_W3 = NH * NI + NH + NH * NH + NH;
static const int OFF_B3 = NH * NI + NH + 2 * NH * NH + NH;
static const int OFF_W4 = NH * NI + 2 * NH + 2 * NH * NH + NH;
static const int OFF_B4 = NH * NI + 2 * NH + 2 * NH * NH + NH + NO * NH;

int cmref_mlp_nparams(void) { return NPARAM; }

static double silu(double x) { return x / (1.0 + exp(-x)); }
static double dsilu(double x)
{
    double s = 1.0 / (1.0 + exp(-x));
    return s * (1.0 + x * (1.0 - s));
}
static double softplus(double x) { return x > 30.0 ? x : log1p(exp(x)); }

/* round a float to the nearest bfloat16 (ties to even), returned as float */
static float bf16_round(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return f; /* inf / nan unchanged */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

double cmref_bf16(double x) { return (double)bf16_round((float)x); }

/* one dense layer: out[o] = sum_i W[o][i] in[i] + b[o] */
static void dense(const double* W, const double* b, const double* in, int ni, int no, double* out)
{
    for (int o = 0; o < no; ++o) {
        double s = 0.0;
        for (int i = 0; i < ni; ++i) s += W[o * ni + i] * in[i];
        out[o] = s + b[o];
    }
}

/* Forward of one standardised input.  bf16 = 0: FP64 throughout.  bf16 = 1:
 * W holds weights already rounded to bfloat16; the input and each hidden
 * activation are rounded to bf16 before they enter a matrix product,
 * products are summed exactly (FP64), and bias and activation are applied in
 * FP32 arithmetic on the sum (the rounding points of the GPU kernels). */
static void forward_one(const double* W, const double* b, const double* x, int bf16, double* o)
{
    const int offW[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4};
    const int offB[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
    double in[NH], a[NH];
    for (int i = 0; i < NI; ++i) in[i] = bf16 ? cmref_bf16(x[i]) : x[i];
    int ni = NI;
    for (int layer = 0; layer < 4; ++layer) {
        const int no = layer == 3 ? NO : NH;
        for (int k = 0; k < no; ++k) {
            double acc = 0.0;
            for (int i = 0; i < ni; ++i) acc += W[offW[layer] + k * ni + i] * in[i];
            if (bf16) {
                const float z = (float)acc + (float)b[offB[layer] + k];
                a[k] = layer == 3 ? (double)z : (double)(z / (1.0f + expf(-z)));
            } else {
                const double z = acc + b[offB[layer] + k];
                a[k] = layer == 3 ? z : silu(z);
            }
        }
        if (layer == 3) {
            for (int k = 0; k < NO; ++k) o[k] = a[k];
        } else {
            for (int k = 0; k < NH; ++k) in[k] = bf16 ? cmref_bf16(a[k]) : a[k];
            ni = NH;
        }
    }
}

/* FP64 forward of a batch of standardised inputs x[n][12] -> raw outputs o[n][2] */
void cmref_mlp_forward(const double* p, const double* x, int n, double* o)
{
    for (int s = 0; s < n; ++s) forward_one(p, p, x + s * NI, 0, o + s * NO);
}

/* The same with bfloat16 matrix operands (see forward_one) */
void cmref_mlp_forward_bf16(const double* p, const double* x, int n, double* o)
{
    double* Wr = (double*)malloc(sizeof(double) * NPARAM);
    for (int q = 0; q < NPARAM; ++q) Wr[q] = cmref_bf16(p[q]);
    for (int s = 0; s < n; ++s) forward_one(Wr, p, x + s * NI, 1, o + s * NO);
    free(Wr);
}

/* Loss L = (1/n) sum_s sum_k (o_sk - t_sk)^2 and its FP64 gradient with
 * respect to every parameter (back-propagation written out layer by layer). */
double cmref_mlp_grad(const double* p, const double* x, const double* t, int n, double* g)
{
    memset(g, 0, sizeof(double) * NPARAM);
    double a1[NH], a2[NH], a3[NH], h1[NH], h2[NH], h3[NH], o[NO];
    double d3[NH], d2[NH], d1[NH], dh[NH], dout[NO];
    double loss = 0.0;
    for (int s = 0; s < n; ++s) {
        const double* xs = x + s * NI;
        dense(p + OFF_W1, p + OFF_B1, xs, NI, NH, a1);
        for (int k = 0; k < NH; ++k) h1[k] = silu(a1[k]);
        dense(p + OFF_W2, p + OFF_B2, h1, NH, NH, a2);
        for (int k = 0; k < NH; ++k) h2[k] = silu(a2[k]);
        dense(p + OFF_W3, p + OFF_B3, h2, NH, NH, a3);
        for (int k = 0; k < NH; ++k) h3[k] = silu(a3[k]);
        dense(p + OFF_W4, p + OFF_B4, h3, NH, NO, o);
        for (int k = 0; k < NO; ++k) {
            double r = o[k] - t[s * NO + k];
            loss += r * r;
            dout[k] = 2.0 * r / n;
        }
        /* layer 4 */
        for (int k = 0; k < NO; ++k) {
            for (int i = 0; i < NH; ++i) g[OFF_W4 + k * NH + i] += dout[k] * h3[i];
            g[OFF_B4 + k] += dout[k];
        }
        for (int i = 0; i < NH; ++i) {
            double s4 = 0.0;
            for (int k = 0; k < NO; ++k) s4 += p[OFF_W4 + k * NH + i] * dout[k];
            d3[i] = s4 * dsilu(a3[i]);
        }
        /* layer 3 */
        for (int k = 0; k < NH; ++k) {
            for (int i = 0; i < NH; ++i) g[OFF_W3 + k * NH + i] += d3[k] * h2[i];
            g[OFF_B3 + k] += d3[k];
        }
        for (int i = 0; i < NH; ++i) {
            double s3 = 0.0;
            for (int k = 0; k < NH; ++k) s3 += p[OFF_W3 + k * NH + i] * d3[k];
            dh[i] = s3;
        }
        for (int i = 0; i < NH; ++i) d2[i] = dh[i] * dsilu(a2[i]);
        /* layer 2 */
        for (int k = 0; k < NH; ++k) {
            for (int i = 0; i < NH; ++i) g[OFF_W2 + k * NH + i] += d2[k] * h1[i];
            g[OFF_B2 + k] += d2[k];
        }
        for (int i = 0; i < NH; ++i) {
            double s2 = 0.0;
            for (int k = 0; k < NH; ++k) s2 += p[OFF_W2 + k * NH + i] * d2[k];
            d1[i] = s2 * dsilu(a1[i]);
        }
        /* layer 1 */
        for (int k = 0; k < NH; ++k) {
            for (int i = 0; i < NI; ++i) g[OFF_W1 + k * NI + i] += d1[k] * xs[i];
            g[OFF_B1 + k] += d1[k];
        }
    }
    return loss / n;
}

static float silu_f(float z) { return z / (1.0f + expf(-z)); }
static float dsilu_f(float z)
{
    float sg = 1.0f / (1.0f + expf(-z));
    return sg * (1.0f + z * (1.0f - sg));
}
static float bfr(double v) { return bf16_round((float)v); }

/* The loss gradient as the GPU's training kernels form it, for an
 * element-wise comparison: every operand of a matrix product (inputs,
 * weights, activations, output and hidden gradients) rounded to bfloat16,
 * the products summed exactly (FP64, where the GPU sums in FP32), sums of
 * products rounded to FP32, then FP32 arithmetic for the bias, SiLU and its
 * derivative, and the output residual 2 (o - t)/n.  mag[q] receives the
 * sum of the magnitudes of the terms that make up g[q] (the scale an FP32
 * summation error is relative to).  Returns the loss. */
double cmref_mlp_grad_bf16(const double* p, const double* x, const double* t, int n, double* g, double* mag)
{
    const int offW[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4};
    const int offB[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
    const int nin[4] = {NI, NH, NH, NH}, nout[4] = {NH, NH, NH, NO};
    float* Wb = (float*)malloc(sizeof(float) * NPARAM);
    for (int q = 0; q < NPARAM; ++q) Wb[q] = bfr(p[q]);
    /* per layer: the bf16 input of the product and the FP32 pre-activation */
    float* in[4];
    float* Z[4];
    for (int l = 0; l < 4; ++l) {
        in[l] = (float*)malloc(sizeof(float) * (size_t)n * nin[l]);
        Z[l] = (float*)malloc(sizeof(float) * (size_t)n * nout[l]);
    }
    for (int s = 0; s < n; ++s)
        for (int i = 0; i < NI; ++i) in[0][s * NI + i] = bfr(x[s * NI + i]);
    for (int l = 0; l < 4; ++l)
        for (int s = 0; s < n; ++s)
            for (int k = 0; k < nout[l]; ++k) {
                double acc = 0.0;
                for (int i = 0; i < nin[l]; ++i) acc += (double)in[l][s * nin[l] + i] * Wb[offW[l] + k * nin[l] + i];
                float z = (float)acc + (float)p[offB[l] + k];
                Z[l][s * nout[l] + k] = z;
                if (l < 3) in[l + 1][s * NH + k] = bf16_round(silu_f(z));
            }
    memset(g, 0, sizeof(double) * NPARAM);
    memset(mag, 0, sizeof(double) * NPARAM);
    /* output residual */
    float* d = (float*)malloc(sizeof(float) * (size_t)n * NH);
    float* dn = (float*)malloc(sizeof(float) * (size_t)n * NH);
    double loss = 0.0;
    for (int s = 0; s < n; ++s)
        for (int k = 0; k < NO; ++k) {
            float r = Z[3][s * NO + k] - (float)t[s * NO + k];
            loss += (double)r * r;
            d[s * NO + k] = 2.0f * r / (float)n;
        }
    for (int l = 3; l >= 0; --l) {
        const int no = nout[l], ni = nin[l];
        /* weight gradient sum_s bf16(d) bf16(in), bias gradient sum_s d */
        for (int k = 0; k < no; ++k) {
            for (int i = 0; i < ni; ++i) {
                double acc = 0.0, am = 0.0;
                for (int s = 0; s < n; ++s) {
                    double term = (double)bf16_round(d[s * no + k]) * in[l][s * ni + i];
                    acc += term;
                    am += fabs(term);
                }
                g[offW[l] + k * ni + i] = (double)(float)acc;
                mag[offW[l] + k * ni + i] = am;
            }
            double acc = 0.0, am = 0.0;
            for (int s = 0; s < n; ++s) { acc += d[s * no + k]; am += fabs(d[s * no + k]); }
            g[offB[l] + k] = (double)(float)acc;
            mag[offB[l] + k] = am;
        }
        if (l == 0) break;
        /* gradient of the layer below's pre-activation */
        for (int s = 0; s < n; ++s)
            for (int i = 0; i < ni; ++i) {
                double acc = 0.0;
                for (int k = 0; k < no; ++k) acc += (double)bf16_round(d[s * no + k]) * Wb[offW[l] + k * ni + i];
                dn[s * ni + i] = (float)acc * dsilu_f(Z[l - 1][s * NH + i]);
            }
        float* tmp = d; d = dn; dn = tmp;
    }
    for (int l = 0; l < 4; ++l) { free(in[l]); free(Z[l]); }
    free(d); free(dn); free(Wb);
    return loss / n;
}

/* One Adam step (Kingma & Ba) with bias correction; step counts from 1. */
void cmref_adam_step(double* p, const double* g, double* m, double* v, int step, double lr, double b1,
                     double b2, double eps)
{
    double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    for (int q = 0; q < NPARAM; ++q) {
        m[q] = b1 * m[q] + (1.0 - b1) * g[q];
        v[q] = b2 * v[q] + (1.0 - b2) * g[q] * g[q];
        double mh = m[q] / c1, vh = v[q] / c2;
        p[q] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Closure at one node for the RHS oracle.  params = [network (9282),
 * mean[12], std[12]]; Wb = the network with bf16-rounded weights, or NULL
 * for the FP64 network; lo/hi = standardised training range.  Returns 1 when
 * the node falls back to Smagorinsky (an input outside the range widened by
 * 10 % of its half-width on each side plus 2^-20 (1 + |mean/std|), or a
 * non-finite output). */
int cmref_mlp_closure(const double* params, const double* Wb, const double* lo, const double* hi,
                      int use_fallback, const double gu[3][3], double N2, double Delta, double nu_sl,
                      double* nu, double* Prt)
{
    const double* mean = params + NPARAM;
    const double* sd = params + NPARAM + NI;
    double raw[NI], x[NI];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) raw[3 * i + j] = gu[i][j];
    raw[9] = N2;
    raw[10] = Delta;
    double k = nu_sl / (0.1 * Delta);
    raw[11] = k * k;
    int out_of_range = 0;
    for (int i = 0; i < NI; ++i) {
        x[i] = (raw[i] - mean[i]) / sd[i];
        double c = 0.5 * (lo[i] + hi[i]), r = 0.5 * (hi[i] - lo[i]);
        /* the margin 2^-20 (1 + |mean/std|) absorbs the float rounding of the
         * normalisation, so an input that was constant in training (zero
         * half-width) passes at its training value */
        double tol = ldexp(1.0 + fabs(mean[i] / sd[i]), -20);
        if (fabs(x[i] - c) > 1.1 * r + tol) out_of_range = 1;
    }
    double o[NO];
    forward_one(Wb ? Wb : params, params, x, Wb != NULL, o);
    double SS = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.5 * (gu[i][j] + gu[j][i]);
            SS += 2.0 * s * s;
        }
    *nu = Delta * Delta * sqrt(SS) * softplus(o[0]);
    *Prt = 0.1 + softplus(o[1]);
    if (use_fallback && (out_of_range || !isfinite(*nu) || !isfinite(*Prt))) return 1;
    return 0;
}

/* network with bf16-rounded weight matrices (biases kept), for the closure */
void cmref_mlp_round_weights(const double* p, double* out)
{
    for (int q = 0; q < NPARAM; ++q) out[q] = cmref_bf16(p[q]);
}
