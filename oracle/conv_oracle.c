/*
 * conv_oracle.c -- plain FP64 reference of the convolutional surrogate.
 *
 * TEST INFRASTRUCTURE ONLY (see pf_oracle.c).  The network (a learned
 * component added by this project; the paper has none) maps the input planes
 * (c, M, kappa) of a Cahn-Hilliard state to the field K explicit steps later:
 *   a0 = (c, M, kappa)                                   [B, H, W, 3]
 *   a_l = relu(conv3x3(a_{l-1}; W_l) + b_l), l = 1, 2, 3  32 channels each
 *   d   = conv3x3(a_3; W_4) + b_4                          1 channel
 *   c_hat = c + d - mean(d)                                (per sample: exact mass)
 * Periodic 3x3 cross-correlation, NHWC layout, weights [ky][kx][cin][cout].
 * Loss L = sum_b mean_p (c_hat - target)^2.
 *
 * With round = 1 every quantity the GPU stores in bfloat16 is rounded to
 * bfloat16 here too, at the same points: the network input, the weights, each
 * hidden activation after bias and relu, and each hidden activation gradient
 * after the relu mask.  With round = 0 everything stays FP64 (used to check
 * this backward pass against finite differences).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* round to the nearest bfloat16 (8 significant bits), ties to even */
double orc_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    double m = frexp(x, &e); /* x = m 2^e, 0.5 <= |m| < 1 */
    double s = ldexp(m, 8);  /* 8 significant bits */
    double r = nearbyint(s); /* default rounding mode: to nearest, ties to even */
    return ldexp(r, e - 8);
}

static double rd(int round, double x) { return round ? orc_bf16(x) : x; }

/* out[b,y,x,co] = bias[co] + sum_{ky,kx,ci} w[ky,kx,ci,co] in[b,(y+ky-1)%H,(x+kx-1)%W,ci] */
static void conv3x3(int B, int H, int W, int Ci, int Co, const double* in, const double* w,
                    const double* bias, double* out)
{
    for (int b = 0; b < B; ++b)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                for (int co = 0; co < Co; ++co) {
                    double s = bias ? bias[co] : 0.0;
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int yy = (y + ky - 1 + H) % H, xx = (x + kx - 1 + W) % W;
                            const double* ip = in + (((size_t)b * H + yy) * W + xx) * Ci;
                            const double* wp = w + ((size_t)(ky * 3 + kx) * Ci) * Co + co;
                            for (int ci = 0; ci < Ci; ++ci) s += wp[(size_t)ci * Co] * ip[ci];
                        }
                    out[(((size_t)b * H + y) * W + x) * Co + co] = s;
                }
}

/* gradient of conv3x3 with respect to its input:
 * gin[b,yy,xx,ci] = sum over (y,x,ky,kx) with yy=(y+ky-1), xx=(x+kx-1) of w[ky,kx,ci,co] gout[b,y,x,co] */
static void conv3x3_dgrad(int B, int H, int W, int Ci, int Co, const double* gout, const double* w,
                          double* gin)
{
    memset(gin, 0, sizeof(double) * (size_t)B * H * W * Ci);
    for (int b = 0; b < B; ++b)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        int yy = (y + ky - 1 + H) % H, xx = (x + kx - 1 + W) % W;
                        double* gp = gin + (((size_t)b * H + yy) * W + xx) * Ci;
                        const double* go = gout + (((size_t)b * H + y) * W + x) * Co;
                        for (int ci = 0; ci < Ci; ++ci) {
                            const double* wp = w + ((size_t)(ky * 3 + kx) * Ci + ci) * Co;
                            double s = 0.0;
                            for (int co = 0; co < Co; ++co) s += wp[co] * go[co];
                            gp[ci] += s;
                        }
                    }
}

/* gradient with respect to the weights and bias (accumulated into gw, gb) */
static void conv3x3_wgrad(int B, int H, int W, int Ci, int Co, const double* in, const double* gout,
                          double* gw, double* gb)
{
    for (int b = 0; b < B; ++b)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                const double* go = gout + (((size_t)b * H + y) * W + x) * Co;
                for (int co = 0; co < Co; ++co) gb[co] += go[co];
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        int yy = (y + ky - 1 + H) % H, xx = (x + kx - 1 + W) % W;
                        const double* ip = in + (((size_t)b * H + yy) * W + xx) * Ci;
                        for (int ci = 0; ci < Ci; ++ci) {
                            double* g = gw + ((size_t)(ky * 3 + kx) * Ci + ci) * Co;
                            for (int co = 0; co < Co; ++co) g[co] += ip[ci] * go[co];
                        }
                    }
            }
}

/* Parameter block, all FP64 "master" values:
 *   W1 [9*3*32], b1[32], W2 [9*32*32], b2[32], W3 [9*32*32], b3[32], W4 [9*32*1], b4[1] */
enum { C_HID = 32 };
static size_t nparam_layout(size_t off[9])
{
    size_t o = 0;
    off[0] = o; o += 9 * 3 * C_HID;
    off[1] = o; o += C_HID;
    off[2] = o; o += 9 * C_HID * C_HID;
    off[3] = o; o += C_HID;
    off[4] = o; o += 9 * C_HID * C_HID;
    off[5] = o; o += C_HID;
    off[6] = o; o += 9 * C_HID;
    off[7] = o; o += 1;
    off[8] = o;
    return o;
}

int64_t orc_nn_nparams(void)
{
    size_t off[9];
    return (int64_t)nparam_layout(off);
}

/* Forward pass and (if grad != NULL) loss gradient with respect to the
 * parameters.  inputs: c, M, kappa planes [B,H,W] each; target [B,H,W] or NULL.
 * Writes c_hat [B,H,W]; returns the loss (0 if target is NULL). */
double orc_nn(int B, int H, int W, const double* c, const double* M, const double* kap,
              const double* target, const double* params, int round, double* chat, double* grad)
{
    size_t off[9];
    const size_t np = nparam_layout(off);
    const size_t P = (size_t)B * H * W;
    double* w = (double*)malloc(sizeof(double) * np);
    for (size_t i = 0; i < np; ++i) w[i] = params[i];
    /* weights are used in bfloat16; biases stay FP32/FP64 */
    for (int l = 0; l < 4; ++l) {
        size_t a = off[2 * l], e = off[2 * l + 1];
        for (size_t i = a; i < e; ++i) w[i] = rd(round, w[i]);
    }
    double* a0 = (double*)malloc(sizeof(double) * P * 3);
    double* a1 = (double*)malloc(sizeof(double) * P * C_HID);
    double* a2 = (double*)malloc(sizeof(double) * P * C_HID);
    double* a3 = (double*)malloc(sizeof(double) * P * C_HID);
    double* d = (double*)malloc(sizeof(double) * P);
    for (size_t p = 0; p < P; ++p) {
        a0[3 * p + 0] = rd(round, c[p]);
        a0[3 * p + 1] = rd(round, M[p]);
        a0[3 * p + 2] = rd(round, kap[p]);
    }
    conv3x3(B, H, W, 3, C_HID, a0, w + off[0], w + off[1], a1);
    for (size_t i = 0; i < P * C_HID; ++i) a1[i] = rd(round, a1[i] > 0.0 ? a1[i] : 0.0);
    conv3x3(B, H, W, C_HID, C_HID, a1, w + off[2], w + off[3], a2);
    for (size_t i = 0; i < P * C_HID; ++i) a2[i] = rd(round, a2[i] > 0.0 ? a2[i] : 0.0);
    conv3x3(B, H, W, C_HID, C_HID, a2, w + off[4], w + off[5], a3);
    for (size_t i = 0; i < P * C_HID; ++i) a3[i] = rd(round, a3[i] > 0.0 ? a3[i] : 0.0);
    conv3x3(B, H, W, C_HID, 1, a3, w + off[6], w + off[7], d);
    const size_t HW = (size_t)H * W;
    double loss = 0.0;
    for (int b = 0; b < B; ++b) {
        double mean = 0.0;
        for (size_t i = 0; i < HW; ++i) mean += d[b * HW + i];
        mean /= (double)HW;
        for (size_t i = 0; i < HW; ++i) chat[b * HW + i] = c[b * HW + i] + d[b * HW + i] - mean;
        if (target) {
            double s = 0.0;
            for (size_t i = 0; i < HW; ++i) {
                double r = chat[b * HW + i] - target[b * HW + i];
                s += r * r;
            }
            loss += s / (double)HW;
        }
    }
    if (grad && target) {
        memset(grad, 0, sizeof(double) * np);
        double* g = (double*)malloc(sizeof(double) * P);
        double* ga = (double*)malloc(sizeof(double) * P * C_HID);
        double* gb = (double*)malloc(sizeof(double) * P * C_HID);
        /* dL/dc_hat, then through the mean projection */
        for (int b = 0; b < B; ++b) {
            double mean = 0.0;
            for (size_t i = 0; i < HW; ++i) {
                g[b * HW + i] = 2.0 * (chat[b * HW + i] - target[b * HW + i]) / (double)HW;
                mean += g[b * HW + i];
            }
            mean /= (double)HW;
            for (size_t i = 0; i < HW; ++i) g[b * HW + i] -= mean;
        }
        conv3x3_wgrad(B, H, W, C_HID, 1, a3, g, grad + off[6], grad + off[7]);
        conv3x3_dgrad(B, H, W, C_HID, 1, g, w + off[6], ga);
        for (size_t i = 0; i < P * C_HID; ++i) ga[i] = rd(round, a3[i] > 0.0 ? ga[i] : 0.0);
        conv3x3_wgrad(B, H, W, C_HID, C_HID, a2, ga, grad + off[4], grad + off[5]);
        conv3x3_dgrad(B, H, W, C_HID, C_HID, ga, w + off[4], gb);
        for (size_t i = 0; i < P * C_HID; ++i) gb[i] = rd(round, a2[i] > 0.0 ? gb[i] : 0.0);
        conv3x3_wgrad(B, H, W, C_HID, C_HID, a1, gb, grad + off[2], grad + off[3]);
        conv3x3_dgrad(B, H, W, C_HID, C_HID, gb, w + off[2], ga);
        for (size_t i = 0; i < P * C_HID; ++i) ga[i] = rd(round, a1[i] > 0.0 ? ga[i] : 0.0);
        conv3x3_wgrad(B, H, W, 3, C_HID, a0, ga, grad + off[0], grad + off[1]);
        free(gb);
        free(ga);
        free(g);
    }
    free(d);
    free(a3);
    free(a2);
    free(a1);
    free(a0);
    free(w);
    return loss;
}

/* One Adam step on FP64 master parameters (Kingma & Ba, bias-corrected). */
void orc_adam(int64_t n, double* p, double* m, double* v, const double* g, double lr, double b1,
              double b2, double eps, int t)
{
    const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
