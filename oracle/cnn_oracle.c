/*
 * CPU oracle of the learned coarse-grid closure -- TEST INFRASTRUCTURE ONLY.
 *
 * A small convolutional network corrects the velocity of a coarse MDF-FDLBM
 * run (a project addition; the paper has no learned component).  This file is
 * the plain definition: direct sums in FP64, nothing blocked or reordered.
 *
 * Network: x = (u, v) / s_in on an H x W periodic grid (channels last);
 *   z_l = conv3x3(a_{l-1}; W_l) + b_l,  a_l = max(z_l, 0) for l = 1, 2, 3,
 *   y = z_4 (2 channels); the correction is (du, dv) = s_out * y.
 * Channels 2 -> 32 -> 32 -> 32 -> 2.  conv3x3 on a periodic grid:
 *   z[y][x][co] = b[co] + sum_{t, ci} W[t][ci][co] a[(y + t/3 - 1) mod H][(x + t%3 - 1) mod W][ci].
 * Parameters (one flat vector): for l = 1..4, W_l[9][cin][cout] then b_l[cout].
 * Loss: L = sum (y - target)^2 / (B H W 2).
 *
 * BF16: round-to-nearest-even of an FP32 value to 8 significant bits
 * (written from the format's definition); the layer check feeds identically
 * rounded operands to this oracle and to the GPU.
 */
#include "cnn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const int CH[5] = {2, 32, 32, 32, 2};

int32_t cnn_param_count(void)
{
    int32_t n = 0;
    for (int l = 0; l < 4; ++l) n += 9 * CH[l] * CH[l + 1] + CH[l + 1];
    return n;
}

/* offset of layer l's weights (l = 0..3) in the flat parameter vector */
static int32_t w_off(int l)
{
    int32_t n = 0;
    for (int k = 0; k < l; ++k) n += 9 * CH[k] * CH[k + 1] + CH[k + 1];
    return n;
}

double cnn_bf16(double v)
{
    /* FP32 first (the GPU holds FP32 values), then keep the top 16 bits of the
       binary32 pattern with round-to-nearest-even on the dropped 16 bits. */
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan unchanged */
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* one periodic 3x3 convolution, channels last; w[9][cin][cout] */
void cnn_conv3x3(int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout, const double* a, const double* w,
                 const double* bias, double* z)
{
    for (int b = 0; b < B; ++b)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                for (int co = 0; co < cout; ++co) {
                    double s = bias ? bias[co] : 0.0;
                    for (int t = 0; t < 9; ++t) {
                        const int yy = (y + t / 3 - 1 + H) % H, xx = (x + t % 3 - 1 + W) % W;
                        const double* ap = a + (((size_t)b * H + yy) * W + xx) * cin;
                        for (int ci = 0; ci < cin; ++ci) s += w[((size_t)t * cin + ci) * cout + co] * ap[ci];
                    }
                    z[(((size_t)b * H + y) * W + x) * cout + co] = s;
                }
}

/* activations of a forward pass: a[0] = x, z[l], a[l] = relu(z[l]) (l = 1..3), z[4] = y */
typedef struct {
    double* a[4];
    double* z[5];
} acts_t;

static void forward_all(const double* params, int32_t B, int32_t H, int32_t W, const double* x, acts_t* A)
{
    const size_t P = (size_t)B * H * W;
    A->a[0] = (double*)malloc(sizeof(double) * P * CH[0]);
    memcpy(A->a[0], x, sizeof(double) * P * CH[0]);
    for (int l = 1; l <= 4; ++l) {
        A->z[l] = (double*)malloc(sizeof(double) * P * CH[l]);
        const double* w = params + w_off(l - 1);
        const double* b = w + 9 * CH[l - 1] * CH[l];
        cnn_conv3x3(B, H, W, CH[l - 1], CH[l], A->a[l - 1], w, b, A->z[l]);
        if (l < 4) {
            A->a[l] = (double*)malloc(sizeof(double) * P * CH[l]);
            for (size_t i = 0; i < P * CH[l]; ++i) A->a[l][i] = A->z[l][i] > 0.0 ? A->z[l][i] : 0.0;
        }
    }
}

static void free_acts(acts_t* A)
{
    for (int l = 0; l < 4; ++l) free(A->a[l]);
    for (int l = 1; l <= 4; ++l) free(A->z[l]);
}

void cnn_forward(const double* params, int32_t B, int32_t H, int32_t W, const double* x, double* y)
{
    acts_t A;
    memset(&A, 0, sizeof A);
    forward_all(params, B, H, W, x, &A);
    memcpy(y, A.z[4], sizeof(double) * (size_t)B * H * W * CH[4]);
    free_acts(&A);
}

/* Loss and its gradient with respect to every parameter, by the chain rule:
 *   dL/dz4 = 2 (y - target) / (B H W 2);
 *   dL/dW_l[t][ci][co] = sum_p a_{l-1}[p + o_t][ci] dL/dz_l[p][co],  dL/db_l[co] = sum_p dL/dz_l[p][co];
 *   dL/da_{l-1}[q][ci] = sum_{t, co} W_l[t][ci][co] dL/dz_l[q - o_t][co];
 *   dL/dz_{l-1} = dL/da_{l-1} * [z_{l-1} > 0]. */
double cnn_loss_grad(const double* params, int32_t B, int32_t H, int32_t W, const double* x, const double* target,
                     double* grad)
{
    const size_t P = (size_t)B * H * W;
    acts_t A;
    memset(&A, 0, sizeof A);
    forward_all(params, B, H, W, x, &A);
    double loss = 0.0;
    const double inv = 1.0 / ((double)P * CH[4]);
    double* g = (double*)malloc(sizeof(double) * P * CH[4]);
    for (size_t i = 0; i < P * CH[4]; ++i) {
        const double d = A.z[4][i] - target[i];
        loss += d * d;
        g[i] = 2.0 * d * inv;
    }
    loss *= inv;
    memset(grad, 0, sizeof(double) * (size_t)cnn_param_count());
    for (int l = 4; l >= 1; --l) {
        const int cin = CH[l - 1], cout = CH[l];
        double* gw = grad + w_off(l - 1);
        double* gb = gw + 9 * cin * cout;
        const double* w = params + w_off(l - 1);
        const double* a = A.a[l - 1];
        for (int b = 0; b < B; ++b)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    const double* gp = g + (((size_t)b * H + y) * W + x) * cout;
                    for (int co = 0; co < cout; ++co) gb[co] += gp[co];
                    for (int t = 0; t < 9; ++t) {
                        const int yy = (y + t / 3 - 1 + H) % H, xx = (x + t % 3 - 1 + W) % W;
                        const double* ap = a + (((size_t)b * H + yy) * W + xx) * cin;
                        for (int ci = 0; ci < cin; ++ci)
                            for (int co = 0; co < cout; ++co) gw[((size_t)t * cin + ci) * cout + co] += ap[ci] * gp[co];
                    }
                }
        if (l == 1) break;
        /* gradient with respect to the layer input, then through the ReLU */
        double* ga = (double*)calloc(P * cin, sizeof(double));
        for (int b = 0; b < B; ++b)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    const double* gp = g + (((size_t)b * H + y) * W + x) * cout;
                    for (int t = 0; t < 9; ++t) {
                        const int yy = (y + t / 3 - 1 + H) % H, xx = (x + t % 3 - 1 + W) % W;
                        double* gap = ga + (((size_t)b * H + yy) * W + xx) * cin;
                        for (int ci = 0; ci < cin; ++ci) {
                            double s = 0.0;
                            for (int co = 0; co < cout; ++co) s += w[((size_t)t * cin + ci) * cout + co] * gp[co];
                            gap[ci] += s;
                        }
                    }
                }
        for (size_t i = 0; i < P * cin; ++i) ga[i] = A.z[l - 1][i] > 0.0 ? ga[i] : 0.0;
        free(g);
        g = ga;
    }
    free(g);
    free_acts(&A);
    return loss;
}

/* f_hat += f^eq(u + du, v + dv, P) - f^eq(u, v, P) at every node (eq. 2.2.5 is
 * linear in u_a for fixed P and quadratic through the flux; both terms are
 * evaluated as written).  f is the dense [10][ny][nx] state, q = alpha*5 + j. */
void cnn_apply_correction(int32_t nx, int32_t ny, double c, const double* du, const double* dv, double* f)
{
    const double w = 0.2, cs2 = 0.4 * c * c, kf = w * c / cs2;
    const size_t n = (size_t)nx * ny;
    for (size_t i = 0; i < n; ++i) {
        double phi[10];
        for (int q = 0; q < 10; ++q) phi[q] = f[q * n + i];
        const double u = phi[0] + phi[1] + phi[2] + phi[3] + phi[4];
        const double v = phi[5] + phi[6] + phi[7] + phi[8] + phi[9];
        const double P = 0.5 * (c * (phi[1] - phi[3] + phi[7] - phi[9]) - (u * u + v * v));
        double e0[10], e1[10];
        for (int k = 0; k < 2; ++k) {
            const double uu = k ? u + du[i] : u, vv = k ? v + dv[i] : v;
            double* e = k ? e1 : e0;
            const double fxu = uu * uu + P, fyu = uu * vv, fxv = vv * uu, fyv = vv * vv + P;
            e[0] = w * uu;
            e[1] = w * uu + kf * fxu;
            e[2] = w * uu + kf * fyu;
            e[3] = w * uu - kf * fxu;
            e[4] = w * uu - kf * fyu;
            e[5] = w * vv;
            e[6] = w * vv + kf * fxv;
            e[7] = w * vv + kf * fyv;
            e[8] = w * vv - kf * fxv;
            e[9] = w * vv - kf * fyv;
        }
        for (int q = 0; q < 10; ++q) f[q * n + i] = phi[q] + (e1[q] - e0[q]);
    }
}
