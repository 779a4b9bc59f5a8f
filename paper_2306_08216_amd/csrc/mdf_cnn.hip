// Learned coarse-grid closure (a project addition): a four-layer periodic
// 3x3 convolutional network, 2 -> 32 -> 32 -> 32 -> 2 channels, ReLU after the
// first three layers, evaluated and trained on gfx950 matrix cores (BF16
// operands, FP32 accumulation), and the step that applies its velocity
// correction to an MDF-FDLBM state through the equilibrium (eq. 2.2.5).
//
// Convolutions are implicit GEMMs on v_mfma_f32_32x32x8_bf16: one wave
// computes 32 pixels of one image row x 32 output channels, K = 9 taps x the
// padded input channels.  Activations are channels-last (NHWC) BF16; packed
// weights are [tap][out channel][in channel] BF16 so that a lane's four K
// values are 8 contiguous bytes for both operands.  The backward pass uses
// the same kernel for the data gradient (taps mirrored, channels transposed)
// and a second MFMA GEMM over pixels for the weight gradient, reduced in a
// fixed order (no atomics: results are bitwise reproducible).
#include <mutex>

#include "mdf_device.hpp"
#include "mdf_internal.hpp"

namespace mdf {

namespace {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kCh[5] = {2, 32, 32, 32, 2};

// FP32 -> BF16, round to nearest, ties to even; NaN stays NaN.
__device__ __forceinline__ unsigned short to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

struct ConvArgs {
    const unsigned short* in;   // [P][cin_pad] BF16, P = B*H*W, channels last
    int cin_pad;                // 8 or 32
    const unsigned short* wp;   // [9][32][cin_pad] BF16
    const float* bias;          // [cout] or null
    const float* zmask;         // [P][32]: multiply by (zmask > 0) (ReLU derivative), or null
    int relu;                   // max(., 0) before the BF16 output
    int cout;                   // output channels written (the rest of the 32 are zero)
    float* out_f32;             // [P][f32_stride] or null
    int f32_stride;
    unsigned short* out_bf16;   // [P][32] or null
    int B, H, W;                // W a multiple of 32
};

// CIN_PAD (the input channel stride, 8 or 32) is a template argument so that
// every operand of the 9 taps is loaded into registers before the MFMA chain
// consumes them, instead of each MFMA waiting for its own two loads (the
// layers are latency-bound at the closure's grid sizes).  The MFMAs
// accumulate in the same order as a tap-by-tap loop.
template <int CIN_PAD>
__global__ __launch_bounds__(64) void k_conv(ConvArgs A)
{
    const int tiles_x = A.W / 32;
    const int tile = blockIdx.x;
    const int x0 = (tile % tiles_x) * 32;
    const int row = tile / tiles_x;   // b * H + y
    const int y = row % A.H, b = row / A.H;
    const int lane = threadIdx.x, i = lane & 31, kh = lane >> 5;
    constexpr int NB = CIN_PAD / 8;
    bf4 av[9][NB], bv[9][NB];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = (y + t / 3 - 1 + A.H) % A.H;
        const int xx = (x0 + i + t % 3 - 1 + A.W) % A.W;
        const unsigned short* ap = A.in + ((size_t)(b * A.H + yy) * A.W + xx) * CIN_PAD + 4 * kh;
        const unsigned short* wp = A.wp + ((size_t)t * 32 + i) * CIN_PAD + 4 * kh;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            av[t][c] = *reinterpret_cast<const bf4*>(ap + 8 * c);
            bv[t][c] = *reinterpret_cast<const bf4*>(wp + 8 * c);
        }
    }
    f32x16 acc = {};
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av[t][c], bv[t][c], acc, 0, 0, 0);
    // lane holds D[m][co] for co = lane % 32, m = 8 (r / 4) + 4 (lane / 32) + r % 4
    const int co = i;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = 8 * (r >> 2) + 4 * kh + (r & 3);
        const size_t p = (size_t)row * A.W + x0 + m;
        float v = acc[r];
        if (A.bias && co < A.cout) v += A.bias[co];
        if (A.zmask) v = A.zmask[p * 32 + co] > 0.0f ? v : 0.0f;
        if (A.out_f32 && co < A.cout) A.out_f32[p * A.f32_stride + co] = v;
        if (A.out_bf16) A.out_bf16[p * 32 + co] = co < A.cout ? to_bf16(A.relu ? fmaxf(v, 0.0f) : v) : 0;
    }
}

// Packed BF16 weights of one layer (W[t][ci][co] FP32 in the flat parameters):
//   wf[t][co][ci]  (cin_pad wide) for the forward convolution,
//   wb[t][ci][co]  (cout_pad wide) = W[8 - t][ci][co] for the data gradient,
// zero outside the layer's channels.
struct PackArgs {
    int woff[4], cin[4], cout[4], cin_pad[4], cout_pad[4];
    unsigned short* wf[4];
    unsigned short* wb[4];
};

__global__ void k_pack_weights(const float* __restrict__ params, PackArgs P)
{
    const int l = blockIdx.y;
    const int cin = P.cin[l], cout = P.cout[l], cin_pad = P.cin_pad[l], cout_pad = P.cout_pad[l];
    unsigned short* __restrict__ wf = P.wf[l];
    unsigned short* __restrict__ wb = P.wb[l];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const float* W = params + P.woff[l];
    if (e < 9 * 32 * cin_pad) {
        const int ci = e % cin_pad, co = (e / cin_pad) % 32, t = e / (32 * cin_pad);
        wf[e] = (co < cout && ci < cin) ? to_bf16(W[(t * cin + ci) * cout + co]) : 0;
    }
    if (e < 9 * 32 * cout_pad) {
        const int co = e % cout_pad, ci = (e / cout_pad) % 32, t = e / (32 * cout_pad);
        wb[e] = (ci < cin && co < cout) ? to_bf16(W[((8 - t) * cin + ci) * cout + co]) : 0;
    }
}

// x = in_scale * (u, v), BF16, 8 channels (6 zero)
__global__ void k_pack_input(const double* __restrict__ uv, int B, int H, int W, double in_scale,
                             unsigned short* __restrict__ x)
{
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t HW = (size_t)H * W;
    if (p >= (size_t)B * HW) return;
    const size_t b = p / HW, s = p % HW;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        x[p * 8 + c] = c < 2 ? to_bf16((float)(in_scale * uv[(b * 2 + c) * HW + s])) : 0;
}

__global__ void k_unpack_output(const float* __restrict__ y, int B, int H, int W, double out_scale,
                                double* __restrict__ duv)
{
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t HW = (size_t)H * W;
    if (p >= (size_t)B * HW) return;
    const size_t b = p / HW, s = p % HW;
    duv[(b * 2 + 0) * HW + s] = out_scale * (double)y[p * 2 + 0];
    duv[(b * 2 + 1) * HW + s] = out_scale * (double)y[p * 2 + 1];
}

// dL/dy for L = mean over pixels and both channels of (y - target/out_scale)^2;
// g as FP32 and BF16 with 32 channels (30 zero); per-block sums of squares.
constexpr int kRedBlock = 256;
__global__ __launch_bounds__(kRedBlock) void k_loss_grad(const float* __restrict__ y, const double* __restrict__ duv_t,
                                                         int B, int H, int W, double out_scale,
                                                         float* __restrict__ g32, unsigned short* __restrict__ g16,
                                                         double* __restrict__ part)
{
    __shared__ double red[kRedBlock];
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t HW = (size_t)H * W, P = (size_t)B * HW;
    double sq = 0.0;
    if (p < P) {
        const size_t b = p / HW, s = p % HW;
        const double inv = 1.0 / (2.0 * (double)P);
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            float gv = 0.0f;
            if (c < 2) {
                const double d = (double)y[p * 2 + c] - duv_t[(b * 2 + c) * HW + s] / out_scale;
                sq += d * d;
                gv = (float)(2.0 * d * inv);
            }
            g32[p * 32 + c] = gv;
            g16[p * 32 + c] = to_bf16(gv);
        }
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int o = kRedBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kRedBlock) void k_sum_final(const double* __restrict__ part, int n, double scale,
                                                         double* __restrict__ out)
{
    __shared__ double red[kRedBlock];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kRedBlock) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kRedBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Partial weight gradient of one tap over one image row (W pixels):
//   part[row][t][ci][co] = sum_x a[(y + dy, x + dx)][ci] g[(y, x)][co]
// as an MFMA GEMM with M = ci, N = co, K = pixels.
__global__ __launch_bounds__(64) void k_wgrad_part(const unsigned short* __restrict__ a, int cin_pad,
                                                   const unsigned short* __restrict__ g, int B, int H, int W,
                                                   float* __restrict__ part)
{
    const int row = blockIdx.x, t = blockIdx.y;
    const int y = row % H, b = row / H;
    const int yy = (y + t / 3 - 1 + H) % H, dx = t % 3 - 1;
    const int lane = threadIdx.x, i = lane & 31, kh = lane >> 5;
    const unsigned short* arow = a + (size_t)(b * H + yy) * W * cin_pad;
    const unsigned short* grow = g + (size_t)row * W * 32;
    f32x16 acc = {};
    for (int s = 0; s < W; s += 8) {
        bf4 av, bv;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int x = s + 4 * kh + q;
            const int xa = (x + dx + W) % W;
            av[q] = i < cin_pad ? (short)arow[(size_t)xa * cin_pad + i] : (short)0;
            bv[q] = (short)grow[(size_t)x * 32 + i];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
    float* out = part + ((size_t)row * 9 + t) * 1024;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = 8 * (r >> 2) + 4 * kh + (r & 3);
        out[m * 32 + i] = acc[r];
    }
}

// grad W[t][ci][co] = sum over rows of the partials, in row order
__global__ void k_wgrad_reduce(const float* __restrict__ part, int rows, int cin, int cout, float* __restrict__ gw)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * cin * cout) return;
    const int co = e % cout, ci = (e / cout) % cin, t = e / (cin * cout);
    float s = 0.0f;
    for (int r = 0; r < rows; ++r) s += part[((size_t)r * 9 + t) * 1024 + ci * 32 + co];
    gw[e] = s;
}

// grad b[co] = sum_p g[p][co]
__global__ __launch_bounds__(kRedBlock) void k_bgrad(const float* __restrict__ g32, size_t P, float* __restrict__ gb)
{
    __shared__ float red[kRedBlock];
    const int co = blockIdx.x;
    float s = 0.0f;
    for (size_t p = threadIdx.x; p < P; p += kRedBlock) s += g32[p * 32 + co];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kRedBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) gb[co] = red[0];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- correction of an MDF state -------------------------------------------

// node moments (pressure identity) of the row-split state
__device__ __forceinline__ void node_uvp(const StepConsts& K, const double* f, int x, int y, double* phi, double& u,
                                         double& v, double& P)
{
    load_node(f, K.pitch, x, y, phi);
    node_moments(phi, K.c, u, v, P);
}

// per block, for the current field (u, v) and the corrected field (u + du, v + dv):
// sums of |u|^2 / 2 and maxima of |div_FD u| (periodic central differences)
constexpr int kGuardBlock = 256;
__global__ __launch_bounds__(kGuardBlock) void k_closure_guard(StepConsts K, const double* __restrict__ f,
                                                               const double* __restrict__ du,
                                                               const double* __restrict__ dv, double hx, double hy,
                                                               double* __restrict__ part)
{
    __shared__ double r[4][kGuardBlock];
    double kp = 0.0, dp = 0.0, kc = 0.0, dc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < K.nx * K.ny; i += gridDim.x * blockDim.x) {
        const int x = i % K.nx, y = i / K.nx;
        double phi[10], P;
        // plain and corrected velocity at a (wrapped) node
        auto vel = [&](int xx, int yy, double* w) {
            xx = (xx + K.nx) % K.nx;
            yy = (yy + K.ny) % K.ny;
            node_uvp(K, f, xx, yy, phi, w[0], w[1], P);
            const size_t j = (size_t)yy * K.nx + xx;
            w[2] = w[0] + (du ? du[j] : 0.0);
            w[3] = w[1] + (dv ? dv[j] : 0.0);
        };
        double c[4], e[4], wv[4], n[4], sv[4];
        vel(x, y, c);
        vel(x + 1, y, e);
        vel(x - 1, y, wv);
        vel(x, y + 1, n);
        vel(x, y - 1, sv);
        kp += 0.5 * (c[0] * c[0] + c[1] * c[1]);
        kc += 0.5 * (c[2] * c[2] + c[3] * c[3]);
        dp = fmax(dp, fabs((e[0] - wv[0]) / (2.0 * hx) + (n[1] - sv[1]) / (2.0 * hy)));
        dc = fmax(dc, fabs((e[2] - wv[2]) / (2.0 * hx) + (n[3] - sv[3]) / (2.0 * hy)));
    }
    r[0][threadIdx.x] = kp;
    r[1][threadIdx.x] = dp;
    r[2][threadIdx.x] = kc;
    r[3][threadIdx.x] = dc;
    __syncthreads();
    for (int o = kGuardBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r[0][threadIdx.x] += r[0][threadIdx.x + o];
            r[1][threadIdx.x] = fmax(r[1][threadIdx.x], r[1][threadIdx.x + o]);
            r[2][threadIdx.x] += r[2][threadIdx.x + o];
            r[3][threadIdx.x] = fmax(r[3][threadIdx.x], r[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = r[threadIdx.x][0];
}

__global__ __launch_bounds__(kGuardBlock) void k_closure_guard_final(const double* __restrict__ part, int n,
                                                                     double* __restrict__ out4)
{
    __shared__ double r[4][kGuardBlock];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += kGuardBlock) {
        a[0] += part[4 * i];
        a[1] = fmax(a[1], part[4 * i + 1]);
        a[2] += part[4 * i + 2];
        a[3] = fmax(a[3], part[4 * i + 3]);
    }
    for (int q = 0; q < 4; ++q) r[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int o = kGuardBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r[0][threadIdx.x] += r[0][threadIdx.x + o];
            r[1][threadIdx.x] = fmax(r[1][threadIdx.x], r[1][threadIdx.x + o]);
            r[2][threadIdx.x] += r[2][threadIdx.x + o];
            r[3][threadIdx.x] = fmax(r[3][threadIdx.x], r[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) out4[threadIdx.x] = r[threadIdx.x][0];
}

// f_hat += f^eq(u + du, v + dv, P) - f^eq(u, v, P) at every node
// Guard decision on the device: state = {ke_ref, fall-backs, flag, windows}.
// The correction is accepted when the corrected field's kinetic energy does
// not exceed ke_ref and its largest divergence is at most div_factor times the
// current field's (both finite); ke_ref becomes the energy of the field the
// window leaves.  reset: ke_ref = the current field's energy, counters zero.
__global__ void k_closure_decide(const double* __restrict__ out4, double* __restrict__ state, double div_factor,
                                 int reset)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (reset) {
        state[0] = out4[0];
        state[1] = 0.0;
        state[2] = 0.0;
        state[3] = 0.0;
        return;
    }
    const bool ok = isfinite(out4[2]) && isfinite(out4[3]) && out4[2] <= state[0] && out4[3] <= div_factor * out4[1];
    state[0] = ok ? out4[2] : out4[0];
    state[1] += ok ? 0.0 : 1.0;
    state[2] = ok ? 1.0 : 0.0;
    state[3] += 1.0;
}

__global__ void k_closure_apply(StepConsts K, double* __restrict__ f, const double* __restrict__ du,
                                const double* __restrict__ dv, const double* __restrict__ flag)
{
    if (flag && *flag == 0.0) return;   // the guard refused this window's correction
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K.nx * K.ny) return;
    const int x = i % K.nx, y = i / K.nx;
    double phi[10], u, v, P, e0[10], e1[10];
    node_uvp(K, f, x, y, phi, u, v, P);
    equilibrium(u, v, P, K, e0);
    equilibrium(u + du[i], v + dv[i], P, K, e1);
#pragma unroll
    for (int q = 0; q < 10; ++q) phi[q] += e1[q] - e0[q];
    store_node(f, K.pitch, x, y, phi);
}

// ---- workspace -------------------------------------------------------------

struct CnnLayout {
    size_t x, z[5], a[4], g32[5], g16[5], wf[4], wb[4], part, red, lossv, total;
    size_t P, rows;
};

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

// Workspace layout for batch B of H x W fields; without `training` only the
// forward pass's buffers (no gradients, partials or loss).
CnnLayout cnn_layout(int B, int H, int W, bool training = true)
{
    CnnLayout L{};
    L.P = (size_t)B * H * W;
    L.rows = (size_t)B * H;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += al(bytes);
        return r;
    };
    L.x = take(L.P * 8 * 2);
    L.a[0] = L.x;
    for (int l = 1; l <= 3; ++l) {
        L.z[l] = take(L.P * 32 * 4);
        L.a[l] = take(L.P * 32 * 2);
    }
    L.z[4] = take(L.P * 2 * 4);
    if (!training) {
        for (int l = 0; l < 4; ++l) {
            L.wf[l] = take(9 * 32 * 32 * 2);
            L.wb[l] = take(9 * 32 * 32 * 2);
        }
        L.total = o;
        return L;
    }
    // gradient of the loss at each layer output z_l (l = 1..4), 32 channels wide
    for (int l = 1; l <= 4; ++l) {
        L.g32[l] = take(L.P * 32 * 4);
        L.g16[l] = take(L.P * 32 * 2);
    }
    for (int l = 0; l < 4; ++l) {
        L.wf[l] = take(9 * 32 * 32 * 2);
        L.wb[l] = take(9 * 32 * 32 * 2);
    }
    L.part = take(L.rows * 9 * 1024 * 4);
    L.red = take(((L.P + kRedBlock - 1) / kRedBlock + 1) * 8);
    L.lossv = take(8);
    L.total = o;
    return L;
}

int cin_pad_of(int l) { return l == 0 ? 8 : 32; }    // input channel stride of layer l (0-based)
int cout_pad_of(int) { return 32; }   // gradients are stored 32 channels wide (zero padded)

int woff_of(int l)
{
    int o = 0;
    for (int k = 0; k < l; ++k) o += 9 * kCh[k] * kCh[k + 1] + kCh[k + 1];
    return o;
}

hipError_t pack_all(const CnnLayout& L, char* ws, const float* params, hipStream_t s)
{
    // the four layers in one launch (blockIdx.y = layer)
    PackArgs A{};
    for (int l = 0; l < 4; ++l) {
        A.woff[l] = woff_of(l);
        A.cin[l] = kCh[l];
        A.cout[l] = kCh[l + 1];
        A.cin_pad[l] = cin_pad_of(l);
        A.cout_pad[l] = cout_pad_of(l);
        A.wf[l] = (unsigned short*)(ws + L.wf[l]);
        A.wb[l] = (unsigned short*)(ws + L.wb[l]);
    }
    const int n = 9 * 32 * 32;
    hipLaunchKernelGGL(k_pack_weights, dim3((n + 255) / 256, 4), dim3(256), 0, s, params, A);
    return hipGetLastError();
}

void launch_conv(const ConvArgs& A, unsigned tiles, hipStream_t s)
{
    if (A.cin_pad == 8)
        hipLaunchKernelGGL(k_conv<8>, dim3(tiles), dim3(64), 0, s, A);
    else
        hipLaunchKernelGGL(k_conv<32>, dim3(tiles), dim3(64), 0, s, A);
}

ConvArgs conv_args(int B, int H, int W)
{
    ConvArgs A{};
    A.B = B;
    A.H = H;
    A.W = W;
    return A;
}

}  // namespace

int32_t cnn_param_count() { return woff_of(4); }

hipError_t cnn_layer_io(const char* ws, int B, int H, int W, int layer, unsigned short* in_bf16, float* z_f32,
                        unsigned short* g_bf16, float* g_f32, hipStream_t s)
{
    if (layer < 1 || layer > 4) return hipErrorInvalidValue;
    const CnnLayout L = cnn_layout(B, H, W);
    const int l = layer - 1;
    hipError_t e = hipSuccess;
    if (in_bf16)
        e = hipMemcpyAsync(in_bf16, ws + L.a[l], L.P * cin_pad_of(l) * 2, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && z_f32)
        e = hipMemcpyAsync(z_f32, ws + L.z[layer], L.P * (layer < 4 ? 32 : 2) * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && g_bf16)
        e = hipMemcpyAsync(g_bf16, ws + L.g16[layer], L.P * 32 * 2, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && g_f32)
        e = hipMemcpyAsync(g_f32, ws + L.g32[layer], L.P * 32 * 4, hipMemcpyDeviceToDevice, s);
    return e;
}

hipError_t cnn_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                    int step, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// at most 2048 blocks (4 partials each): the caller's partial buffer holds 8192 doubles
int closure_guard_blocks(const StepConsts& K)
{
    const int nb = (K.nx * K.ny + kGuardBlock - 1) / kGuardBlock;
    return nb < 2048 ? nb : 2048;
}

hipError_t launch_closure_guard(const StepConsts& K, const double* f, const double* du, const double* dv, double hx,
                                double hy, double* part, double* out4, hipStream_t s)
{
    const int nb = closure_guard_blocks(K);
    hipLaunchKernelGGL(k_closure_guard, dim3(nb), dim3(kGuardBlock), 0, s, K, f, du, dv, hx, hy, part);
    hipLaunchKernelGGL(k_closure_guard_final, dim3(1), dim3(kGuardBlock), 0, s, part, nb, out4);
    return hipGetLastError();
}

hipError_t launch_closure_apply(const StepConsts& K, double* f, const double* du, const double* dv, const double* flag,
                                hipStream_t s)
{
    const int n = K.nx * K.ny;
    hipLaunchKernelGGL(k_closure_apply, dim3((n + 255) / 256), dim3(256), 0, s, K, f, du, dv, flag);
    return hipGetLastError();
}

hipError_t launch_closure_decide(const double* out4, double* state, double div_factor, bool reset, hipStream_t s)
{
    hipLaunchKernelGGL(k_closure_decide, dim3(1), dim3(64), 0, s, out4, state, div_factor, reset ? 1 : 0);
    return hipGetLastError();
}

size_t cnn_workspace_size(int B, int H, int W) { return cnn_layout(B, H, W).total; }

namespace {

hipError_t forward_at(const CnnLayout& L, char* ws, const float* params, int B, int H, int W, const double* uv,
                      double in_scale, double out_scale, double* duv, hipStream_t s)
{
    hipError_t e = pack_all(L, ws, params, s);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((L.P + 255) / 256);
    hipLaunchKernelGGL(k_pack_input, dim3(nb), dim3(256), 0, s, uv, B, H, W, in_scale, (unsigned short*)(ws + L.x));
    const unsigned tiles = (unsigned)(L.P / 32);
    for (int l = 0; l < 4; ++l) {
        ConvArgs A = conv_args(B, H, W);
        A.in = (const unsigned short*)(ws + L.a[l]);
        A.cin_pad = cin_pad_of(l);
        A.wp = (const unsigned short*)(ws + L.wf[l]);
        A.bias = params + woff_of(l) + 9 * kCh[l] * kCh[l + 1];
        A.relu = l < 3;
        A.cout = kCh[l + 1];
        A.out_f32 = (float*)(ws + L.z[l + 1]);
        A.f32_stride = l < 3 ? 32 : 2;
        A.out_bf16 = l < 3 ? (unsigned short*)(ws + L.a[l + 1]) : nullptr;
        launch_conv(A, tiles, s);
    }
    hipLaunchKernelGGL(k_unpack_output, dim3(nb), dim3(256), 0, s, (const float*)(ws + L.z[4]), B, H, W, out_scale,
                       duv);
    return hipGetLastError();
}

// Scratch of the forward pass for callers that cannot allocate: a fixed
// device array (one copy per GPU, held until the process ends) sized for the
// inference layout of up to kNoAllocPixels pixels.  Host code never passes
// the array's name to a kernel: it is a host-side stand-in, and its device
// address is looked up once per device with that device current.
constexpr size_t kNoAllocBytes = (size_t)10 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The copy of the device that runs `s` (the current device for the null
// stream); its address is looked up the first time with that device current.
hipError_t scratch_address(hipStream_t s, void** out)
{
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    int dev = cur;
    if (s) {
        hipDevice_t sd = 0;
        e = hipStreamGetDevice(s, &sd);
        if (e != hipSuccess) return e;
        dev = (int)sd;
    }
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

hipError_t cnn_forward(char* ws, const float* params, int B, int H, int W, const double* uv, double in_scale,
                       double out_scale, double* duv, hipStream_t s)
{
    return forward_at(cnn_layout(B, H, W), ws, params, B, H, W, uv, in_scale, out_scale, duv, s);
}

size_t cnn_noalloc_capacity() { return kNoAllocBytes; }

size_t cnn_noalloc_bytes(int B, int H, int W) { return cnn_layout(B, H, W, false).total; }

hipError_t cnn_forward_noalloc(const float* params, int B, int H, int W, const double* uv, double in_scale,
                               double out_scale, double* duv, hipStream_t s)
{
    const CnnLayout L = cnn_layout(B, H, W, false);
    if (L.total > kNoAllocBytes) return hipErrorInvalidValue;
    void* ws = nullptr;
    const hipError_t e = scratch_address(s, &ws);
    if (e != hipSuccess) return e;
    return forward_at(L, (char*)ws, params, B, H, W, uv, in_scale, out_scale, duv, s);
}

hipError_t cnn_backward(char* ws, const float* params, int B, int H, int W, const double* duv_t, double out_scale,
                        float* grad, double* loss_dev, hipStream_t s)
{
    const CnnLayout L = cnn_layout(B, H, W);
    const unsigned nb = (unsigned)((L.P + kRedBlock - 1) / kRedBlock);
    double* red = (double*)(ws + L.red);
    hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(kRedBlock), 0, s, (const float*)(ws + L.z[4]), duv_t, B, H, W,
                       out_scale, (float*)(ws + L.g32[4]), (unsigned short*)(ws + L.g16[4]), red);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kRedBlock), 0, s, red, (int)nb, 1.0 / (2.0 * (double)L.P),
                       loss_dev ? loss_dev : (double*)(ws + L.lossv));
    const unsigned tiles = (unsigned)(L.P / 32);
    for (int l = 3; l >= 0; --l) {
        const int cin = kCh[l], cout = kCh[l + 1];
        const float* g32 = (const float*)(ws + L.g32[l + 1]);
        const unsigned short* g16 = (const unsigned short*)(ws + L.g16[l + 1]);
        float* gw = grad + woff_of(l);
        float* gb = gw + 9 * cin * cout;
        hipLaunchKernelGGL(k_wgrad_part, dim3((unsigned)L.rows, 9), dim3(64), 0, s,
                           (const unsigned short*)(ws + L.a[l]), cin_pad_of(l), g16, B, H, W, (float*)(ws + L.part));
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((9 * cin * cout + 255) / 256), dim3(256), 0, s,
                           (const float*)(ws + L.part), (int)L.rows, cin, cout, gw);
        hipLaunchKernelGGL(k_bgrad, dim3(cout), dim3(kRedBlock), 0, s, g32, L.P, gb);
        if (l == 0) break;
        // data gradient of layer l through the ReLU of layer l-1:
        // dA[q][ci] = sum_{t, co} W[t][ci][co] g[q - o_t][co], masked by z_{l} > 0
        ConvArgs A = conv_args(B, H, W);
        A.in = g16;
        A.cin_pad = cout_pad_of(l);
        A.wp = (const unsigned short*)(ws + L.wb[l]);
        A.zmask = (const float*)(ws + L.z[l]);
        A.cout = cin;
        A.out_f32 = (float*)(ws + L.g32[l]);
        A.f32_stride = 32;
        A.out_bf16 = (unsigned short*)(ws + L.g16[l]);
        launch_conv(A, tiles, s);
    }
    return hipGetLastError();
}

}  // namespace mdf
