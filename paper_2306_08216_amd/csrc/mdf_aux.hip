// Auxiliary kernels: initialisation, wall rule on a stored field, moments,
// local derived quantities, diagnostics reductions, state copies, and the
// tiled time step (Steps (1)-(3) in one kernel, Step (4) in a second, wall
// nodes after each).
#include "mdf_device.hpp"
#include "mdf_internal.hpp"

namespace mdf {

namespace {

__device__ __forceinline__ void load10(const StepConsts& K, const double* f, int x, int y, double* phi)
{
    load_node(f, K.pitch, x, y, phi);
}

__device__ __forceinline__ void store10(const StepConsts& K, double* f, int x, int y, const double* phi)
{
    store_node(f, K.pitch, x, y, phi);
}

// component q (= alpha*5 + j) of node (x, y)
__device__ __forceinline__ double comp(const StepConsts& K, const double* f, int x, int y, int q)
{
    return f[comp_off(K.pitch, x, y, q)];
}

// inward neighbours of a wall node; returns false for interior nodes
__device__ __forceinline__ bool wall_neighbours(const StepConsts& K, int x, int y, int& x1, int& y1, int& x2, int& y2,
                                                double& uw)
{
    int ix = 0, iy = 0;
    if (K.bcx) ix = (x == 0) ? 1 : (x == K.nx - 1 ? -1 : 0);
    if (K.bcy) iy = (y == 0) ? 1 : (y == K.ny - 1 ? -1 : 0);
    if (ix == 0 && iy == 0) return false;
    const bool corner = ix != 0 && iy != 0;
    uw = (K.bcy && y == K.ny - 1 && !corner) ? K.lid_u : 0.0;
    x1 = x + ix;
    y1 = y + iy;
    x2 = x + 2 * ix;
    y2 = y + 2 * iy;
    return true;
}

__global__ void k_init(StepConsts K, const double* __restrict__ u0, const double* __restrict__ v0,
                       const double* __restrict__ p0, double* __restrict__ f)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= K.nx || y >= K.ny) return;
    const long long s = (long long)y * K.nx + x;
    double fe[10];
    equilibrium(u0[s], v0[s], p0[s], K, fe);
    store10(K, f, x, y, fe);
}

__global__ void k_moments(StepConsts K, const double* __restrict__ f, double* __restrict__ u, double* __restrict__ v,
                          double* __restrict__ p)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= K.nx || y >= K.ny) return;
    double phi[10], uu, vv, PP;
    load10(K, f, x, y, phi);
    node_moments(phi, K.c, uu, vv, PP);
    if (K.rsrc) PP += K.r_hat * source_at(K, x, y);
    const long long s = (long long)y * K.nx + x;
    if (u) u[s] = uu;
    if (v) v[s] = vv;
    if (p) p[s] = PP;
}

// Local derived quantities (Sec. 2.4) at node (x, y): out[14] in the list order of mdf.h.
// M(f - f^eq) = M(f_hat - f^eq)/(1 + s dt/2), so eq. 2.4.1 reads
// grad_b u_a = -sum_j c_{j,b} (f_hat - f^eq)_{j,a} / (nu + c_s^2 dt/2).
__device__ __forceinline__ void derived_node(const StepConsts& K, const double* fh, int x, int y, double* out)
{
    double u, v, P, fe[10];
    node_moments(fh, K.c, u, v, P);
    if (K.rsrc) P += K.r_hat * source_at(K, x, y);
    equilibrium(u, v, P, K, fe);
    const double nu = K.pl == PL_NEWTON ? K.nu : powerlaw_nu_sq(K, noneq_shear_sq(fh, fe, K.c), K.theta1);
    const double inv = -K.c / (nu + K.theta1);
    const double ux = inv * ((fh[1] - fe[1]) - (fh[3] - fe[3]));
    const double uy = inv * ((fh[2] - fe[2]) - (fh[4] - fe[4]));
    const double vx = inv * ((fh[6] - fe[6]) - (fh[8] - fe[8]));
    const double vy = inv * ((fh[7] - fe[7]) - (fh[9] - fe[9]));
    const double sxy = 0.5 * (uy + vx);
    out[0] = ux;
    out[1] = uy;
    out[2] = vx;
    out[3] = vy;
    out[4] = ux + vy;
    out[5] = ux;
    out[6] = sxy;
    out[7] = vy;
    out[8] = 2.0 * nu * ux;
    out[9] = 2.0 * nu * sxy;
    out[10] = 2.0 * nu * vy;
    out[11] = 0.5 * (uy - vx);
    out[12] = vx - uy;
    out[13] = nu;
}

__global__ void k_derived(StepConsts K, const double* __restrict__ f, double* __restrict__ out, uint32_t mask)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= K.nx || y >= K.ny) return;
    double fh[10], d[14];
    load10(K, f, x, y, fh);
    derived_node(K, fh, x, y, d);
    const long long n = (long long)K.nx * K.ny, s = (long long)y * K.nx + x;
    int slot = 0;
#pragma unroll
    for (int k = 0; k < 14; ++k)
        if (mask & (1u << k)) out[(slot++) * n + s] = d[k];
}

// ---- diagnostics: per-block partials in fixed order, then one block ----

constexpr int DIAG_BLOCK = 256;

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

__device__ __forceinline__ void block_reduce8(double* vals, double* part)
{
    __shared__ double red[DIAG_BLOCK / 64][8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const bool mx = (k == 4 || k == 5);
        const double r = mx ? wave_max(vals[k]) : wave_sum(vals[k]);
        if (lane == 0) red[wv][k] = r;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const int k = threadIdx.x;
        const bool mx = (k == 4 || k == 5);
        double acc = red[0][k];
        for (int i = 1; i < DIAG_BLOCK / 64; ++i) acc = mx ? fmax(acc, red[i][k]) : acc + red[i][k];
        part[k] = acc;
    }
}

// Tiles of 64 x 16 nodes: the block loads every node of the tile and of a
// one-node halo around it once, keeps (u, v) in LDS, and adds each tile
// node's own terms as it loads it; then the central-difference divergence of
// every non-wall tile node reads its neighbours from LDS.  A block walks its
// tiles in a fixed order and writes 8 partials; the final kernel reduces them
// in order.
constexpr int DT_X = 64, DT_Y = 16, DH_X = DT_X + 2, DH_Y = DT_Y + 2;

__global__ __launch_bounds__(DIAG_BLOCK) void k_diag_partial(StepConsts K, const double* __restrict__ f,
                                                              double* __restrict__ partials)
{
    __shared__ double tu[DH_Y][DH_X], tv[DH_Y][DH_X];
    const int tiles_x = (K.nx + DT_X - 1) / DT_X, tiles = tiles_x * ((K.ny + DT_Y - 1) / DT_Y);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int x0 = (t % tiles_x) * DT_X, y0 = (t / tiles_x) * DT_Y;
        if constexpr (kPoisonLds) {
            for (int c = threadIdx.x; c < DH_X * DH_Y; c += DIAG_BLOCK)
                tu[c / DH_X][c % DH_X] = tv[c / DH_X][c % DH_X] = lds_poison_value();
            __syncthreads();
        }
        for (int c = threadIdx.x; c < DH_X * DH_Y; c += DIAG_BLOCK) {
            const int cy = c / DH_X, cx = c - cy * DH_X;
            int x = x0 - 1 + cx, y = y0 - 1 + cy;
            // wrapped on a periodic axis; beyond a wall (or past the grid) the cell is
            // never read: only wall nodes, which take no divergence, border it
            if (!K.bcx) x = x < 0 ? x + K.nx : (x >= K.nx ? x - K.nx : x);
            if (!K.bcy) y = y < 0 ? y + K.ny : (y >= K.ny ? y - K.ny : y);
            double u = 0.0, v = 0.0;
            if (x >= 0 && x < K.nx && y >= 0 && y < K.ny) {
                double fh[10], P;
                load10(K, f, x, y, fh);
                node_moments(fh, K.c, u, v, P);
                const bool own = cx >= 1 && cx <= DT_X && cy >= 1 && cy <= DT_Y && x0 - 1 + cx < K.nx &&
                                 y0 - 1 + cy < K.ny;
                if (own) {
                    double d[14];
                    derived_node(K, fh, x, y, d);
                    double dA = 1.0 / (gx_at(K, x) * gy_at(K, y));
                    const size_t nn = (size_t)K.nx * K.ny, ii = (size_t)y * K.nx + x;
                    if (K.met) dA = 1.0 / fabs(K.met[ii] * K.met[3 * nn + ii] - K.met[nn + ii] * K.met[2 * nn + ii]);
                    acc[0] += u;
                    acc[1] += v;
                    acc[2] += 0.5 * (u * u + v * v) * dA;
                    acc[3] += 0.5 * d[12] * d[12] * dA;
                    acc[4] = fmax(acc[4], sqrt(u * u + v * v));
                    int bad = 0;
#pragma unroll
                    for (int k = 0; k < 10; ++k) bad += isfinite(fh[k]) ? 0 : 1;
                    acc[6] += (double)bad;
                    acc[7] += dA;
                }
            }
            tu[cy][cx] = u;
            tv[cy][cx] = v;
        }
        __syncthreads();
        for (int c = threadIdx.x; c < DT_X * DT_Y; c += DIAG_BLOCK) {
            const int ly = c / DT_X, lx = c - ly * DT_X;
            const int x = x0 + lx, y = y0 + ly;
            if (x >= K.nx || y >= K.ny || is_wall(K, x, y)) continue;
            const int cx = lx + 1, cy = ly + 1;
            const double ue = tu[cy][cx + 1], uw = tu[cy][cx - 1], un = tu[cy + 1][cx], us = tu[cy - 1][cx];
            const double ve = tv[cy][cx + 1], vw = tv[cy][cx - 1], vn = tv[cy + 1][cx], vs = tv[cy - 1][cx];
            double div = (ue - uw) * gx_at(K, x) * 0.5 + (vn - vs) * gy_at(K, y) * 0.5;
            if (K.met) {
                // chain rule: du/dx + dv/dy from both index differences of u and v
                const size_t nn = (size_t)K.nx * K.ny, ii = (size_t)y * K.nx + x;
                div = K.met[ii] * (ue - uw) * 0.5 + K.met[2 * nn + ii] * (un - us) * 0.5 +
                      K.met[nn + ii] * (ve - vw) * 0.5 + K.met[3 * nn + ii] * (vn - vs) * 0.5;
            }
            acc[5] = fmax(acc[5], fabs(div));
        }
        __syncthreads();
    }
    block_reduce8(acc, partials + 8 * blockIdx.x);
}

__global__ __launch_bounds__(DIAG_BLOCK) void k_diag_final(const double* __restrict__ partials, int nblocks,
                                                            double* __restrict__ out)
{
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += DIAG_BLOCK) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double v = partials[8 * b + k];
            acc[k] = (k == 4 || k == 5) ? fmax(acc[k], v) : acc[k] + v;
        }
    }
    block_reduce8(acc, out);
}

// copy between the pitched state and a dense 10 x ny x nx array
__global__ void k_pack(StepConsts K, const double* __restrict__ f, double* __restrict__ dense)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= K.nx || y >= K.ny) return;
    const long long n = (long long)K.nx * K.ny, s = (long long)y * K.nx + x;
#pragma unroll
    for (int k = 0; k < 10; ++k) dense[k * n + s] = comp(K, f, x, y, k);
}

__global__ void k_unpack(StepConsts K, const double* __restrict__ dense, double* __restrict__ f)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= K.nx || y >= K.ny) return;
    const long long n = (long long)K.nx * K.ny, s = (long long)y * K.nx + x;
    double phi[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) phi[k] = dense[k * n + s];
    store_node(f, K.pitch, x, y, phi);
}

// wall nodes of the perimeter: rows y = 0, ny-1 (y walls), then columns
// x = 0, nx-1 (x walls) without the corners the rows already hold
__device__ __forceinline__ bool perimeter_node(const StepConsts& K, int i, int& x, int& y)
{
    const int nrow = K.bcy ? 2 * K.nx : 0;
    if (i < nrow) {
        x = i % K.nx;
        y = i < K.nx ? 0 : K.ny - 1;
        return true;
    }
    i -= nrow;
    const int ncol = K.bcy ? K.ny - 2 : K.ny;
    if (K.bcx && i < 2 * ncol) {
        y = (K.bcy ? 1 : 0) + i % ncol;
        x = i < ncol ? 0 : K.nx - 1;
        return true;
    }
    return false;
}

inline int perimeter_count(const StepConsts& K)
{
    return (K.bcy ? 2 * K.nx : 0) + (K.bcx ? 2 * (K.bcy ? K.ny - 2 : K.ny) : 0);
}

// ---- tiled step ----

// pressure offset of a stored form with coefficient r at node (x, y): SRC only
template <bool SRC>
__device__ __forceinline__ double src_dp(const StepConsts& K, double r, int x, int y)
{
    if constexpr (SRC) return r * source_at(K, x, y);
    return 0.0;
}

// Wall nodes of a field the tiled pass has just written at every interior
// node (f(t+h) after pass B, f_hat(t+dt) after pass C): the wall rule from the
// two inward neighbours, which are interior nodes, as the method applies it
// after each sub-step.  r is the pressure offset per unit source of the
// field's stored form.  One thread per perimeter wall node.
template <bool SRC>
__global__ __launch_bounds__(256) void k_perimeter_wall(StepConsts K, double* __restrict__ f, double r)
{
    int x, y;
    if (!perimeter_node(K, (int)(blockIdx.x * blockDim.x + threadIdx.x), x, y)) return;
    int x1, y1, x2, y2;
    double uw = 0.0, p1[10], p2[10], out[10];
    if (!wall_neighbours(K, x, y, x1, y1, x2, y2, uw)) return;
    load10(K, f, x1, y1, p1);
    load10(K, f, x2, y2, p2);
    wall_extrapolate<SRC>(K, p1, p2, uw, out, src_dp<SRC>(K, r, x1, y1), src_dp<SRC>(K, r, x2, y2));
    store10(K, f, x, y, out);
}

// ---- tiled sub-steps (interior nodes) ----
// A 64 x 8 tile of nodes stages the moving components of its input field with a halo of 2 in LDS, so
// each stencil value is loaded from memory once per tile instead of once per
// use; the stencil then reads LDS.  Wall nodes are set afterwards from the
// written interior (k_perimeter_wall).  The half step computes its input,
// f_bar^+, while it fills the tile (Step (1) at every tile and halo node,
// from f_hat), so f_bar^+ never goes to memory.
constexpr int TB_X = 64, TB_Y = 8, TB_HALO = 2;
constexpr int TS_X = TB_X + 2 * TB_HALO, TS_Y = TB_Y + 2 * TB_HALO;

// All 10 components of node (x, y) of a field for the tile, node(x, y, phi)
// giving them at a grid node: wrapped on a periodic axis, the quadratic ghost
// one node beyond a wall; positions a stencil never reads (further beyond a
// wall, or beyond two walls) get zeros.
template <class Node>
__device__ __forceinline__ void tile_node(const StepConsts& K, int x, int y, double* phi, Node node)
{
    if (!K.bcx) x = ((x % K.nx) + K.nx) % K.nx;
    if (!K.bcy) y = ((y % K.ny) + K.ny) % K.ny;
    const bool out_x = x < 0 || x >= K.nx, out_y = y < 0 || y >= K.ny;
    if (x < -1 || x > K.nx || y < -1 || y > K.ny || (out_x && out_y)) {
#pragma unroll
        for (int q = 0; q < 10; ++q) phi[q] = 0.0;
        return;
    }
    if (!out_x && !out_y) {
        node(x, y, phi);
        return;
    }
    // one node beyond a wall: ghost from the wall node and the next two inward
    int x0 = x, y0 = y, dx = 0, dy = 0;
    if (x == -1) x0 = 0, dx = 1;
    if (x == K.nx) x0 = K.nx - 1, dx = -1;
    if (y == -1) y0 = 0, dy = 1;
    if (y == K.ny) y0 = K.ny - 1, dy = -1;
    double a[10], b[10], c[10];
    node(x0, y0, a);
    node(x0 + dx, y0 + dy, b);
    node(x0 + 2 * dx, y0 + 2 * dy, c);
#pragma unroll
    for (int q = 0; q < 10; ++q) phi[q] = ghost(a[q], b[q], c[q]);
}

// tau c_j . grad Pi_j of component q at tile position (cx, cy), node (x, y)
__device__ __forceinline__ double transport_tile(const StepConsts& K, const double (*t)[TS_X], int cx, int cy, int q,
                                                 int x, int y, double lam)
{
    const int j = q % 5;
    if (j == 0) return 0.0;
    double U, V;
    if (K.met) {
        const size_t n = (size_t)K.nx * K.ny, i = (size_t)y * K.nx + x;
        const double ex = j == 1 ? 1.0 : (j == 3 ? -1.0 : 0.0), ey = j == 2 ? 1.0 : (j == 4 ? -1.0 : 0.0);
        U = ex * K.met[i] + ey * K.met[n + i];
        V = ex * K.met[2 * n + i] + ey * K.met[3 * n + i];
    } else {
        U = j == 1 ? gx_at(K, x) : (j == 3 ? -gx_at(K, x) : 0.0);
        V = j == 2 ? gy_at(K, y) : (j == 4 ? -gy_at(K, y) : 0.0);
    }
    double r = 0.0;
    if (U > 0.0)
        r += transport_pos(K, lam * U, t[cy][cx - 2], t[cy][cx - 1], t[cy][cx], t[cy][cx + 1]);
    else if (U < 0.0)
        r += transport_neg(K, -lam * U, t[cy][cx - 1], t[cy][cx], t[cy][cx + 1], t[cy][cx + 2]);
    if (V > 0.0)
        r += transport_pos(K, lam * V, t[cy - 2][cx], t[cy - 1][cx], t[cy][cx], t[cy + 1][cx]);
    else if (V < 0.0)
        r += transport_neg(K, -lam * V, t[cy - 1][cx], t[cy][cx], t[cy + 1][cx], t[cy + 2][cx]);
    return r;
}

// Only the eight moving components (j != 0) are streamed, so only they go
// through the tile (a 64 x 8 tile and its halo: 52 KB of LDS, two workgroups
// of eight waves per compute unit); slot s holds component q = s + 1 (s < 4)
// or s + 2.
__host__ __device__ constexpr int moving_slot(int q) { return q < 5 ? q - 1 : q - 2; }

// FULL = false: pass B, src = f_hat: Step (1) into the tile, the half step of
// f_bar^+, then Step (3), into f(t+h);
// FULL = true: pass C, src = f(t+h): Step (4) with f_hat^+ recomputed from f_hat.
template <bool FULL, bool SRC>
__global__ __launch_bounds__(TB_X* TB_Y) void k_pass_tiled(StepConsts K, const double* __restrict__ src,
                                                           const double* __restrict__ fh, double* __restrict__ dst)
{
    __shared__ double tile[8][TS_Y][TS_X];
    // pass B: f_bar^+ j = 0 of both sets at every tile position
    __shared__ double rest[FULL ? 1 : 2][FULL ? 1 : TS_Y][FULL ? 1 : TS_X];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int ox = (int)blockIdx.x * TB_X - TB_HALO, oy = (int)blockIdx.y * TB_Y - TB_HALO;
    if constexpr (kPoisonLds) {
        for (int idx = ty * TB_X + tx; idx < 8 * TS_X * TS_Y; idx += TB_X * TB_Y)
            (&tile[0][0][0])[idx] = lds_poison_value();
        if constexpr (!FULL)
            for (int idx = ty * TB_X + tx; idx < 2 * TS_X * TS_Y; idx += TB_X * TB_Y)
                (&rest[0][0][0])[idx] = lds_poison_value();
        __syncthreads();
    }
    for (int idx = ty * TB_X + tx; idx < TS_X * TS_Y; idx += TB_X * TB_Y) {
        const int ly = idx / TS_X, lx = idx - ly * TS_X;
        double phi[10];
        if constexpr (FULL) {
            tile_node(K, ox + lx, oy + ly, phi, [&](int x, int y, double* o) { load_node(src, K.pitch, x, y, o); });
        } else {
            // Step (1) at the interior nodes; wall nodes and the ghosts beyond
            // them follow from the tile below
            int x = ox + lx, y = oy + ly;
            if (!K.bcx) x = ((x % K.nx) + K.nx) % K.nx;
            if (!K.bcy) y = ((y % K.ny) + K.ny) % K.ny;
            if (x >= 0 && x < K.nx && y >= 0 && y < K.ny && !is_wall(K, x, y)) {
                double a[10];
                load10(K, src, x, y, a);
                collide1_bar<SRC>(K, a, phi, src_dp<SRC>(K, K.r_hat, x, y));
            } else {
#pragma unroll
                for (int q = 0; q < 10; ++q) phi[q] = 0.0;
            }
            rest[0][ly][lx] = phi[0];
            rest[FULL ? 0 : 1][ly][lx] = phi[5];
        }
#pragma unroll
        for (int q = 0; q < 10; ++q)
            if (q % 5 != 0) tile[moving_slot(q)][ly][lx] = phi[q];
    }
    __syncthreads();
    if constexpr (!FULL) {
        // A tile that holds wall nodes (uniform over the workgroup).  Their
        // inward neighbours are interior nodes of the same tile (grids have at
        // least 5 nodes per axis), so the wall rule takes their f_bar^+ from
        // LDS; then the ghost one node beyond a wall is the quadratic
        // extrapolation from the wall node and the next two inward nodes
        // (positions beyond two walls stay zero).
        const bool edge = (K.bcx && (ox <= 0 || ox + TS_X >= K.nx)) || (K.bcy && (oy <= 0 || oy + TS_Y >= K.ny));
        if (edge) {
            auto at = [&](int lx, int ly, double* o) {
#pragma unroll
                for (int q = 0; q < 10; ++q)
                    o[q] = q % 5 == 0 ? rest[FULL ? 0 : q / 5][ly][lx] : tile[moving_slot(q)][ly][lx];
            };
            for (int idx = ty * TB_X + tx; idx < TS_X * TS_Y; idx += TB_X * TB_Y) {
                const int ly = idx / TS_X, lx = idx - ly * TS_X;
                int x = ox + lx, y = oy + ly;
                if (!K.bcx) x = ((x % K.nx) + K.nx) % K.nx;
                if (!K.bcy) y = ((y % K.ny) + K.ny) % K.ny;
                int x1, y1, x2, y2;
                double uw;
                if (x < 0 || x >= K.nx || y < 0 || y >= K.ny || !wall_neighbours(K, x, y, x1, y1, x2, y2, uw))
                    continue;
                double p1[10], p2[10], out[10];
                at(lx + (x1 - x), ly + (y1 - y), p1);
                at(lx + (x2 - x), ly + (y2 - y), p2);
                wall_extrapolate<SRC>(K, p1, p2, uw, out, src_dp<SRC>(K, K.r_bp, x1, y1),
                                      src_dp<SRC>(K, K.r_bp, x2, y2));
                rest[0][ly][lx] = out[0];
                rest[FULL ? 0 : 1][ly][lx] = out[5];
#pragma unroll
                for (int q = 0; q < 10; ++q)
                    if (q % 5 != 0) tile[moving_slot(q)][ly][lx] = out[q];
            }
            __syncthreads();
            for (int idx = ty * TB_X + tx; idx < TS_X * TS_Y; idx += TB_X * TB_Y) {
                const int ly = idx / TS_X, lx = idx - ly * TS_X;
                const int x = ox + lx, y = oy + ly;
                const bool ox_ = K.bcx && (x == -1 || x == K.nx), oy_ = K.bcy && (y == -1 || y == K.ny);
                const bool in_x = !K.bcx || (x >= 0 && x < K.nx), in_y = !K.bcy || (y >= 0 && y < K.ny);
                if (!((ox_ && in_y) || (oy_ && in_x))) continue;
                const int dx = ox_ ? (x == -1 ? 1 : -1) : 0, dy = oy_ ? (y == -1 ? 1 : -1) : 0;
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    tile[s][ly][lx] = ghost(tile[s][ly + dy][lx + dx], tile[s][ly + 2 * dy][lx + 2 * dx],
                                            tile[s][ly + 3 * dy][lx + 3 * dx]);
            }
            __syncthreads();
        }
    }
    const int x = (int)blockIdx.x * TB_X + tx, y = (int)blockIdx.y * TB_Y + ty;
    if (x >= K.nx || y >= K.ny || is_wall(K, x, y)) return;
    const int cx = tx + TB_HALO, cy = ty + TB_HALO;
    double base[10], out[10];
    if (FULL) {
        double a[10];
        load_node(fh, K.pitch, x, y, a);
        collide1_hat<SRC>(K, a, base, src_dp<SRC>(K, K.r_hat, x, y));
    } else {
#pragma unroll
        for (int q = 0; q < 10; ++q)
            base[q] = q % 5 == 0 ? rest[FULL ? 0 : q / 5][FULL ? 0 : cy][FULL ? 0 : cx] : tile[moving_slot(q)][cy][cx];
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const double tr = q % 5 == 0 ? 0.0 : transport_tile(K, tile[moving_slot(q)], cx, cy, q, x, y,
                                                             FULL ? K.lam_dt : K.lam_h);
        out[q] = base[q] - tr + (FULL ? dwf_at(K, x, y, q / 5) : hwf_at(K, x, y, q / 5));
    }
    if (FULL) {
        store_node(dst, K.pitch, x, y, out);
    } else {
        double fm[10];
        collide3<SRC>(K, out, fm, src_dp<SRC>(K, K.r_bar, x, y));
        store_node(dst, K.pitch, x, y, fm);
    }
}

inline dim3 grid2d(const StepConsts& K, dim3 b) { return dim3((K.nx + b.x - 1) / b.x, (K.ny + b.y - 1) / b.y); }

}  // namespace

hipError_t launch_init(const StepConsts& K, const double* u0, const double* v0, const double* p0, double* f,
                       hipStream_t s)
{
    const dim3 b(64, 4);
    hipLaunchKernelGGL(k_init, grid2d(K, b), b, 0, s, K, u0, v0, p0, f);
    return hipGetLastError();
}

// wall rule on the wall nodes of a stored f_hat: one thread per perimeter
// node (a launch over every node cost 30 us at 2048^2, this one about 6 us)
hipError_t launch_wall_fix(const StepConsts& K, double* f, hipStream_t s)
{
    const int nper = perimeter_count(K);
    if (nper <= 0) return hipSuccess;
    const dim3 g((nper + 255) / 256), b(256);
    if (K.rsrc)
        hipLaunchKernelGGL(k_perimeter_wall<true>, g, b, 0, s, K, f, K.r_hat);
    else
        hipLaunchKernelGGL(k_perimeter_wall<false>, g, b, 0, s, K, f, 0.0);
    return hipGetLastError();
}

hipError_t launch_moments(const StepConsts& K, const double* f, double* u, double* v, double* p, hipStream_t s)
{
    const dim3 b(64, 4);
    hipLaunchKernelGGL(k_moments, grid2d(K, b), b, 0, s, K, f, u, v, p);
    return hipGetLastError();
}

hipError_t launch_derived(const StepConsts& K, const double* f, double* out, uint32_t mask, hipStream_t s)
{
    const dim3 b(64, 4);
    hipLaunchKernelGGL(k_derived, grid2d(K, b), b, 0, s, K, f, out, mask);
    return hipGetLastError();
}

int diag_blocks(const StepConsts& K)
{
    const long long tiles = (long long)((K.nx + DT_X - 1) / DT_X) * ((K.ny + DT_Y - 1) / DT_Y);
    return (int)(tiles < kDiagMaxBlocks ? tiles : kDiagMaxBlocks);
}

hipError_t launch_diagnostics(const StepConsts& K, const double* f, double* partials, double* out8, hipStream_t s)
{
    const int nb = diag_blocks(K);
    hipLaunchKernelGGL(k_diag_partial, dim3(nb), dim3(DIAG_BLOCK), 0, s, K, f, partials);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(DIAG_BLOCK), 0, s, partials, nb, out8);
    return hipGetLastError();
}

// Streaming copy: each thread moves four 16-byte units per pass, 256 units
// apart so that a wave's loads cover 1 KiB contiguous each; the grid is sized
// to keep every compute unit busy and loops over the rest.
__global__ __launch_bounds__(256) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     size_t n16)
{
    const size_t stride = (size_t)gridDim.x * 1024;
    size_t i = (size_t)blockIdx.x * 1024 + threadIdx.x;
    for (; i + 768 < n16; i += stride) {
        const uint4 a = src[i], b = src[i + 256], c = src[i + 512], d = src[i + 768];
        dst[i] = a;
        dst[i + 256] = b;
        dst[i + 512] = c;
        dst[i + 768] = d;
    }
    for (int k = 0; k < 4; ++k)
        if (i + 256 * k < n16) dst[i + 256 * k] = src[i + 256 * k];
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    size_t blocks = (n16 + 1023) / 1024;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

hipError_t launch_pack(const StepConsts& K, const double* f, double* dense, hipStream_t s)
{
    const dim3 b(64, 4);
    hipLaunchKernelGGL(k_pack, grid2d(K, b), b, 0, s, K, f, dense);
    return hipGetLastError();
}

hipError_t launch_unpack(const StepConsts& K, const double* dense, double* f, hipStream_t s)
{
    const dim3 b(64, 4);
    hipLaunchKernelGGL(k_unpack, grid2d(K, b), b, 0, s, K, dense, f);
    return hipGetLastError();
}

namespace {
template <bool SRC>
void tiled_step(const StepConsts& K, const double* fh, double* fmid, double* fnew, hipStream_t s)
{
    const dim3 bt(TB_X, TB_Y);
    const int nper = perimeter_count(K);
    hipLaunchKernelGGL((k_pass_tiled<false, SRC>), grid2d(K, bt), bt, 0, s, K, fh, nullptr, fmid);
    if (nper > 0) hipLaunchKernelGGL(k_perimeter_wall<SRC>, dim3((nper + 255) / 256), dim3(256), 0, s, K, fmid, K.r_f);
    hipLaunchKernelGGL((k_pass_tiled<true, SRC>), grid2d(K, bt), bt, 0, s, K, fmid, fh, fnew);
    if (nper > 0) hipLaunchKernelGGL(k_perimeter_wall<SRC>, dim3((nper + 255) / 256), dim3(256), 0, s, K, fnew, K.r_hat);
}
}  // namespace

// the kernels with the mass source's pressure offsets are separate instances,
// so a run without source executes exactly the plain step
hipError_t launch_tiled_step(const StepConsts& K, const double* fh, double* fmid, double* fnew, hipStream_t s)
{
    if (K.rsrc)
        tiled_step<true>(K, fh, fmid, fnew, s);
    else
        tiled_step<false>(K, fh, fmid, fnew, s);
    return hipGetLastError();
}

}  // namespace mdf
