// Fused single-pass MDF-FDLBM time step for gfx950 (kernel templates).
//
// One workgroup owns a column strip of TW lanes (one column per lane; the 4
// columns at each side are halo) and marches up the rows of one segment.  For
// the row k entering the march it runs, in registers:
//   A   load f_hat(k); Step (1) collision -> f_hat^+(k), f_bar^+(k)   (eqs. 2.2.14-15)
//   A'  x-neighbours of f_bar^+ through LDS; x part of the half step of row k
//   B   y part of the half step of row m = k-2 from a 4-row register window,
//       Step (3) collision -> f(t+h)(m)                              (eqs. 2.3.25, 2.2.16)
//   B'  x-neighbours of f(t+h) through LDS; x part of Step (4) for row m -> store
//   C   y part of Step (4) for row r = k-4 from the f(t+h) window -> store (eq. 2.3.24)
// so HBM sees one read and one write of the 10 distribution planes per node.
// B does not depend on the exchange of A', so both rows publish their
// x-streamed components first and meet at a single LDS barrier per row.
// Row windows are 4-deep register rings indexed by (row - first row) & 3; the
// march is unrolled by 4 so every ring index is a compile-time constant.
//
// Walls: the wall rule (non-equilibrium extrapolation from the two inward
// neighbours) is applied to f_bar^+ and to f(t+h) inside the march; wall nodes
// of f_hat(t+dt) are not written here -- the stored wall values never enter
// the next step, and the host applies the rule to the final state once per
// mdf_step call.  Beyond a wall the stencil uses the quadratic ghost node.
#pragma once

#include <type_traits>

#include "mdf_device.hpp"
#include "mdf_internal.hpp"

namespace mdf {
namespace fusedk {

struct FusedGrid {
    int nstrips, nsegs, chunk, nwg;
    const int4* table;   // (strip, ys0, ys1, 0) per workgroup, or null: nsegs equal segments per strip
    // Strip s covers columns xoff + s*xspan/nstrips .. xoff + (s+1)*xspan/nstrips - 1.  With
    // wall tasks (xoff = kWallCols) the columns next to each x wall are not cut into strips:
    // table entries (-1 - j, 0, 0, 0) run TW/64 single-wave tasks (xs0, xs1, ys0, ys1) read
    // from table[nwg + j*TW/64 + wave].
    int xoff, xspan;
};

// equilibrium component (velocity along the wall normal axis) used by the wall
// rule; `ax` is the axis of c_j (0 = x, 1 = y), sg the sign of c_j.
__device__ __forceinline__ double feq_comp(const StepConsts& K, int a, int ax, double sg, double u, double v, double P)
{
    const double ua = a == 0 ? u : v;
    const double flux = ax == 0 ? (a == 0 ? u * u + P : v * u) : (a == 0 ? u * v : v * v + P);
    return K.w * ua + sg * K.kf * flux;
}

// wall value of one component from the inward neighbours n1, n2 (moments m1, m2)
__device__ __forceinline__ double wall_comp(const StepConsts& K, int a, int ax, double sg, double p1, double p2,
                                            const double* m1, const double* m2, double uw)
{
    const double e1 = feq_comp(K, a, ax, sg, m1[0], m1[1], m1[2]);
    const double e2 = feq_comp(K, a, ax, sg, m2[0], m2[1], m2[2]);
    const double ew = feq_comp(K, a, ax, sg, uw, 0.0, m1[2]);
    return ew + 2.0 * (p1 - e1) - (p2 - e2);
}

template <int TW>
__device__ __forceinline__ int lclamp(int l)
{
    return l < 0 ? 0 : (l >= TW ? TW - 1 : l);
}

// Read the x-neighbours (offsets -2..2) of the 4 exchanged components; at
// x-walls replace the wall column by the wall rule and the column beyond it
// by the ghost node.  comp c = (alpha = c/2, j = 1 if c even else 3).
// X = [4 components][their non-equilibrium parts g = f - f^eq][P][lane]: the
// wall rule f_w = f^eq_w + 2 g(n1) - g(n2) then needs no equilibrium of the
// neighbours, only f^eq at the wall (u = v = 0, P = P(n1)): +-kf P for the u
// set and 0 for the v set along x.  The inward neighbours n1, n2 are fixed
// columns (1, 2 at the left wall; nx-2, nx-3 at the right), so every lane
// reads them at the same LDS address, in the same round trip as its own
// neighbours, and the lanes next to the wall select the result.
template <int TW, bool WX>
__device__ __forceinline__ void x_neighbours(const StepConsts& K, double (*X)[TW], int lane, int x, double nb[4][5],
                                             bool wall_strip)
{
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int d = -2; d <= 2; ++d) nb[c][d + 2] = X[c][lclamp<TW>(lane + d)];
    if (WX && wall_strip) {
        const int x0 = __builtin_amdgcn_readfirstlane(x - lane);   // column of lane 0
        if (x0 <= 2) {   // the strip holds column 1 or 2
            const int l1 = lclamp<TW>(1 - x0), l2 = lclamp<TW>(2 - x0);
            const double kp = K.kf * X[8][l1];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double ew = c >= 2 ? 0.0 : ((c & 1) ? -kp : kp);
                const double w0 = ew + 2.0 * X[4 + c][l1] - X[4 + c][l2];
                const double gh = ghost(w0, X[c][l1], X[c][l2]);
                nb[c][1] = x == 1 ? w0 : nb[c][1];
                nb[c][0] = x == 1 ? gh : (x == 2 ? w0 : nb[c][0]);
            }
        }
        if (x0 + TW - 1 >= K.nx - 3) {   // the strip holds column nx-3 or nx-2
            const int l1 = lclamp<TW>(K.nx - 2 - x0), l2 = lclamp<TW>(K.nx - 3 - x0);
            const double kp = K.kf * X[8][l1];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double ew = c >= 2 ? 0.0 : ((c & 1) ? -kp : kp);
                const double w0 = ew + 2.0 * X[4 + c][l1] - X[4 + c][l2];
                const double gh = ghost(w0, X[c][l1], X[c][l2]);
                nb[c][3] = x == K.nx - 2 ? w0 : nb[c][3];
                nb[c][4] = x == K.nx - 2 ? gh : (x == K.nx - 3 ? w0 : nb[c][4]);
            }
        }
    }
}

// The march of one strip segment: output columns xs0..xs1-1, rows ys0..ys1-1.
// FF: a steady force field F(x) (K.ff, (F_x, F_y) per node, uniform part
// included) replaces the uniform force; its rows arrive with the state rows.
template <int TW, bool WX, bool WY, int PLK, int PF, bool UNI, bool FF>
__device__ __forceinline__ void fused_march(const StepConsts& K, const double* __restrict__ fin,
                                            double* __restrict__ fout, const double* __restrict__ gyp, int xs0,
                                            int xs1, int ys0, int ys1, double (*xs)[9][TW], int lane)
{
    const int x = xs0 - 4 + lane;
    int xg;
    if (WX) {
        xg = x < 0 ? 0 : (x >= K.nx ? K.nx - 1 : x);
    } else {
        xg = x % K.nx;
        if (xg < 0) xg += K.nx;
    }
    const bool outc = (x >= xs0) && (x < xs1) && (!WX || (x >= 1 && x <= K.nx - 2));
    // workgroup-uniform: only strips holding lanes for columns 1-2 or nx-3..nx-2
    // (lanes span xs0-4 .. xs1+3) and segments whose march reaches rows 0-2 or
    // ny-3..ny-1 run the wall-rule code; the margin of 8 is generous
    const bool wall_strip = WX && (xs0 <= 8 || xs1 >= K.nx - 8);
    const bool wall_seg = WY && (ys0 <= 8 || ys1 >= K.ny - 8);
    // x stencils: constants on a uniform grid, per lane (column) on a mapped one
    const double gxl = UNI ? 0.0 : K.gx[xg];
    const Stencil SXh = UNI ? stencil_of(K.sh[0]) : make_stencil(K, K.lam_h * gxl, true);
    const Stencil SXd = UNI ? stencil_of(K.sd[0]) : make_stencil(K, K.lam_dt * gxl, false);
    // y stencils from the derivative scale gy of the row (mapped grids; the
    // scale arrives with the row's prefetch)
    auto y_stencil_h = [&](double gyr) -> Stencil {
        return UNI ? stencil_of(K.sh[1]) : make_stencil(K, K.lam_h * gyr, true);
    };
    auto y_stencil_d = [&](double gyr) -> Stencil {
        return UNI ? stencil_of(K.sd[1]) : make_stencil(K, K.lam_dt * gyr, false);
    };
    // Every row access goes through a buffer descriptor of that one row
    // (scalar registers), so the lane offsets below are the only vector
    // addresses.  A row that must not be touched gets zero records: its loads
    // return 0 (rows beyond a y wall) and its stores are dropped; halo lanes
    // store to an offset past the end of the row.
    // byte offsets of this lane's node within a row: x-part block, y-part block
    const unsigned vx = (unsigned)xg * 48u, vy = (unsigned)K.pitch * 48u + (unsigned)xg * 32u;
    const unsigned vx_st = outc ? vx : 0x7fffff00u, vy_st = outc ? vy : 0x7fffff00u;
    // An output column needs f_bar^+ up to 4 columns away (two stencils of
    // reach 2), so lanes past xs1 + 3 -- the surplus of a strip narrower than
    // its lanes -- feed no output: their loads read past the row's records
    // (zeros, no memory traffic) and their results are never stored.
    const bool lane_needed = x <= xs1 + 3;
    const unsigned vx_ld = lane_needed ? vx : 0x7fffff00u, vy_ld = lane_needed ? vy : 0x7fffff00u;
    const int row_bytes = K.pitch * 80;

    auto wrap_y = [&](int k) -> int {
        if (WY) return k;
        return k < 0 ? k + K.ny : (k >= K.ny ? k - K.ny : k);
    };
    auto row_ok = [&](int k) -> bool { return WY ? (k >= 0 && k < K.ny) : true; };

    // rows kbeg..kend enter the march, padded to whole 4-row groups (the
    // padding rows reach no output) so the unrolled loop has no partial group
    const int kbeg = ys0 - 4, kend = ys1 + 3;
    const int kpad = kbeg + ((kend - kbeg + 4) & ~3) - 1;

    // prefetch ring: row k lives in slot (k - kbeg) & 3 and is requested PF rows
    // ahead.  Every body issues the same loads and stores whatever its row, so
    // the compiler counts the memory operations in flight exactly and waits
    // only for the row it consumes.
    double pre[4][10], pgy[4] = {0.0, 0.0, 0.0, 0.0}, pff[4][2];
    const unsigned vf = lane_needed ? (unsigned)xg * 16u : 0x7fffff00u;   // this lane's (F_x, F_y) in a force row
    auto load_row = [&](int k, double* dst, double& gyr, double* fdst) {
        const bool on = k <= kend && row_ok(k);   // rows past kend are never used
        const BufRes rs = row_res(fin, row_bytes, on ? wrap_y(k) : 0, on);
        if (!UNI) gyr = gyp[on ? wrap_y(k) : 0];
        if (FF) {
            const dvec2 fv = buf_load2(row_res(K.ff, K.pitch * 16, on ? wrap_y(k) : 0, on), vf);
            fdst[0] = fv.x;
            fdst[1] = fv.y;
        }
        const dvec2 a = buf_load2(rs, vx_ld), b = buf_load2(rs, vx_ld + 16u), c = buf_load2(rs, vx_ld + 32u);
        const dvec2 d = buf_load2(rs, vy_ld), e = buf_load2(rs, vy_ld + 16u);
        dst[0] = a.x; dst[1] = a.y; dst[3] = b.x;   // x part: j = 0, 1, 3 of each set
        dst[5] = b.y; dst[6] = c.x; dst[8] = c.y;
        dst[2] = d.x; dst[4] = d.y;                 // y part: j = 2, 4 of each set
        dst[7] = e.x; dst[9] = e.y;
    };

    double W2[4][2], W4[4][2], F2[4][2], F4[4][2], Qy[4][4], Qx[2][6], Qb[2][6];
    double gring[4] = {0.0, 0.0, 0.0, 0.0};   // gy of the last four rows (mapped grids)
    double fring[4][2];                         // F of the last four rows (force field)
#pragma unroll
    for (int i = 0; i < 4; ++i) fring[i][0] = fring[i][1] = pff[i][0] = pff[i][1] = 0.0;
    double ub_prev[3] = {0, 0, 0}, uf_prev[3] = {0, 0, 0}, pend_b[4] = {0, 0, 0, 0}, pend_f[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        W2[i][0] = W2[i][1] = W4[i][0] = W4[i][1] = 0.0;
        F2[i][0] = F2[i][1] = F4[i][0] = F4[i][1] = 0.0;
        Qy[i][0] = Qy[i][1] = Qy[i][2] = Qy[i][3] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 6; ++q) Qx[i][q] = Qb[i][q] = 0.0;

#pragma unroll
    for (int i = 0; i < PF; ++i) load_row(kbeg + i, pre[i], pgy[i], pff[i]);

    // LOOP: a body of the loop (row k >= ys0) of the wall-free Newtonian
    // march.  There both collisions of a row run unconditionally (rows no
    // output needs are computed and never stored), so stages A and B form one
    // basic block the scheduler can interleave: +1.4 % on a periodic grid,
    // +2.5 % on the batch.  The power-law collisions lose 8-30 % that way (the
    // interleaved root solves crowd the register file), and the peeled first
    // group keeps the branches everywhere.
    auto body = [&](auto PC, int k, auto LP) {
        constexpr int P = decltype(PC)::value;
        constexpr bool LOOP = decltype(LP)::value && PLK == PL_NEWTON && !WX && !WY;
        constexpr int S1 = (P + 3) & 3, S2 = (P + 2) & 3, S3 = (P + 1) & 3;   // rows k-1, k-2, k-3
        double cur[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) cur[q] = pre[P][q];
        // gy of rows k-1..k-4 by ring slot: m = k-2 in S2, r = k-4 in slot P
        // (read before the push of row k below)
        const double gy_m = gring[S2], gy_r = gring[P];
        gring[P] = pgy[P];
        // force terms h w F and dt w F of rows k (A'), m = k-2 (B, B') and
        // r = k-4 (C); the F ring works like the gy ring
        double hwk[2], hwm[2], dwm[2], dwr[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (FF) {
                hwk[a] = K.hw * pff[P][a];
                hwm[a] = K.hw * fring[S2][a];
                dwm[a] = K.dw * fring[S2][a];
                dwr[a] = K.dw * fring[P][a];
            } else {
                hwk[a] = hwm[a] = K.hwf[a];
                dwm[a] = dwr[a] = K.dwf[a];
            }
        }
        if (FF) {
            fring[P][0] = pff[P][0];
            fring[P][1] = pff[P][1];
        }
        load_row(k + PF, pre[(P + PF) & 3], pgy[(P + PF) & 3], pff[(P + PF) & 3]);

        // ---- A: Step (1) on row k ----
        double fbp[10], fhp[10], ub[3], gb[4];
        {
            double fe[10];
            node_moments(cur, K.c, ub[0], ub[1], ub[2]);
            equilibrium(ub[0], ub[1], ub[2], K, fe);
            Relax ra, rb;
            step1_factors_t<PLK>(K, cur, fe, ra, rb);
            relax(cur, fe, rb, fbp);
            gb[0] = fbp[1] - fe[1];
            gb[1] = fbp[3] - fe[3];
            gb[2] = fbp[6] - fe[6];
            gb[3] = fbp[8] - fe[8];
            if (LOOP || (k >= ys0 && k < ys1)) {
                relax(cur, fe, ra, fhp);
            } else {
#pragma unroll
                for (int q = 0; q < 10; ++q) fhp[q] = 0.0;
            }
        }
        double b2[2] = {fbp[2], fbp[7]};
        W4[P][0] = fbp[4];
        W4[P][1] = fbp[9];
        if (WY && wall_seg) {
            if (k == 2) {   // bottom wall row 0 from rows 1 and 2
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    W2[S2][a] = wall_comp(K, a, 1, 1.0, W2[S1][a], b2[a], ub_prev, ub, 0.0);
                    W4[S2][a] = wall_comp(K, a, 1, -1.0, W4[S1][a], W4[P][a], ub_prev, ub, 0.0);
                }
            }
            if (k == K.ny - 2) {   // top wall row ny-1 from rows ny-2 and ny-3, used next row
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    pend_b[2 * a] = wall_comp(K, a, 1, 1.0, b2[a], W2[S1][a], ub, ub_prev, K.lid_u);
                    pend_b[2 * a + 1] = wall_comp(K, a, 1, -1.0, W4[P][a], W4[S1][a], ub, ub_prev, K.lid_u);
                }
            }
            if (k == K.ny - 1) {
                b2[0] = pend_b[0];
                b2[1] = pend_b[2];
                W4[P][0] = pend_b[1];
                W4[P][1] = pend_b[3];
            }
        }

        // ---- A' (publish): the x-streamed components of row k ----
        // Both exchanges of the body (A' for row k, B' for row m) go through
        // one barrier.  Their buffers alternate with the body's parity, so a
        // wave's next writes never reach a buffer another wave still reads.
        double(*XA)[TW] = xs[2 * (P & 1)];
        double(*XB)[TW] = xs[2 * (P & 1) + 1];
        if constexpr (kPoisonLds) {
#pragma unroll
            for (int c = 0; c < 9; ++c) XA[c][lane] = XB[c][lane] = lds_poison_value();
        }
        XA[0][lane] = fbp[1];
        XA[1][lane] = fbp[3];
        XA[2][lane] = fbp[6];
        XA[3][lane] = fbp[8];
        if (WX && wall_strip) {
#pragma unroll
            for (int c = 0; c < 4; ++c) XA[4 + c][lane] = gb[c];
            XA[8][lane] = ub[2];
        }

        // ---- B: half step (y part) and Step (3) on row m = k-2 ----
        const int m = k - 2;
        const bool needB = (m >= ys0 - 2) && (m < ys1 + 2) && (WY ? (m >= 1 && m <= K.ny - 2) : true);
        double f2c[2] = {0.0, 0.0};
        double fm[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, uf[3] = {0.0, 0.0, 0.0};
        double gf[4] = {0.0, 0.0, 0.0, 0.0};
        if (LOOP || needB) {
            const Stencil SYh = y_stencil_h(gy_m);
            double fb[10];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                double a2[4] = {W2[P][a], W2[S3][a], W2[S2][a], W2[S1][a]};   // rows m-2 .. m+1
                double a4[4] = {W4[S3][a], W4[S2][a], W4[S1][a], W4[P][a]};   // rows m-1 .. m+2
                if (WY && wall_seg && m == 1) a2[0] = ghost(a2[1], a2[2], a2[3]);
                if (WY && wall_seg && m == K.ny - 2) a4[3] = ghost(a4[2], a4[1], a4[0]);
                fb[5 * a + 0] = Qb[P & 1][3 * a + 0];
                fb[5 * a + 1] = Qb[P & 1][3 * a + 1];
                fb[5 * a + 3] = Qb[P & 1][3 * a + 2];
                fb[5 * a + 2] = upd_pos(SYh, hwm[a], a2[0], a2[1], a2[2], a2[3]);
                fb[5 * a + 4] = upd_neg(SYh, hwm[a], a4[0], a4[1], a4[2], a4[3]);
            }
            double fe[10];
            node_moments(fb, K.c, uf[0], uf[1], uf[2]);
            equilibrium(uf[0], uf[1], uf[2], K, fe);
            const Relax rq = step3_factors_t<PLK>(K, fb, fe);
            relax(fb, fe, rq, fm);
            gf[0] = fm[1] - fe[1];
            gf[1] = fm[3] - fe[3];
            gf[2] = fm[6] - fe[6];
            gf[3] = fm[8] - fe[8];
            F4[S2][0] = fm[4];
            F4[S2][1] = fm[9];
            f2c[0] = fm[2];
            f2c[1] = fm[7];
        }
        if (WY && wall_seg) {
            if (m == 2) {   // bottom wall row 0 of f(t+h)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    F2[P][a] = wall_comp(K, a, 1, 1.0, F2[S3][a], f2c[a], uf_prev, uf, 0.0);
                    F4[P][a] = wall_comp(K, a, 1, -1.0, F4[S3][a], F4[S2][a], uf_prev, uf, 0.0);
                }
            }
            if (m == K.ny - 2) {
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    pend_f[2 * a] = wall_comp(K, a, 1, 1.0, f2c[a], F2[S3][a], uf, uf_prev, K.lid_u);
                    pend_f[2 * a + 1] = wall_comp(K, a, 1, -1.0, F4[S2][a], F4[S3][a], uf, uf_prev, K.lid_u);
                }
            }
            if (m == K.ny - 1) {
                f2c[0] = pend_f[0];
                f2c[1] = pend_f[2];
                F4[S2][0] = pend_f[1];
                F4[S2][1] = pend_f[3];
            }
        }

        // ---- B' (publish): the x-streamed components of f(t+h) on row m ----
        XB[0][lane] = fm[1];
        XB[1][lane] = fm[3];
        XB[2][lane] = fm[6];
        XB[3][lane] = fm[8];
        if (WX && wall_strip) {
#pragma unroll
            for (int c = 0; c < 4; ++c) XB[4 + c][lane] = gf[c];
            XB[8][lane] = uf[2];
        }
        exchange_barrier<TW / 64>();

        // ---- A': x part of the half step for row k ----
        double bx[6];
        {
            double nb[4][5];
            x_neighbours<TW, WX>(K, XA, lane, x, nb, wall_strip);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                bx[3 * a + 0] = fbp[5 * a] + hwk[a];
                bx[3 * a + 1] = upd_pos(SXh, hwk[a], nb[2 * a][0], nb[2 * a][1], nb[2 * a][2], nb[2 * a][3]);
                bx[3 * a + 2] =
                    upd_neg(SXh, hwk[a], nb[2 * a + 1][1], nb[2 * a + 1][2], nb[2 * a + 1][3], nb[2 * a + 1][4]);
            }
        }

        // ---- B': x part of Step (4) on row m ----
        const bool outm = needB && (m >= ys0) && (m < ys1);
        {
            double h[2][3];
            double nb[4][5];
            x_neighbours<TW, WX>(K, XB, lane, x, nb, wall_strip);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                h[a][0] = Qx[P & 1][3 * a + 0] + dwm[a];
                h[a][1] = upd_pos(SXd, Qx[P & 1][3 * a + 1] + dwm[a], nb[2 * a][0], nb[2 * a][1], nb[2 * a][2],
                                  nb[2 * a][3]);
                h[a][2] = upd_neg(SXd, Qx[P & 1][3 * a + 2] + dwm[a], nb[2 * a + 1][1], nb[2 * a + 1][2],
                                  nb[2 * a + 1][3], nb[2 * a + 1][4]);
            }
            // x part of row m is final: one contiguous 48 B block per node
            const BufRes rs = row_res(fout, row_bytes, outm ? wrap_y(m) : 0, outm);
            buf_store2(rs, vx_st, dvec2{h[0][0], h[0][1]});
            buf_store2(rs, vx_st + 16u, dvec2{h[0][2], h[1][0]});
            buf_store2(rs, vx_st + 32u, dvec2{h[1][1], h[1][2]});
        }

        // ---- C: y part of Step (4) on row r = k-4 ----
        const int r = k - 4;
        const bool outr = (r >= ys0) && (r < ys1) && (WY ? (r >= 1 && r <= K.ny - 2) : true);
        {
            const Stencil SYd = y_stencil_d(gy_r);
            double hy[2][2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                double c2[4] = {F2[S2][a], F2[S1][a], F2[P][a], F2[S3][a]};   // rows r-2 .. r+1
                double c4[4] = {F4[S1][a], F4[P][a], F4[S3][a], F4[S2][a]};   // rows r-1 .. r+2
                if (WY && wall_seg && r == 1) c2[0] = ghost(c2[1], c2[2], c2[3]);
                if (WY && wall_seg && r == K.ny - 2) c4[3] = ghost(c4[2], c4[1], c4[0]);
                hy[a][0] = upd_pos(SYd, Qy[P][2 * a] + dwr[a], c2[0], c2[1], c2[2], c2[3]);
                hy[a][1] = upd_neg(SYd, Qy[P][2 * a + 1] + dwr[a], c4[0], c4[1], c4[2], c4[3]);
            }
            // y part of row r is final: one contiguous 32 B block per node
            const BufRes rs = row_res(fout, row_bytes, outr ? wrap_y(r) : 0, outr);
            buf_store2(rs, vy_st, dvec2{hy[0][0], hy[0][1]});
            buf_store2(rs, vy_st + 16u, dvec2{hy[1][0], hy[1][1]});
        }

        // ---- ring pushes ----
        W2[P][0] = b2[0];
        W2[P][1] = b2[1];
        Qy[P][0] = fhp[2];
        Qy[P][1] = fhp[4];
        Qy[P][2] = fhp[7];
        Qy[P][3] = fhp[9];
        Qx[P & 1][0] = fhp[0];
        Qx[P & 1][1] = fhp[1];
        Qx[P & 1][2] = fhp[3];
        Qx[P & 1][3] = fhp[5];
        Qx[P & 1][4] = fhp[6];
        Qx[P & 1][5] = fhp[8];
#pragma unroll
        for (int q = 0; q < 6; ++q) Qb[P & 1][q] = bx[q];
        F2[S2][0] = f2c[0];
        F2[S2][1] = f2c[1];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            ub_prev[q] = ub[q];
            uf_prev[q] = needB ? uf[q] : uf_prev[q];   // a select: a conditional store here lands in scratch
        }
    };

    // the first group is peeled so that the loop is entered with the same
    // memory operations in flight as on its back edge
    using Peeled = std::false_type;
    using Loop = std::true_type;
    body(std::integral_constant<int, 0>{}, kbeg, Peeled{});
    body(std::integral_constant<int, 1>{}, kbeg + 1, Peeled{});
    body(std::integral_constant<int, 2>{}, kbeg + 2, Peeled{});
    body(std::integral_constant<int, 3>{}, kbeg + 3, Peeled{});
    for (int k = kbeg + 4; k <= kpad; k += 4) {
        body(std::integral_constant<int, 0>{}, k, Loop{});
        body(std::integral_constant<int, 1>{}, k + 1, Loop{});
        body(std::integral_constant<int, 2>{}, k + 2, Loop{});
        body(std::integral_constant<int, 3>{}, k + 3, Loop{});
    }
}

// One single-wave task (xs0, xs1, ys0, ys1) of a workgroup of TW lanes: a 64-lane march on
// this wave's share of the workgroup's exchange buffers, with wave barriers only, so the
// wave runs at its own pace.  An empty task (xs0 >= xs1) returns at once.
template <int TW, bool WY, int PLK, int PF, bool UNI, bool FF>
__device__ __forceinline__ void wall_tasks(const StepConsts& K, const double* __restrict__ fin,
                                           double* __restrict__ fout, const double* __restrict__ gyp, int4 t,
                                           double (*xs)[9][TW])
{
    if (t.x >= t.y) return;
    double(*xw)[9][64] = reinterpret_cast<double(*)[9][64]>(&xs[0][0][0] + (threadIdx.x >> 6) * (4 * 9 * 64));
    const int lane = (int)(threadIdx.x & 63);
    const bool near_x = t.x <= 8 || t.y >= K.nx - 8;
    const bool near_y = WY && (t.z <= 8 || t.w >= K.ny - 8);
    if (near_x && near_y)
        fused_march<64, true, WY, PLK, PF, UNI, FF>(K, fin, fout, gyp, t.x, t.y, t.z, t.w, xw, lane);
    else if (near_x)
        fused_march<64, true, false, PLK, PF, UNI, FF>(K, fin, fout, gyp, t.x, t.y, t.z, t.w, xw, lane);
    else if (near_y)
        fused_march<64, false, WY, PLK, PF, UNI, FF>(K, fin, fout, gyp, t.x, t.y, t.z, t.w, xw, lane);
    else
        fused_march<64, false, false, PLK, PF, UNI, FF>(K, fin, fout, gyp, t.x, t.y, t.z, t.w, xw, lane);
}

template <int TW, bool WX, bool WY, int PLK, int PF, bool UNI, bool FF>
__global__ __launch_bounds__(TW) void k_fused(StepConsts K, const double* __restrict__ fin, double* __restrict__ fout,
                                              const double* __restrict__ gyp, FusedGrid G)
{
    __shared__ double xs[4][9][TW];

    // XCD-aware order: consecutive segments of a strip land on the same XCD
    const int L = (int)(blockIdx.x % 8) * G.chunk + (int)(blockIdx.x / 8);
    if (L >= G.nwg) return;
    int strip, ys0, ys1;
    if (G.table) {
        const int4 d = G.table[L];
        if constexpr (WX && TW > 64) {
            if (d.x < 0) {   // TW/64 independent single-wave tasks next to the x walls
                wall_tasks<TW, WY, PLK, PF, UNI, FF>(K, fin, fout, gyp, G.table[G.nwg + (TW / 64) * (-1 - d.x) +
                                                                                  (int)(threadIdx.x >> 6)], xs);
                return;
            }
        }
        strip = d.x;
        ys0 = d.y;
        ys1 = d.z;
    } else {
        // equal segments (products stay below 2^31 for any grid the ABI accepts)
        strip = L / G.nsegs;
        const int seg = L - strip * G.nsegs;
        ys0 = (int)((unsigned)(seg * K.ny) / (unsigned)G.nsegs);
        ys1 = (int)((unsigned)((seg + 1) * K.ny) / (unsigned)G.nsegs);
    }
    const int xs0 = G.xoff + (int)((unsigned)(strip * G.xspan) / (unsigned)G.nstrips);
    const int xs1 = G.xoff + (int)((unsigned)((strip + 1) * G.xspan) / (unsigned)G.nstrips);

    if constexpr (WX || WY) {
        // A segment whose march (columns xs0-4..xs1+3, rows ys0-4..ys1+3) stays
        // more than 4 nodes away from every wall meets no wall rule, ghost node
        // or wrap: the wall-free march computes exactly the same values with
        // less code and fewer live registers.
        // Likewise a segment near walls of one axis only runs the march that
        // handles that axis alone.
        const bool near_x = WX && (xs0 <= 8 || xs1 >= K.nx - 8);
        const bool near_y = WY && (ys0 <= 8 || ys1 >= K.ny - 8);
        if (!near_x && !near_y) {
            fused_march<TW, false, false, PLK, PF, UNI, FF>(K, fin, fout, gyp, xs0, xs1, ys0, ys1, xs, (int)threadIdx.x);
            return;
        }
        if constexpr (WX && WY) {
            if (!near_y) {
                fused_march<TW, true, false, PLK, PF, UNI, FF>(K, fin, fout, gyp, xs0, xs1, ys0, ys1, xs, (int)threadIdx.x);
                return;
            }
            if (!near_x) {
                fused_march<TW, false, true, PLK, PF, UNI, FF>(K, fin, fout, gyp, xs0, xs1, ys0, ys1, xs, (int)threadIdx.x);
                return;
            }
        }
    }
    fused_march<TW, WX, WY, PLK, PF, UNI, FF>(K, fin, fout, gyp, xs0, xs1, ys0, ys1, xs, (int)threadIdx.x);
}

// Batched step: table entry L = (strip, ys0, ys1, instance); every instance
// is periodic on a uniform grid with its own constants and state offset, cut
// into strips of TW - 8 output columns as the plan cuts them.
template <int TW, int PLK, int PF>
__global__ __launch_bounds__(TW) void k_fused_batch(const BatchInst* __restrict__ insts, const int4* __restrict__ table,
                                                    int nwg, int chunk, const double* __restrict__ fin,
                                                    double* __restrict__ fout)
{
    __shared__ double xs[4][9][TW];
    const int L = (int)(blockIdx.x % 8) * chunk + (int)(blockIdx.x / 8);
    if (L >= nwg) return;
    const int4 d = table[L];
    const BatchInst& I = insts[d.w];
    const int nstrips = (I.K.nx + TW - 9) / (TW - 8);
    const int xs0 = (int)((unsigned)(d.x * I.K.nx) / (unsigned)nstrips);
    const int xs1 = (int)((unsigned)((d.x + 1) * I.K.nx) / (unsigned)nstrips);
    fused_march<TW, false, false, PLK, PF, true, false>(I.K, fin + I.off, fout + I.off, nullptr, xs0, xs1, d.y, d.z,
                                                          xs, (int)threadIdx.x);
}


// Launch of one kernel family: every wall combination of k_fused for one
// (TW, PLK, PF, UNI, FF).
template <int TW, int PLK, int PF, bool UNI, bool FF>
hipError_t launch_tw(const StepConsts& K, const FusedGrid& G, const double* fin, double* fout, hipStream_t s)
{
    const dim3 grid(G.chunk * 8), block(TW);
    if (K.bcx && K.bcy)
        hipLaunchKernelGGL((k_fused<TW, true, true, PLK, PF, UNI, FF>), grid, block, 0, s, K, fin, fout, K.gy, G);
    else if (K.bcx)
        hipLaunchKernelGGL((k_fused<TW, true, false, PLK, PF, UNI, FF>), grid, block, 0, s, K, fin, fout, K.gy, G);
    else if (K.bcy)
        hipLaunchKernelGGL((k_fused<TW, false, true, PLK, PF, UNI, FF>), grid, block, 0, s, K, fin, fout, K.gy, G);
    else
        hipLaunchKernelGGL((k_fused<TW, false, false, PLK, PF, UNI, FF>), grid, block, 0, s, K, fin, fout, K.gy, G);
    return hipGetLastError();
}

}  // namespace fusedk

// Every k_fused instantiation of one tile width and fluid model (PLK: the
// collision's viscosity law, a compile-time constant so that no uniform
// branch splits the march), chosen by prefetch depth (2 or 3 rows; a force
// field takes 2), grid mapping and force field.
template <int TW, int PLK>
hipError_t launch_fused_pl(const StepConsts& K, const fusedk::FusedGrid& G, int prefetch, const double* fin,
                           double* fout, hipStream_t s)
{
    using namespace fusedk;
    if constexpr (TW == 64) {
        if (K.ff) {   // force field: 64 lanes, prefetch 2
            if (K.uniform) return launch_tw<64, PLK, 2, true, true>(K, G, fin, fout, s);
            return launch_tw<64, PLK, 2, false, true>(K, G, fin, fout, s);
        }
    }
    if (K.ff) return hipErrorInvalidValue;
    if (prefetch >= 3) {
        if (K.uniform) return launch_tw<TW, PLK, 3, true, false>(K, G, fin, fout, s);
        return launch_tw<TW, PLK, 3, false, false>(K, G, fin, fout, s);
    }
    if (K.uniform) return launch_tw<TW, PLK, 2, true, false>(K, G, fin, fout, s);
    return launch_tw<TW, PLK, 2, false, false>(K, G, fin, fout, s);
}

// The families of one tile width, Newtonian (PLW false) or power law (both
// indices).  Each (TW, PLW) pair is instantiated in a translation unit of its
// own (mdf_fused_w*.hip) so that the six compile in parallel.
template <int TW, bool PLW>
hipError_t launch_fused_family(const StepConsts& K, const fusedk::FusedGrid& G, int prefetch, const double* fin,
                               double* fout, hipStream_t s)
{
    if constexpr (!PLW) {
        return launch_fused_pl<TW, PL_NEWTON>(K, G, prefetch, fin, fout, s);
    } else {
        if (K.pl == PL_HALF) return launch_fused_pl<TW, PL_HALF>(K, G, prefetch, fin, fout, s);
        return launch_fused_pl<TW, PL_THREE_HALVES>(K, G, prefetch, fin, fout, s);
    }
}

// Batched step of one tile width and viscosity law.
template <int TW, int PLK>
hipError_t launch_batch_pl(const BatchInst* insts, const int4* table, int nwg, int prefetch, const double* fin,
                           double* fout, hipStream_t s)
{
    using namespace fusedk;
    const int chunk = (nwg + 7) / 8;
    const dim3 grid(chunk * 8), block(TW);
    if (prefetch >= 3)
        hipLaunchKernelGGL((k_fused_batch<TW, PLK, 3>), grid, block, 0, s, insts, table, nwg, chunk, fin, fout);
    else
        hipLaunchKernelGGL((k_fused_batch<TW, PLK, 2>), grid, block, 0, s, insts, table, nwg, chunk, fin, fout);
    return hipGetLastError();
}

// pl: the viscosity law the instances share (K.pl).
template <int TW, bool PLW>
hipError_t launch_batch_family(const BatchInst* insts, const int4* table, int nwg, int pl, int prefetch,
                               const double* fin, double* fout, hipStream_t s)
{
    if constexpr (!PLW) {
        return launch_batch_pl<TW, PL_NEWTON>(insts, table, nwg, prefetch, fin, fout, s);
    } else {
        if (pl == PL_HALF) return launch_batch_pl<TW, PL_HALF>(insts, table, nwg, prefetch, fin, fout, s);
        return launch_batch_pl<TW, PL_THREE_HALVES>(insts, table, nwg, prefetch, fin, fout, s);
    }
}

}  // namespace mdf
