// Fused single-pass MDF-FDLBM time step, one wave per velocity component.
//
// The two distribution sets of the method (the u and v equations, Remark 1)
// are coupled only through the moments u, v, P in the equilibrium
// (eq. 2.2.5) -- and, for a power-law fluid, through the strain rate that sets
// the local viscosity.  A workgroup therefore runs two waves on the same
// 64-column strip: wave 0 advances the u set, wave 1 the v set, and at each of
// the two collisions per row they swap two partial moments per node through
// LDS (sum_j phi_j and the diagonal first moment; plus the two off-axis
// non-equilibrium first moments for a power law).  Each wave holds half the
// state of a one-wave-per-strip design, which leaves room for two or three
// waves per SIMD to hide memory and dependency latency.
//
// Per row k entering the march (own set only):
//   A   load f_hat(k); Step (1) collision -> f_hat^+(k), f_bar^+(k)     (eqs. 2.2.14-15)
//   A'  x-neighbours of f_bar^+ through LDS; x part of the half step of row k
//   B   y part of the half step of row m = k-2 (4-row register window);
//       Step (3) collision -> f(t+h)(m)                                (eqs. 2.3.25, 2.2.16)
//   B'  x-neighbours of f(t+h); x part of Step (4) for row m -> store
//   C   y part of Step (4) for row r = k-4 -> store                   (eq. 2.3.24)
// Rings are indexed by (row - first row) & 3 and the march is unrolled by 4.
// Walls: the wall rule (non-equilibrium extrapolation from the two inward
// neighbours) is applied to f_bar^+ and f(t+h) inside the march and the
// quadratic ghost node is used beyond a wall; wall nodes of f_hat(t+dt) are
// left to the host-side pass that follows each mdf_step call.
#include <type_traits>

#include "mdf_device.hpp"
#include "mdf_internal.hpp"

namespace mdf {

namespace {

constexpr int TW2 = 64;   // lanes (columns) per strip, 56 output columns

struct Grid2 {
    int nstrips, nsegs, chunk, nwg;
    const int4* table;   // (strip, ys0, ys1, 0) per workgroup, or null: nsegs equal segments per strip
};

// equilibrium component j of set a at the moments (u, v, P) (eq. 2.2.5)
__device__ __forceinline__ double feq_j(const StepConsts& K, int a, int j, double u, double v, double P)
{
    const double ua = a == 0 ? u : v;
    if (j == 0) return K.w * ua;
    const bool xax = (j == 1 || j == 3);
    const double flux = xax ? (a == 0 ? u * u + P : v * u) : (a == 0 ? u * v : v * v + P);
    return (j == 1 || j == 2) ? K.w * ua + K.kf * flux : K.w * ua - K.kf * flux;
}

// wall rule for component j of set a from the inward neighbours n1, n2
__device__ __forceinline__ double wall_j(const StepConsts& K, int a, int j, double p1, double p2, const double* m1,
                                         const double* m2, double uw)
{
    const double e1 = feq_j(K, a, j, m1[0], m1[1], m1[2]);
    const double e2 = feq_j(K, a, j, m2[0], m2[1], m2[2]);
    const double ew = feq_j(K, a, j, uw, 0.0, m1[2]);
    return ew + 2.0 * (p1 - e1) - (p2 - e2);
}

__device__ __forceinline__ int lc(int l) { return l < 0 ? 0 : (l >= TW2 ? TW2 - 1 : l); }

// x-neighbours (offsets -2..2) of the two exchanged components (j = 1, 3) of
// set a from X = [j1, j3, g1, g3, P][lane] with g = f - f^eq; at x walls the
// wall column takes the wall rule f_w = f^eq_w + 2 g(n1) - g(n2), where f^eq at
// the wall (u = v = 0, P = P(n1)) is +-kf P for the u set and 0 for the v
// set, and the column beyond it the ghost node.  n1 and n2 are fixed columns,
// read by every lane at one LDS address; the lanes next to the wall select.
template <bool WX>
__device__ __forceinline__ void x_nb(const StepConsts& K, const double (*X)[TW2], int a, int lane, int x,
                                     double nb[2][5], bool wall_strip)
{
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int d = -2; d <= 2; ++d) nb[c][d + 2] = X[c][lc(lane + d)];
    if (WX && wall_strip) {
        const int x0 = __builtin_amdgcn_readfirstlane(x - lane);   // column of lane 0
        if (x0 <= 2) {   // the strip holds column 1 or 2
            const int l1 = lc(1 - x0), l2 = lc(2 - x0);
            const double kp = a == 0 ? K.kf * X[4][l1] : 0.0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double w0 = (c == 0 ? kp : -kp) + 2.0 * X[2 + c][l1] - X[2 + c][l2];
                const double gh = ghost(w0, X[c][l1], X[c][l2]);
                nb[c][1] = x == 1 ? w0 : nb[c][1];
                nb[c][0] = x == 1 ? gh : (x == 2 ? w0 : nb[c][0]);
            }
        }
        if (x0 + TW2 - 1 >= K.nx - 3) {   // the strip holds column nx-3 or nx-2
            const int l1 = lc(K.nx - 2 - x0), l2 = lc(K.nx - 3 - x0);
            const double kp = a == 0 ? K.kf * X[4][l1] : 0.0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double w0 = (c == 0 ? kp : -kp) + 2.0 * X[2 + c][l1] - X[2 + c][l2];
                const double gh = ghost(w0, X[c][l1], X[c][l2]);
                nb[c][3] = x == K.nx - 2 ? w0 : nb[c][3];
                nb[c][4] = x == K.nx - 2 ? gh : (x == K.nx - 3 ? w0 : nb[c][4]);
            }
        }
    }
}

// Moments of a node for the collision of one set: the two waves swap their
// partial sums through LDS (M = [quantity][set][lane]); returns (u, v, P) in m,
// the own set's f^eq in e and, for a power law, the squared non-equilibrium
// strain magnitude 2 S^:S^ of the collided field.
template <bool PLW>
__device__ __forceinline__ void collide_moments(const StepConsts& K, double (*M)[2][TW2], int a, int lane,
                                                const double* phi, double* m, double* e, double& gam_sq)
{
    const double s = ((phi[0] + phi[1]) + (phi[2] + phi[3])) + phi[4];
    const double q = K.c * (a == 0 ? phi[1] - phi[3] : phi[2] - phi[4]);
    if constexpr (kPoisonLds) {
#pragma unroll
        for (int c = 0; c < 4; ++c) M[c][a][lane] = lds_poison_value();
    }
    M[0][a][lane] = s;
    M[1][a][lane] = q;
    lds_barrier();
    const double so = M[0][1 - a][lane], qo = M[1][1 - a][lane];
    const double u = a == 0 ? s : so, v = a == 0 ? so : s;
    m[0] = u;
    m[1] = v;
    m[2] = 0.5 * ((a == 0 ? q + qo : qo + q) - (u * u + v * v));
#pragma unroll
    for (int j = 0; j < 5; ++j) e[j] = feq_j(K, a, j, u, v, m[2]);
    gam_sq = 0.0;
    if (PLW) {
        const double mx = K.c * ((phi[1] - e[1]) - (phi[3] - e[3]));
        const double my = K.c * ((phi[2] - e[2]) - (phi[4] - e[4]));
        M[2][a][lane] = mx;
        M[3][a][lane] = my;
        lds_barrier();
        const double mxo = M[2][1 - a][lane], myo = M[3][1 - a][lane];
        const double mxx = a == 0 ? mx : mxo, mxy = a == 0 ? my : myo;
        const double myx = a == 0 ? mxo : mx, myy = a == 0 ? myo : my;
        const double s12 = 0.5 * (mxy + myx);
        gam_sq = 2.0 * (mxx * mxx + myy * myy + 2.0 * s12 * s12);
    }
}

// out = f^eq + R_{k,k'}(phi - f^eq) for one set
__device__ __forceinline__ void relax5(const double* phi, const double* e, Relax r, double* o)
{
    const double dk = 0.5 * (r.k - r.kp);
    const double g0 = phi[0] - e[0], g1 = phi[1] - e[1], g2 = phi[2] - e[2], g3 = phi[3] - e[3], g4 = phi[4] - e[4];
    const double dx = dk * (g1 - g3), dy = dk * (g2 - g4);
    o[0] = e[0] + r.kp * g0;
    o[1] = e[1] + (r.kp * g1 + dx);
    o[3] = e[3] + (r.kp * g3 - dx);
    o[2] = e[2] + (r.kp * g2 + dy);
    o[4] = e[4] + (r.kp * g4 - dy);
}

// The march of one strip segment: output columns xs0..xs1-1, rows ys0..ys1-1.
template <bool WX, bool WY, bool PLW, int PF, bool UNI>
__device__ __forceinline__ void fused2_march(const StepConsts& K, const double* __restrict__ fin,
                                             double* __restrict__ fout, int xs0, int xs1, int ys0, int ys1,
                                             double (*mom)[4][2][TW2], double (*xch)[2][5][TW2])
{
    const int lane = threadIdx.x & (TW2 - 1);
    const int a = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // own set, uniform per wave
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
    // and segments whose march reaches rows 0-2 or ny-3..ny-1 run wall code
    const bool wall_strip = WX && (xs0 <= 8 || xs1 >= K.nx - 8);
    const bool wall_seg = WY && (ys0 <= 8 || ys1 >= K.ny - 8);

    const double gxl = UNI ? 0.0 : K.gx[xg];
    const Stencil SXh = UNI ? stencil_of(K.sh[0]) : make_stencil(K, K.lam_h * gxl, true);
    const Stencil SXd = UNI ? stencil_of(K.sd[0]) : make_stencil(K, K.lam_dt * gxl, false);
    auto y_stencil_h = [&](int row) -> Stencil {
        return UNI ? stencil_of(K.sh[1]) : make_stencil(K, K.lam_h * K.gy[row], true);
    };
    auto y_stencil_d = [&](int row) -> Stencil {
        return UNI ? stencil_of(K.sd[1]) : make_stencil(K, K.lam_dt * K.gy[row], false);
    };
    const double hwf = a == 0 ? K.hwf[0] : K.hwf[1];
    const double dwf = a == 0 ? K.dwf[0] : K.dwf[1];

    auto wrap_y = [&](int k) -> int {
        if (WY) return k;
        return k < 0 ? k + K.ny : (k >= K.ny ? k - K.ny : k);
    };
    auto row_ok = [&](int k) -> bool { return WY ? (k >= 0 && k < K.ny) : true; };
    // the own set of this lane's node in row k: j = 0, 1, 3 in the x-part block,
    // j = 2, 4 in the y-part block of the row
    auto xo = [&](int k) -> size_t { return xpart_off(K.pitch, xg, wrap_y(k)) + 3 * (size_t)a; };
    auto yo = [&](int k) -> size_t { return ypart_off(K.pitch, xg, wrap_y(k)) + 2 * (size_t)a; };

    // rows kbeg..kend enter the march; it is padded to a whole number of
    // 4-row groups (the padding rows reach no output) so that the unrolled loop
    // has no partial group and the row loads are unconditional
    const int kbeg = ys0 - 4, kend = ys1 + 3;
    const int kpad = kbeg + ((kend - kbeg + 4) & ~3) - 1;

    // Every prefetch load is issued unconditionally from an in-range row (rows
    // past kend repeat row kend; rows beyond a y wall repeat the wall row) so
    // that the compiler can count the loads in flight and wait only for the row
    // being consumed; rows outside the domain are replaced by zero at use.
    double pre[4][5];
    auto load_row = [&](int k, double* dst) {
        int kl = k > kend ? kend : k;
        if (WY) kl = kl < 0 ? 0 : (kl >= K.ny ? K.ny - 1 : kl);
        const double* px = fin + xo(kl);
        const double* py = fin + yo(kl);
        dst[0] = px[0];
        dst[1] = px[1];
        dst[3] = px[2];
        dst[2] = py[0];
        dst[4] = py[1];
    };

    double W2[4], W4[4], F2[4], F4[4], Qy[4][2], Qx[2][3], Qb[2][3];
    double ub_prev[3] = {0, 0, 0}, uf_prev[3] = {0, 0, 0}, pend_b[2] = {0, 0}, pend_f[2] = {0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) W2[i] = W4[i] = F2[i] = F4[i] = Qy[i][0] = Qy[i][1] = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) Qx[i][q] = Qb[i][q] = 0.0;

#pragma unroll
    for (int i = 0; i < PF; ++i) load_row(kbeg + i, pre[i]);

    auto body = [&](auto PC, int k) {
        constexpr int P = decltype(PC)::value;
        constexpr int S1 = (P + 3) & 3, S2 = (P + 2) & 3, S3 = (P + 1) & 3;   // rows k-1, k-2, k-3
        double cur[5];
        const bool live = row_ok(k);
#pragma unroll
        for (int j = 0; j < 5; ++j) cur[j] = live ? pre[P][j] : 0.0;
        load_row(k + PF, pre[(P + PF) & 3]);

        // ---- A: Step (1) on row k ----
        double fbp[5], fhp[5], ub[3], gb[2];
        {
            double e[5], gam;
            collide_moments<PLW>(K, mom[0], a, lane, cur, ub, e, gam);
            Relax ra, rb;
            if (PLW) {
                relax_ab_nu(K, powerlaw_nu_sq(K, gam, K.theta1), ra, rb);
            } else {
                ra = Relax{K.a_s, K.a_p};
                rb = Relax{K.b_s, K.b_p};
            }
            relax5(cur, e, rb, fbp);
            gb[0] = fbp[1] - e[1];
            gb[1] = fbp[3] - e[3];
            if (k >= ys0 && k < ys1) {
                relax5(cur, e, ra, fhp);
            } else {
#pragma unroll
                for (int j = 0; j < 5; ++j) fhp[j] = 0.0;
            }
        }
        double b2 = fbp[2];
        W4[P] = fbp[4];
        if (WY && wall_seg) {
            if (k == 2) {   // bottom wall row 0 from rows 1 and 2
                W2[S2] = wall_j(K, a, 2, W2[S1], b2, ub_prev, ub, 0.0);
                W4[S2] = wall_j(K, a, 4, W4[S1], W4[P], ub_prev, ub, 0.0);
            }
            if (k == K.ny - 2) {   // top wall row ny-1 from rows ny-2 and ny-3, used next row
                pend_b[0] = wall_j(K, a, 2, b2, W2[S1], ub, ub_prev, K.lid_u);
                pend_b[1] = wall_j(K, a, 4, W4[P], W4[S1], ub, ub_prev, K.lid_u);
            }
            if (k == K.ny - 1) {
                b2 = pend_b[0];
                W4[P] = pend_b[1];
            }
        }

        // ---- A': x part of the half step for row k ----
        double bx[3];
        {
            double(*X)[TW2] = xch[0][a];
            if constexpr (kPoisonLds) {
#pragma unroll
                for (int c = 0; c < 5; ++c) X[c][lane] = lds_poison_value();
            }
            X[0][lane] = fbp[1];
            X[1][lane] = fbp[3];
            if (WX && wall_strip) {
                X[2][lane] = gb[0];
                X[3][lane] = gb[1];
                X[4][lane] = ub[2];
            }
            lds_barrier();
            double nb[2][5];
            x_nb<WX>(K, X, a, lane, x, nb, wall_strip);
            bx[0] = fbp[0] + hwf;
            bx[1] = upd_pos(SXh, hwf, nb[0][0], nb[0][1], nb[0][2], nb[0][3]);
            bx[2] = upd_neg(SXh, hwf, nb[1][1], nb[1][2], nb[1][3], nb[1][4]);
        }

        // ---- B: half step (y part) and Step (3) on row m = k-2 ----
        const int m = k - 2;
        const bool needB = (m >= ys0 - 2) && (m < ys1 + 2) && (WY ? (m >= 1 && m <= K.ny - 2) : true);
        double f2c = 0.0;
        double fm[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, uf[3] = {0.0, 0.0, 0.0}, gf[2] = {0.0, 0.0};
        if (needB) {
            const Stencil SYh = y_stencil_h(wrap_y(m));
            double a2[4] = {W2[P], W2[S3], W2[S2], W2[S1]};   // rows m-2 .. m+1
            double a4[4] = {W4[S3], W4[S2], W4[S1], W4[P]};   // rows m-1 .. m+2
            if (WY && wall_seg && m == 1) a2[0] = ghost(a2[1], a2[2], a2[3]);
            if (WY && wall_seg && m == K.ny - 2) a4[3] = ghost(a4[2], a4[1], a4[0]);
            double fb[5];
            fb[0] = Qb[P & 1][0];
            fb[1] = Qb[P & 1][1];
            fb[3] = Qb[P & 1][2];
            fb[2] = upd_pos(SYh, hwf, a2[0], a2[1], a2[2], a2[3]);
            fb[4] = upd_neg(SYh, hwf, a4[0], a4[1], a4[2], a4[3]);
            double e[5], gam;
            collide_moments<PLW>(K, mom[1], a, lane, fb, uf, e, gam);
            Relax rq;
            if (PLW) {
                rq = relax_q_nu(K, powerlaw_nu_sq(K, gam, K.theta3));
            } else {
                rq = Relax{K.q_s, K.q_p};
            }
            relax5(fb, e, rq, fm);
            gf[0] = fm[1] - e[1];
            gf[1] = fm[3] - e[3];
            F4[S2] = fm[4];
            f2c = fm[2];
        }
        if (WY && wall_seg) {
            if (m == 2) {   // bottom wall row 0 of f(t+h)
                F2[P] = wall_j(K, a, 2, F2[S3], f2c, uf_prev, uf, 0.0);
                F4[P] = wall_j(K, a, 4, F4[S3], F4[S2], uf_prev, uf, 0.0);
            }
            if (m == K.ny - 2) {
                pend_f[0] = wall_j(K, a, 2, f2c, F2[S3], uf, uf_prev, K.lid_u);
                pend_f[1] = wall_j(K, a, 4, F4[S2], F4[S3], uf, uf_prev, K.lid_u);
            }
            if (m == K.ny - 1) {
                f2c = pend_f[0];
                F4[S2] = pend_f[1];
            }
        }

        // ---- B': x part of Step (4) on row m ----
        const bool outm = needB && (m >= ys0) && (m < ys1);
        if (outm) {
            double(*X)[TW2] = xch[1][a];
            if constexpr (kPoisonLds) {
#pragma unroll
                for (int c = 0; c < 5; ++c) X[c][lane] = lds_poison_value();
            }
            X[0][lane] = fm[1];
            X[1][lane] = fm[3];
            if (WX && wall_strip) {
                X[2][lane] = gf[0];
                X[3][lane] = gf[1];
                X[4][lane] = uf[2];
            }
            lds_barrier();
            double nb[2][5];
            x_nb<WX>(K, X, a, lane, x, nb, wall_strip);
            if (outc) {
                double* o = fout + xo(m);
                o[0] = Qx[P & 1][0] + dwf;
                o[1] = upd_pos(SXd, Qx[P & 1][1] + dwf, nb[0][0], nb[0][1], nb[0][2], nb[0][3]);
                o[2] = upd_neg(SXd, Qx[P & 1][2] + dwf, nb[1][1], nb[1][2], nb[1][3], nb[1][4]);
            }
        } else {
            lds_barrier();   // keeps the LDS buffers strictly alternating
        }

        // ---- C: y part of Step (4) on row r = k-4 ----
        const int r = k - 4;
        const bool outr = (r >= ys0) && (r < ys1) && (WY ? (r >= 1 && r <= K.ny - 2) : true);
        if (outr && outc) {
            const Stencil SYd = y_stencil_d(wrap_y(r));
            double c2[4] = {F2[S2], F2[S1], F2[P], F2[S3]};   // rows r-2 .. r+1
            double c4[4] = {F4[S1], F4[P], F4[S3], F4[S2]};   // rows r-1 .. r+2
            if (WY && wall_seg && r == 1) c2[0] = ghost(c2[1], c2[2], c2[3]);
            if (WY && wall_seg && r == K.ny - 2) c4[3] = ghost(c4[2], c4[1], c4[0]);
            double* o = fout + yo(r);
            o[0] = upd_pos(SYd, Qy[P][0] + dwf, c2[0], c2[1], c2[2], c2[3]);
            o[1] = upd_neg(SYd, Qy[P][1] + dwf, c4[0], c4[1], c4[2], c4[3]);
        }

        // ---- ring pushes ----
        W2[P] = b2;
        Qy[P][0] = fhp[2];
        Qy[P][1] = fhp[4];
        Qx[P & 1][0] = fhp[0];
        Qx[P & 1][1] = fhp[1];
        Qx[P & 1][2] = fhp[3];
        Qb[P & 1][0] = bx[0];
        Qb[P & 1][1] = bx[1];
        Qb[P & 1][2] = bx[2];
        F2[S2] = f2c;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            ub_prev[q] = ub[q];
            uf_prev[q] = needB ? uf[q] : uf_prev[q];   // a select: a conditional store here lands in scratch
        }
    };

    for (int k = kbeg; k <= kpad; k += 4) {
        body(std::integral_constant<int, 0>{}, k);
        body(std::integral_constant<int, 1>{}, k + 1);
        body(std::integral_constant<int, 2>{}, k + 2);
        body(std::integral_constant<int, 3>{}, k + 3);
    }
}

template <bool WX, bool WY, bool PLW, int PF, bool UNI>
__global__ __launch_bounds__(2 * TW2) void k_fused2(StepConsts K, const double* __restrict__ fin,
                                                    double* __restrict__ fout, Grid2 G)
{
    __shared__ double mom[2][4][2][TW2];   // [collision][quantity][set][lane]
    __shared__ double xch[2][2][5][TW2];   // [exchange][set][j1 j3 g1 g3 P][lane]

    // XCD-aware order: consecutive segments of a strip land on the same XCD
    const int L = (int)(blockIdx.x % 8) * G.chunk + (int)(blockIdx.x / 8);
    if (L >= G.nwg) return;
    int strip, ys0, ys1;
    if (G.table) {
        const int4 d = G.table[L];
        strip = d.x;
        ys0 = d.y;
        ys1 = d.z;
    } else {
        strip = L / G.nsegs;
        const int seg = L - strip * G.nsegs;
        ys0 = (int)((unsigned)(seg * K.ny) / (unsigned)G.nsegs);
        ys1 = (int)((unsigned)((seg + 1) * K.ny) / (unsigned)G.nsegs);
    }
    const int xs0 = (int)((unsigned)(strip * K.nx) / (unsigned)G.nstrips);
    const int xs1 = (int)((unsigned)((strip + 1) * K.nx) / (unsigned)G.nstrips);

    if constexpr (WX || WY) {
        // a segment whose march stays more than 4 nodes away from every wall
        // meets no wall rule, ghost node or wrap: the wall-free march computes
        // exactly the same values with less code
        const bool near_x = WX && (xs0 <= 8 || xs1 >= K.nx - 8);
        const bool near_y = WY && (ys0 <= 8 || ys1 >= K.ny - 8);
        if (!near_x && !near_y) {
            fused2_march<false, false, PLW, PF, UNI>(K, fin, fout, xs0, xs1, ys0, ys1, mom, xch);
            return;
        }
        // near walls of one axis only: the march that handles that axis alone
        if constexpr (WX && WY) {
            if (!near_y) {
                fused2_march<true, false, PLW, PF, UNI>(K, fin, fout, xs0, xs1, ys0, ys1, mom, xch);
                return;
            }
            if (!near_x) {
                fused2_march<false, true, PLW, PF, UNI>(K, fin, fout, xs0, xs1, ys0, ys1, mom, xch);
                return;
            }
        }
    }
    fused2_march<WX, WY, PLW, PF, UNI>(K, fin, fout, xs0, xs1, ys0, ys1, mom, xch);
}

// Batched step: table entry L = (strip, ys0, ys1, instance); every instance
// is periodic on a uniform grid with its own constants and state offset.
template <bool PLW, int PF>
__global__ __launch_bounds__(2 * TW2) void k_fused2_batch(const BatchInst* __restrict__ insts,
                                                          const int4* __restrict__ table, int nwg, int chunk,
                                                          const double* __restrict__ fin, double* __restrict__ fout)
{
    __shared__ double mom[2][4][2][TW2];
    __shared__ double xch[2][2][5][TW2];
    const int L = (int)(blockIdx.x % 8) * chunk + (int)(blockIdx.x / 8);
    if (L >= nwg) return;
    const int4 d = table[L];
    const BatchInst& I = insts[d.w];
    const int xs0 = (int)((unsigned)(d.x * I.K.nx) / (unsigned)I.nstrips);
    const int xs1 = (int)((unsigned)((d.x + 1) * I.K.nx) / (unsigned)I.nstrips);
    fused2_march<false, false, PLW, PF, true>(I.K, fin + I.off, fout + I.off, xs0, xs1, d.y, d.z, mom, xch);
}

template <bool PLW, int PF, bool UNI>
hipError_t launch_bc(const StepConsts& K, const Grid2& G, const double* fin, double* fout, hipStream_t s)
{
    const dim3 grid(G.chunk * 8), block(2 * TW2);
    if (K.bcx && K.bcy)
        hipLaunchKernelGGL((k_fused2<true, true, PLW, PF, UNI>), grid, block, 0, s, K, fin, fout, G);
    else if (K.bcx)
        hipLaunchKernelGGL((k_fused2<true, false, PLW, PF, UNI>), grid, block, 0, s, K, fin, fout, G);
    else if (K.bcy)
        hipLaunchKernelGGL((k_fused2<false, true, PLW, PF, UNI>), grid, block, 0, s, K, fin, fout, G);
    else
        hipLaunchKernelGGL((k_fused2<false, false, PLW, PF, UNI>), grid, block, 0, s, K, fin, fout, G);
    return hipGetLastError();
}

template <int PF>
hipError_t launch_pf2(const StepConsts& K, const Grid2& G, const double* fin, double* fout, hipStream_t s)
{
    if (K.pl == PL_NEWTON) {
        if (K.uniform) return launch_bc<false, PF, true>(K, G, fin, fout, s);
        return launch_bc<false, PF, false>(K, G, fin, fout, s);
    }
    if (K.uniform) return launch_bc<true, PF, true>(K, G, fin, fout, s);
    return launch_bc<true, PF, false>(K, G, fin, fout, s);
}

}  // namespace

hipError_t launch_fused2_batch(const BatchInst* insts, const int4* table, int nwg, bool powerlaw, int prefetch,
                               const double* fin, double* fout, hipStream_t s)
{
    if (nwg <= 0) return hipErrorInvalidValue;
    const int chunk = (nwg + 7) / 8;
    const dim3 grid(chunk * 8), block(2 * TW2);
    if (powerlaw) {
        if (prefetch <= 2)
            hipLaunchKernelGGL((k_fused2_batch<true, 2>), grid, block, 0, s, insts, table, nwg, chunk, fin, fout);
        else
            hipLaunchKernelGGL((k_fused2_batch<true, 3>), grid, block, 0, s, insts, table, nwg, chunk, fin, fout);
    } else {
        if (prefetch <= 2)
            hipLaunchKernelGGL((k_fused2_batch<false, 2>), grid, block, 0, s, insts, table, nwg, chunk, fin, fout);
        else
            hipLaunchKernelGGL((k_fused2_batch<false, 3>), grid, block, 0, s, insts, table, nwg, chunk, fin, fout);
    }
    return hipGetLastError();
}

hipError_t launch_fused2(const StepConsts& K, FusedShape sh, const double* fin, double* fout, hipStream_t s)
{
    if (K.ff) return hipErrorInvalidValue;   // no force-field path in this kernel
    Grid2 G;
    const int wout = TW2 - 8;
    G.nstrips = (K.nx + wout - 1) / wout;
    if (sh.seg_h > 0) {
        G.nsegs = (K.ny + sh.seg_h - 1) / sh.seg_h;
        G.nwg = G.nstrips * G.nsegs;
        G.table = nullptr;
    } else {
        if (!sh.table || sh.nwg <= 0) return hipErrorInvalidValue;
        G.nsegs = 0;
        G.nwg = sh.nwg;
        G.table = sh.table;
    }
    G.chunk = (G.nwg + 7) / 8;
    if (sh.prefetch <= 2) return launch_pf2<2>(K, G, fin, fout, s);
    return launch_pf2<3>(K, G, fin, fout, s);
}

}  // namespace mdf
