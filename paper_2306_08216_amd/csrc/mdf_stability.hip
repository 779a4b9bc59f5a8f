// Von Neumann screen of the MDF-FDLBM step (host code; no device work).
//
// Sec. 3.1 analyses the stability of the method by the growth matrix of a
// Fourier mode of a small perturbation about a uniform state.  The screen
// here builds that matrix for the scheme as this library runs it: one full
// time step, Steps (1)-(4) of Sec. 2.2, linearised about the uniform state
// (U, V) on a periodic uniform grid (the uniform pressure does not enter the
// linearisation, f^eq being linear in P), for the Fourier mode
// exp(i (theta_x x/dx + theta_y y/dy)).  With J the Jacobian of the linear
// equilibrium (eq. 2.2.5) with respect to the 10 distributions (through
// u = sum f, v = sum g and the pressure identity), R_k the collision pair of
// rates (s, s') (a, b or q of Steps (1)-(3)), H_j = 1 - h c_j . D_j(theta) the
// half step of component j and Q_j = -dt c_j . D_j(theta) the full-step
// transport (D_j the symbol of the mixed difference of eqs. 2.2.12-2.2.13
// along the axis of c_j), the step maps the mode's amplitudes by
//   M = [J + R_a (I - J)] + diag(Q) [J + R_q (I - J)] diag(H) [J + R_b (I - J)],
// a 10 x 10 complex matrix.  The mode is stable when the spectral radius of
// M is at most 1; the radius is computed by Gelfand's formula, rho =
// lim ||M^(2^m)||^(2^-m), with 48 normalised squarings.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>

#include "../../include/mdf.h"

namespace {

using cplx = std::complex<double>;
constexpr int N = 10;

struct Mat {
    cplx a[N][N];
};

Mat mul(const Mat& x, const Mat& y)
{
    Mat z;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < N; ++k) s += x.a[i][k] * y.a[k][j];
            z.a[i][j] = s;
        }
    return z;
}

double fro(const Mat& x)
{
    double s = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) s += std::norm(x.a[i][j]);
    return std::sqrt(s);
}

// spectral radius by Gelfand's formula with normalised repeated squaring
double spectral_radius(Mat m)
{
    double lognorm = 0.0;   // log of the scale of m^(2^k) divided by 2^k
    double weight = 1.0;
    for (int k = 0; k <= 48; ++k) {
        const double nrm = fro(m);
        if (!(nrm > 1e-300)) return 0.0;
        if (!std::isfinite(nrm)) return INFINITY;
        lognorm += weight * std::log(nrm);
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) m.a[i][j] /= nrm;
        if (k == 48) break;
        m = mul(m, m);
        weight *= 0.5;
    }
    return std::exp(lognorm);
}

// D2Q5 velocities (units of c); components q = alpha*5 + j
const int CX[5] = {0, 1, 0, -1, 0};
const int CY[5] = {0, 0, 1, 0, -1};

struct Screen {
    double c, cs2, w, kf, dt, h, hx, hy, eta;
    double a_s, a_p, b_s, b_p, q_s, q_p;
    double U, V;
    double J[N][N];   // d f^eq / d f at (U, V)

    void build_jacobian()
    {
        // moments of a perturbation: u' = sum_j f_j, v' = sum_j g_j,
        // P' = (sum_j c_jx f_j + c_jy g_j)/2 - U u' - V v' (pressure identity)
        double du[N] = {}, dv[N] = {}, dP[N] = {};
        for (int j = 0; j < 5; ++j) {
            du[j] = 1.0;
            dv[5 + j] = 1.0;
        }
        for (int q = 0; q < N; ++q)
            dP[q] = 0.5 * c * (q < 5 ? CX[q % 5] : CY[q % 5]) - U * du[q] - V * dv[q];
        // f^eq_{j,u} = w u + kf (c_jx (u u + P) + c_jy u v); f^eq_{j,v} = w v + kf (c_jx v u + c_jy (v v + P)),
        // with kf = w c / c_s^2 and c_j in units of c
        for (int q = 0; q < N; ++q)
            for (int j = 0; j < 5; ++j) {
                J[j][q] = w * du[q] + kf * (CX[j] * (2.0 * U * du[q] + dP[q]) + CY[j] * (U * dv[q] + V * du[q]));
                J[5 + j][q] = w * dv[q] + kf * (CX[j] * (V * du[q] + U * dv[q]) + CY[j] * (2.0 * V * dv[q] + dP[q]));
            }
    }

    // J + R_{k,kp} (I - J), R = kp I + (k - kp) P_c with (P_c g)_1 = -(P_c g)_3 = (g_1 - g_3)/2 etc.
    void collide_map(double k, double kp, double out[N][N]) const
    {
        double G[N][N];
        for (int i = 0; i < N; ++i)
            for (int q = 0; q < N; ++q) G[i][q] = (i == q ? 1.0 : 0.0) - J[i][q];
        const double d = 0.5 * (k - kp);
        for (int a = 0; a < 2; ++a)
            for (int q = 0; q < N; ++q) {
                double g[5];
                for (int j = 0; j < 5; ++j) g[j] = G[5 * a + j][q];
                const double dx = d * (g[1] - g[3]), dy = d * (g[2] - g[4]);
                const double r[5] = {kp * g[0], kp * g[1] + dx, kp * g[2] + dy, kp * g[3] - dx, kp * g[4] - dy};
                for (int j = 0; j < 5; ++j) out[5 * a + j][q] = J[5 * a + j][q] + r[j];
            }
    }

    // c_j . D_j(theta) for component j with the mixed scheme of eqs. 2.2.12-2.2.13
    cplx transport_symbol(int j, double tx, double ty) const
    {
        if (j == 0) return 0.0;
        const bool xaxis = CX[j] != 0;
        const int sg = xaxis ? CX[j] : CY[j];
        const double th = xaxis ? tx : ty, dd = xaxis ? hx : hy;
        const cplx e1 = std::polar(1.0, th), em1 = std::polar(1.0, -th);
        const cplx e2 = std::polar(1.0, 2.0 * th), em2 = std::polar(1.0, -2.0 * th);
        cplx D;
        if (sg > 0)
            D = (eta * (e1 - em1) + (1.0 - eta) * (3.0 - 4.0 * em1 + em2)) / (2.0 * dd);
        else
            D = (eta * (e1 - em1) - (1.0 - eta) * (3.0 - 4.0 * e1 + e2)) / (2.0 * dd);
        return c * double(sg) * D;
    }

    double radius(double tx, double ty) const
    {
        double Lh[N][N], Lb[N][N], L3[N][N];
        collide_map(a_s, a_p, Lh);
        collide_map(b_s, b_p, Lb);
        collide_map(q_s, q_p, L3);
        cplx H[N], Q[N];
        for (int q = 0; q < N; ++q) {
            const cplx s = transport_symbol(q % 5, tx, ty);
            H[q] = 1.0 - h * s;
            Q[q] = -dt * s;
        }
        // M = Lh + diag(Q) L3 diag(H) Lb
        Mat M;
        for (int i = 0; i < N; ++i)
            for (int q = 0; q < N; ++q) {
                cplx s = 0.0;
                for (int k = 0; k < N; ++k) s += L3[i][k] * H[k] * Lb[k][q];
                M.a[i][q] = Lh[i][q] + Q[i] * s;
            }
        return spectral_radius(M);
    }
};

}  // namespace

extern "C" mdf_status mdf_stability(const mdf_params* p, double u0, double v0, int32_t nk, double* rho, double* worst)
{
    if (!p || nk < 1 || nk > 4096 || !worst) return MDF_EINVAL;
    if (!(p->nu > 0.0) || !(p->cfl > 0.0) || !(p->c > 0.0) || !(p->eta >= 0.0 && p->eta <= 1.0) ||
        !(p->s_ratio > 0.0) || p->nx < 1 || p->ny < 1 || !(p->lx > 0.0) || !(p->ly > 0.0) || p->pl_n != 1.0 ||
        !std::isfinite(u0) || !std::isfinite(v0))
        return MDF_EINVAL;
    Screen S{};
    S.c = p->c;
    S.w = 0.2;
    S.cs2 = 0.4 * p->c * p->c;
    S.kf = S.w * p->c / S.cs2;
    S.hx = p->lx / p->nx;   // periodic spacing (the screen is a periodic analysis)
    S.hy = p->ly / p->ny;
    S.dt = p->cfl * (S.hx < S.hy ? S.hx : S.hy) / p->c;
    S.h = 0.5 * S.dt;
    S.eta = p->eta;
    const double s = S.cs2 / p->nu, sp = p->s_ratio * s;
    auto a = [&](double sig) { return (1.0 - 0.5 * sig * S.dt) / (1.0 + 0.5 * sig * S.dt); };
    S.a_s = a(s);
    S.a_p = a(sp);
    S.b_s = 0.25 * (1.0 + 3.0 * S.a_s);
    S.b_p = 0.25 * (1.0 + 3.0 * S.a_p);
    S.q_s = 1.0 / (1.0 + 0.25 * s * S.dt);
    S.q_p = 1.0 / (1.0 + 0.25 * sp * S.dt);
    S.U = u0;
    S.V = v0;
    S.build_jacobian();
    const double pi = 3.14159265358979323846;
    worst[0] = -1.0;
    worst[1] = worst[2] = 0.0;
    for (int iy = 0; iy < nk; ++iy)
        for (int ix = 0; ix < nk; ++ix) {
            // theta on (-pi, pi]: nk points per axis including pi
            const double tx = -pi + 2.0 * pi * (ix + 1) / nk, ty = -pi + 2.0 * pi * (iy + 1) / nk;
            const double r = S.radius(tx, ty);
            if (rho) rho[iy * nk + ix] = r;
            if (!(r <= worst[0])) {
                worst[0] = r;
                worst[1] = tx;
                worst[2] = ty;
            }
        }
    return MDF_OK;
}
