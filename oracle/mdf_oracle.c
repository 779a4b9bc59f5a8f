/*
 * MDF-FDLBM CPU oracle -- TEST INFRASTRUCTURE ONLY (see mdf_oracle.h).
 *
 * Plain sequential FP64 loops, compiled with -O2 -ffp-contract=off.  The step
 * follows the four-step algorithm of Sec. 2.2 (Steps (1)-(4), eqs. 2.2.14-2.2.16)
 * with the simplified evolution equations of Remark 2 (eqs. 2.3.24-2.3.25), the
 * alpha = 0 equation dropped per Remark 1, the time step of eq. 3.1 and the
 * D2Q5 lattice of eq. 3.1.0.  Collision operators are built as dense 5x5
 * matrices exactly as the equations write them (the paper's "2 x 5 x 5"
 * cycles of Sec. 4.2); nothing is fused or reordered.
 *
 * The OpenMP build of this same file runs the node loops of each sub-step in
 * parallel; every node of a sub-step only reads the previous sub-step's
 * arrays, so the results are identical to the sequential build.
 *
 * Readings taken where the paper is silent or garbled:
 *  - c_s^2 follows from the second-moment condition of eq. 2.3.4 with w_j = 1/5;
 *  - the MRT matrix is M^-1 diag(s',s,s,s',s') M with an orthogonal D2Q5 basis;
 *  - eta multiplies the central part of the mixed scheme (eq. 2.2.12); the
 *    c < 0 upwind branch of eq. 2.2.13b uses Pi(chi + 2 dchi) as its last term;
 *  - walls use a non-equilibrium extrapolation, linear in the two inward
 *    neighbours (diagonal at corners), and a quadratic ghost node beyond a wall;
 *  - non-uniform grids use a separable mapping x = X(xi), d/dx = (1/X') d/dxi;
 *  - a power-law fluid takes nu = K gdot^(n-1) per node, with gdot from the
 *    non-equilibrium first moment of the field being collided (eq. 2.4.1).
 */
#include "mdf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 5
#define NPL 10

/* D2Q5 velocities in units of c and weights w_j = 1/5 (Sec. 3.1, eq. 3.1.0). */
static const double CX[NQ] = {0.0, 1.0, 0.0, -1.0, 0.0};
static const double CY[NQ] = {0.0, 0.0, 1.0, 0.0, -1.0};
static const double WJ[NQ] = {0.2, 0.2, 0.2, 0.2, 0.2};

struct orc_state {
    orc_params p;
    int nx, ny;
    size_t n;
    double c, cs2, dt, h;
    double *gx, *gy;          /* derivative scale 1/(X' dxi) at each node */
    double *met;              /* general mapping: d i/dx, d i/dy, d j/dx, d j/dy planes, or NULL */
    double *Fx, *Fy;          /* body force F_alpha at each node (eq. 2.2.6) */
    double *fhat;             /* state f_hat(t)            */
    double *fhat_plus;        /* f_hat^+(t)   (eq. 2.2.14) */
    double *fbar_plus;        /* f_bar^+(t)   (eq. 2.2.15) */
    double *fbar;             /* f_bar(t+h)   (eq. 2.2.11) */
    double *fmid;             /* f(t+h)       (eq. 2.2.16) */
    double *fnew;             /* f_hat(t+dt)  (eq. 2.3.24) */
    double mats[125];         /* Newtonian collision matrices */
    double *R;                /* mass source R at each node (eq. 2.1.1), or NULL */
    double kinv[4][25];       /* (I + kappa Lambda~)^-1 of the four stored forms (with R) */
    double kap[4];            /* their kappa: dt/2, h/2, -h/2, 0 */
    /* alpha = 0 distributions (rho0), when tracked: f_hat, f_hat^+, f_bar^+, f_bar, f, new */
    double *r0hat, *r0hatp, *r0barp, *r0bar, *r0mid, *r0new;
    /* momentum flux (u u + P, u v, v u, v v + P) at the last two steps, and at this one */
    double *q1, *q2, *qn;
    int nq;                   /* how many of q1, q2 hold values */
    int64_t steps;
};

/* stored forms phi = f + kappa Lambda~ (f - f^eq): f_hat (eq. 2.2.2), f_bar (eq. 2.2.9a),
 * f_bar^+ (eq. 2.2.9b), f itself */
enum { FORM_HAT = 0, FORM_BAR = 1, FORM_BARPLUS = 2, FORM_F = 3 };

/* ------------------------------------------------------------------ */
/* small dense linear algebra                                          */
/* ------------------------------------------------------------------ */

/* Gauss-Jordan inverse with partial pivoting of a 5x5 row-major matrix. */
static void inv5(const double* A, double* Ainv)
{
    double a[NQ][2 * NQ];
    for (int i = 0; i < NQ; ++i)
        for (int k = 0; k < NQ; ++k) {
            a[i][k] = A[i * NQ + k];
            a[i][NQ + k] = (i == k) ? 1.0 : 0.0;
        }
    for (int col = 0; col < NQ; ++col) {
        int piv = col;
        for (int r = col + 1; r < NQ; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (piv != col)
            for (int k = 0; k < 2 * NQ; ++k) {
                double t = a[col][k];
                a[col][k] = a[piv][k];
                a[piv][k] = t;
            }
        double d = a[col][col];
        for (int k = 0; k < 2 * NQ; ++k) a[col][k] /= d;
        for (int r = 0; r < NQ; ++r) {
            if (r == col) continue;
            double m = a[r][col];
            if (m == 0.0) continue;
            for (int k = 0; k < 2 * NQ; ++k) a[r][k] -= m * a[col][k];
        }
    }
    for (int i = 0; i < NQ; ++i)
        for (int k = 0; k < NQ; ++k) Ainv[i * NQ + k] = a[i][NQ + k];
}

static void mul5(const double* A, const double* B, double* C)
{
    for (int i = 0; i < NQ; ++i)
        for (int k = 0; k < NQ; ++k) {
            double s = 0.0;
            for (int m = 0; m < NQ; ++m) s += A[i * NQ + m] * B[m * NQ + k];
            C[i * NQ + k] = s;
        }
}

/* y = A x */
static void mv5(const double* A, const double* x, double* y)
{
    for (int i = 0; i < NQ; ++i) {
        double s = 0.0;
        for (int k = 0; k < NQ; ++k) s += A[i * NQ + k] * x[k];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* the method's local pieces                                           */
/* ------------------------------------------------------------------ */

/* c_s^2 from the second-moment condition of eq. 2.3.4:
 * sum_j w_j c_jx c_jx = c_s^2 (the third identity with u_alpha factored out). */
static double lattice_cs2(double c)
{
    double s = 0.0;
    for (int j = 0; j < NQ; ++j) s += WJ[j] * (c * CX[j]) * (c * CX[j]);
    return s;
}

/* Moments of any stored form phi (f, f_hat, f_hat^+, f_bar^+, f_bar):
 * u_alpha = sum_j phi_{j,alpha} (eq. 2.3.4, first identity; the collision
 * matrix keeps the zeroth moment, eq. 2.2.4) and the pressure of eq. 2.3.23
 * with R = 0 and d = 2:  P = (sum_alpha sum_j c_{j,alpha} phi_{j,alpha} - |u|^2)/2.
 * Eq. 2.3.23 is written for f; since P is defined so that the trace of the
 * non-equilibrium first moment vanishes, and every stored form differs from f
 * by a multiple of Lambda~ (f - f^eq) whose first moment is s times that of
 * f - f^eq (eq. 2.2.4), the same sum evaluated on any stored form gives the
 * same P.  A test checks this against the explicit f of eq. 2.2.2. */
void orc_node_moments(double c, const double* phi, double* u, double* v, double* P)
{
    double su = 0.0, sv = 0.0, q = 0.0;
    for (int j = 0; j < NQ; ++j) {
        su += phi[j];
        sv += phi[NQ + j];
    }
    for (int j = 0; j < NQ; ++j) {
        q += c * CX[j] * phi[j];       /* alpha = 1: c_{j,x} f_{j,1} */
        q += c * CY[j] * phi[NQ + j];  /* alpha = 2: c_{j,y} f_{j,2} */
    }
    *u = su;
    *v = sv;
    *P = 0.5 * (q - (su * su + sv * sv));
}

/* Linear equilibrium of eq. 2.2.5:
 * f^eq_{j,alpha} = w_j [u_alpha + c_j . (u_alpha u + P E_alpha) / c_s^2]. */
void orc_feq(double c, double u, double v, double P, double* out)
{
    double cs2 = lattice_cs2(c);
    double ua[2] = {u, v};
    for (int a = 0; a < 2; ++a) {
        double flux_x = ua[a] * u + (a == 0 ? P : 0.0);
        double flux_y = ua[a] * v + (a == 1 ? P : 0.0);
        for (int j = 0; j < NQ; ++j) {
            double cdot = c * CX[j] * flux_x + c * CY[j] * flux_y;
            out[a * NQ + j] = WJ[j] * (ua[a] + cdot / cs2);
        }
    }
}

/* Pressure of eq. 2.3.23 with the mass source R, at a node whose stored
 * distributions are phi = f + kappa Lambda~ (f - f^eq(u, P)):
 *   P = (sum_alpha sum_j c_{j,alpha} f_{j,alpha} + (c_s^2/s) R - |u|^2) / d,  d = 2,
 * where f itself follows from phi and P through
 *   f = (I + kappa Lambda~)^{-1} (phi + kappa Lambda~ f^eq(u, P))     (Minv below).
 * The definition is therefore an equation in P.  Its residual
 *   r(P) = P - (sum c f(P) + (c_s^2/s) R - |u|^2) / 2
 * is affine in P (f^eq is linear in P), so the root is r(0) / (r(0) - r(1)).
 * u and v are the zeroth moments of phi (Lambda~ keeps them, eq. 2.2.4), and
 * c_s^2/s = nu (eq. 2.3.14) for the Newtonian fluid this needs. */
static double solve_pressure(const orc_state* st, const double* phi, const double* Minv, double kappa, double R,
                             double u, double v)
{
    const double* Lt = st->mats; /* Lambda~ */
    double r[2];
    for (int k = 0; k < 2; ++k) {
        const double Ptry = (double)k;
        double fe[NPL], T = 0.0;
        orc_feq(st->c, u, v, Ptry, fe);
        for (int a = 0; a < 2; ++a) {
            double lf[NQ], rhs[NQ], f[NQ];
            mv5(Lt, fe + a * NQ, lf);
            for (int q = 0; q < NQ; ++q) rhs[q] = phi[a * NQ + q] + kappa * lf[q];
            mv5(Minv, rhs, f);
            for (int q = 0; q < NQ; ++q) T += st->c * (a == 0 ? CX[q] : CY[q]) * f[q];
        }
        r[k] = Ptry - 0.5 * (T + st->p.nu * R - (u * u + v * v));
    }
    return r[0] / (r[0] - r[1]);
}

static double form_kappa(const orc_state* st, int form)
{
    return form == FORM_HAT ? 0.5 * st->dt : form == FORM_BAR ? 0.5 * st->h : form == FORM_BARPLUS ? -0.5 * st->h : 0.0;
}

static void form_inverse(const orc_state* st, int form, double* Minv)
{
    double M[25];
    const double kappa = form_kappa(st, form);
    for (int k = 0; k < 25; ++k) M[k] = ((k % 6) == 0 ? 1.0 : 0.0) + kappa * st->mats[k];
    inv5(M, Minv);
}

double orc_form_pressure(const orc_state* st, const double* phi, int32_t form, double R)
{
    if (form < 0 || form > 3 || st->p.pl_n != 1.0) return NAN;
    double u, v, Pform, Minv[25];
    orc_node_moments(st->c, phi, &u, &v, &Pform);
    form_inverse(st, form, Minv);
    return solve_pressure(st, phi, Minv, form_kappa(st, form), R, u, v);
}

/* u, v and P of a stored form at a node with mass source R: for R = 0 the
 * pressure sum evaluated on the form itself (orc_node_moments); else the
 * solve above, with the form's inverse taken once at set-up. */
static void node_state(const orc_state* st, const double* phi, int form, double R, double* u, double* v, double* P)
{
    orc_node_moments(st->c, phi, u, v, P);
    if (R == 0.0) return;
    *P = solve_pressure(st, phi, st->kinv[form], st->kap[form], R, *u, *v);
}

static double source_at(const orc_state* st, size_t i) { return st->R ? st->R[i] : 0.0; }

/* Equilibrium of the alpha = 0 equation (eq. 2.2.5 with u_bar_0 = rho0 and
 * E_0 = 0): f^eq_{j,0} = w_j [rho0 + c_j . (rho0 u) / c_s^2]. */
static void feq_rho0(double c, double cs2, double rho, double u, double v, double* out)
{
    for (int j = 0; j < NQ; ++j) out[j] = WJ[j] * (rho + c * (CX[j] * u + CY[j] * v) * rho / cs2);
}

/* MRT collision matrix Lambda~ = M^-1 S M (eq. 2.2.4, Sec. 3.1 rates
 * s_0 = s_3 = s_4 = s', s_1 = s_2 = s) with the orthogonal D2Q5 basis
 * {1, c_x, c_y, 5 c^2/c^2 - 4, c_x^2 - c_y^2} (rows in units of c). */
static void mrt_lambda(double s, double sp, double* L)
{
    static const double M[25] = {
         1.0, 1.0,  1.0,  1.0,  1.0,
         0.0, 1.0,  0.0, -1.0,  0.0,
         0.0, 0.0,  1.0,  0.0, -1.0,
        -4.0, 1.0,  1.0,  1.0,  1.0,
         0.0, 1.0, -1.0,  1.0, -1.0,
    };
    double Minv[25], SM[25];
    const double S[NQ] = {sp, s, s, sp, sp};
    inv5(M, Minv);
    for (int m = 0; m < NQ; ++m)
        for (int k = 0; k < NQ; ++k) SM[m * NQ + k] = S[m] * M[m * NQ + k];
    mul5(Minv, SM, L);
}

void orc_collision_matrices(double s, double sp, double dt, double* out)
{
    double* Lt = out;          /* Lambda~                         */
    double* ImL = out + 25;    /* I - Lambda                      */
    double* Ib = out + 50;     /* I - 3/4 Lambda                  */
    double* Cinv = out + 75;   /* (I + h/2 Lambda~)^-1, h = dt/2  */
    double* Ainv = out + 100;  /* (I + dt/2 Lambda~)^-1           */
    double A[25], B[25], C[25];
    double h = 0.5 * dt;
    mrt_lambda(s, sp, Lt);
    for (int i = 0; i < NQ; ++i)
        for (int k = 0; k < NQ; ++k) {
            double id = (i == k) ? 1.0 : 0.0;
            A[i * NQ + k] = id + 0.5 * dt * Lt[i * NQ + k];
            B[i * NQ + k] = id - 0.5 * dt * Lt[i * NQ + k];
            C[i * NQ + k] = id + 0.5 * h * Lt[i * NQ + k];
        }
    inv5(A, Ainv);
    /* Lambda = I - (I - dt/2 Lambda~)(I + dt/2 Lambda~)^-1 (below eq. 2.2.14) */
    mul5(B, Ainv, ImL);
    for (int i = 0; i < 25; ++i) {
        int diag = (i % 6) == 0;
        double lam = (diag ? 1.0 : 0.0) - ImL[i];
        Ib[i] = (diag ? 1.0 : 0.0) - 0.75 * lam;
    }
    inv5(C, Cinv);
}

/* ------------------------------------------------------------------ */
/* power-law viscosity (reading of the keyword "power-law fluid")      */
/* ------------------------------------------------------------------ */

/* Magnitude gam_hat = sqrt(2 S^:S^) of S^ = -sym(M^ne), where
 * M^ne_{alpha beta} = sum_j c_{j,beta} (phi - f^eq)_{j,alpha}.  By eq. 2.4.1
 * (rewritten for the stored form phi) the shear rate is gam_hat/(nu + theta). */
static double noneq_shear(double c, const double* phi, const double* feq)
{
    double m[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < NQ; ++j) {
            double g = phi[a * NQ + j] - feq[a * NQ + j];
            m[a][0] += c * CX[j] * g;
            m[a][1] += c * CY[j] * g;
        }
    double s11 = -m[0][0], s22 = -m[1][1], s12 = -0.5 * (m[0][1] + m[1][0]);
    return sqrt(2.0 * (s11 * s11 + s22 * s22 + 2.0 * s12 * s12));
}

/* Solve nu = K (gam_hat/(nu + theta))^(n-1) for nu, clamp to [nu_min, nu_max].
 * n = 1: nu = K.  n = 1/2: the quadratic nu^2 - (K^2/g) nu - K^2 theta/g = 0,
 * positive root.  n = 3/2: the cubic nu^3 + theta nu^2 - K^2 g = 0 by 50 Newton
 * steps from nu_max. */
double orc_powerlaw_nu(const orc_state* st, double g, double theta)
{
    const orc_params* p = &st->p;
    double K = p->nu, nu;
    if (p->pl_n == 1.0) return K;
    if (p->pl_n == 0.5) {
        if (g == 0.0) return p->nu_max;
        double b = K * K / g;
        nu = 0.5 * (b + sqrt(b * b + 4.0 * K * K * theta / g));
    } else { /* 1.5 */
        if (g == 0.0) return p->nu_min;
        nu = p->nu_max;
        for (int it = 0; it < 50; ++it) {
            double f = nu * nu * nu + theta * nu * nu - K * K * g;
            double df = 3.0 * nu * nu + 2.0 * theta * nu;
            nu = nu - f / df;
        }
    }
    if (nu < p->nu_min) nu = p->nu_min;
    if (nu > p->nu_max) nu = p->nu_max;
    return nu;
}

/* Viscosity at a node for the collision of the stored form phi, whose
 * non-equilibrium first moment is (1 + s theta/c_s^2) times that of f. */
static double node_nu(const orc_state* st, const double* phi, const double* feq, double theta)
{
    if (st->p.pl_n == 1.0) return st->p.nu;
    return orc_powerlaw_nu(st, noneq_shear(st->c, phi, feq), theta);
}

/* Collision matrices of a node: the shared Newtonian set, or a fresh set for
 * the node's own power-law viscosity (s = c_s^2/nu, eq. 2.3.14; s' = ratio*s). */
static const double* node_mats(const orc_state* st, double nu, double* scratch)
{
    if (st->p.pl_n == 1.0) return st->mats;
    double s = st->cs2 / nu;
    orc_collision_matrices(s, st->p.s_ratio * s, st->dt, scratch);
    return scratch;
}

/* ------------------------------------------------------------------ */
/* grid helpers                                                        */
/* ------------------------------------------------------------------ */

static int is_wall(const orc_state* st, int x, int y)
{
    const orc_params* p = &st->p;
    if (p->bc_x == ORC_WALL && (x == 0 || x == st->nx - 1)) return 1;
    if (p->bc_y == ORC_WALL && (y == 0 || y == st->ny - 1)) return 1;
    return 0;
}

/* Value of plane `pl` at integer position (x, y) where one coordinate may lie
 * one node beyond a wall (quadratic ghost 3 Pi_0 - 3 Pi_1 + Pi_2, exact for the
 * quadratic profiles the stencil itself is exact on) or anywhere on a periodic
 * axis (wrapped). */
static double at(const orc_state* st, const double* pl, int x, int y)
{
    int nx = st->nx, ny = st->ny;
    if (st->p.bc_x == ORC_PERIODIC) x = ((x % nx) + nx) % nx;
    if (st->p.bc_y == ORC_PERIODIC) y = ((y % ny) + ny) % ny;
    if (x == -1) return 3.0 * at(st, pl, 0, y) - 3.0 * at(st, pl, 1, y) + at(st, pl, 2, y);
    if (x == nx) return 3.0 * at(st, pl, nx - 1, y) - 3.0 * at(st, pl, nx - 2, y) + at(st, pl, nx - 3, y);
    if (y == -1) return 3.0 * at(st, pl, x, 0) - 3.0 * at(st, pl, x, 1) + at(st, pl, x, 2);
    if (y == ny) return 3.0 * at(st, pl, x, ny - 1) - 3.0 * at(st, pl, x, ny - 2) + at(st, pl, x, ny - 3);
    return pl[(size_t)y * nx + x];
}

/* Mixed difference of eq. 2.2.12: eta * central (eq. 2.2.13a) + (1 - eta) *
 * second-order upwind (eq. 2.2.13b) along `axis` for a velocity of sign `sg`.
 * On a mapped grid d/dx = (1/X') d/dxi, so 1/(2 dchi) becomes g_i/2. */
static double mixed_d(const orc_state* st, const double* pl, int x, int y, int axis, int sg)
{
    int dx = axis == 0 ? 1 : 0, dy = axis == 0 ? 0 : 1;
    double g = axis == 0 ? st->gx[x] : st->gy[y];
    double eta = st->p.eta;
    double pm1 = at(st, pl, x - dx, y - dy);
    double p0 = at(st, pl, x, y);
    double pp1 = at(st, pl, x + dx, y + dy);
    double central = (pp1 - pm1) * g / 2.0;
    double upwind;
    if (sg >= 0) {
        double pm2 = at(st, pl, x - 2 * dx, y - 2 * dy);
        upwind = (3.0 * p0 - 4.0 * pm1 + pm2) * g / 2.0;
    } else {
        double pp2 = at(st, pl, x + 2 * dx, y + 2 * dy);
        upwind = -(3.0 * p0 - 4.0 * pp1 + pp2) * g / 2.0;
    }
    return eta * central + (1.0 - eta) * upwind;
}

/* Mixed difference along an index axis with unit spacing (the general
 * mapping carries the node spacing in its metric). */
static double mixed_unit(const orc_state* st, const double* pl, int x, int y, int axis, int sg)
{
    int dx = axis == 0 ? 1 : 0, dy = axis == 0 ? 0 : 1;
    double eta = st->p.eta;
    double pm1 = at(st, pl, x - dx, y - dy);
    double p0 = at(st, pl, x, y);
    double pp1 = at(st, pl, x + dx, y + dy);
    double central = (pp1 - pm1) / 2.0;
    double upwind;
    if (sg >= 0) {
        double pm2 = at(st, pl, x - 2 * dx, y - 2 * dy);
        upwind = (3.0 * p0 - 4.0 * pm1 + pm2) / 2.0;
    } else {
        double pp2 = at(st, pl, x + 2 * dx, y + 2 * dy);
        upwind = -(3.0 * p0 - 4.0 * pp1 + pp2) / 2.0;
    }
    return eta * central + (1.0 - eta) * upwind;
}

/* c_j . grad Pi_j with the mixed scheme.  Separable grids: only the axis of
 * c_j contributes.  General mapping: by the chain rule c_j . grad =
 * U d/di + V d/dj with the contravariant components U = c_j . grad i and
 * V = c_j . grad j of the node, each index derivative upwinded by the sign of
 * its own component (eqs. 2.2.12-2.2.13 along each index line). */
static double cdotgrad(const orc_state* st, const double* pl, int x, int y, int j)
{
    double c = st->c;
    if (st->met) {
        size_t n = st->n, i = (size_t)y * st->nx + x;
        double U = c * (CX[j] * st->met[i] + CY[j] * st->met[n + i]);
        double V = c * (CX[j] * st->met[2 * n + i] + CY[j] * st->met[3 * n + i]);
        double r = 0.0;
        if (U != 0.0) r += U * mixed_unit(st, pl, x, y, 0, U > 0.0 ? 1 : -1);
        if (V != 0.0) r += V * mixed_unit(st, pl, x, y, 1, V > 0.0 ? 1 : -1);
        return r;
    }
    if (CX[j] != 0.0) return c * CX[j] * mixed_d(st, pl, x, y, 0, CX[j] > 0 ? 1 : -1);
    if (CY[j] != 0.0) return c * CY[j] * mixed_d(st, pl, x, y, 1, CY[j] > 0 ? 1 : -1);
    return 0.0;
}

void orc_mixed_derivative(const orc_state* st, const double* field, int32_t axis, int32_t sign, double* out)
{
    for (int y = 0; y < st->ny; ++y)
        for (int x = 0; x < st->nx; ++x)
            out[(size_t)y * st->nx + x] =
                is_wall(st, x, y) ? 0.0 : mixed_d(st, field, x, y, axis, sign >= 0 ? 1 : -1);
}

static void gather(const orc_state* st, const double* field, size_t i, double* phi)
{
    for (int k = 0; k < NPL; ++k) phi[k] = field[(size_t)k * st->n + i];
}

static void scatter(const orc_state* st, double* field, size_t i, const double* phi)
{
    for (int k = 0; k < NPL; ++k) field[(size_t)k * st->n + i] = phi[k];
}

/* Wall rule (non-equilibrium extrapolation, the scheme named for the
 * Poiseuille and cavity flows of Secs. 4.3-4.4): at a wall node w with inward
 * neighbours n1 = w + d and n2 = w + 2d (d the inward normal, diagonal at a
 * corner), the wall value is the equilibrium at the wall velocity u_w and the
 * neighbour pressure plus the non-equilibrium part extrapolated linearly,
 *   Pi_j(w) = f^eq_j(u_w, P_n1) + 2 [Pi_j(n1) - f^eq_j(n1)] - [Pi_j(n2) - f^eq_j(n2)],
 * where f^eq_j(n) is the equilibrium of the moments of Pi(n).  u_w is the lid
 * speed on the top wall (corners excluded) and zero elsewhere.  The linear
 * extrapolation keeps the scheme second order at walls, as the GREs of the
 * Poiseuille table require (a zeroth-order copy of Pi(n1) - f^eq(n1) gives a
 * first-order wall error about 16 times the tabulated value at 32 x 32). */
static void wall_update(const orc_state* st, double* field, int form)
{
    const orc_params* p = &st->p;
    int nx = st->nx, ny = st->ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (!is_wall(st, x, y)) continue;
            int ix = 0, iy = 0;
            if (p->bc_x == ORC_WALL) ix = (x == 0) ? 1 : (x == nx - 1 ? -1 : 0);
            if (p->bc_y == ORC_WALL) iy = (y == 0) ? 1 : (y == ny - 1 ? -1 : 0);
            int corner = (ix != 0 && iy != 0);
            double uw = (p->bc_y == ORC_WALL && y == ny - 1 && !corner) ? p->lid_u : 0.0;
            size_t i1 = (size_t)(y + iy) * nx + (x + ix);
            size_t i2 = (size_t)(y + 2 * iy) * nx + (x + 2 * ix);
            double ph1[NPL], ph2[NPL], fe1[NPL], fe2[NPL], few[NPL];
            double u1, v1, P1, u2, v2, P2;
            gather(st, field, i1, ph1);
            gather(st, field, i2, ph2);
            node_state(st, ph1, form, source_at(st, i1), &u1, &v1, &P1);
            node_state(st, ph2, form, source_at(st, i2), &u2, &v2, &P2);
            orc_feq(st->c, u1, v1, P1, fe1);
            orc_feq(st->c, u2, v2, P2, fe2);
            orc_feq(st->c, uw, 0.0, P1, few);
            double out[NPL];
            for (int k = 0; k < NPL; ++k)
                out[k] = few[k] + 2.0 * (ph1[k] - fe1[k]) - (ph2[k] - fe2[k]);
            scatter(st, field, (size_t)y * nx + x, out);
        }
}

void orc_wall_update(const orc_state* st, double* field) { wall_update(st, field, FORM_HAT); }

/* ------------------------------------------------------------------ */
/* Step (1): collision at t (eqs. 2.2.14 and 2.2.15)                    */
/* ------------------------------------------------------------------ */

static void collide_step1(const orc_state* st, const double* fhat, double R, double* fhat_plus, double* fbar_plus)
{
    double u, v, P, feq[NPL], scratch[125];
    node_state(st, fhat, FORM_HAT, R, &u, &v, &P);
    orc_feq(st->c, u, v, P, feq);
    double nu = node_nu(st, fhat, feq, st->cs2 * st->dt / 2.0);
    const double* mats = node_mats(st, nu, scratch);
    const double* ImL = mats + 25;
    const double* Ib = mats + 50;
    for (int a = 0; a < 2; ++a) {
        const double* fh = fhat + a * NQ;
        const double* fe = feq + a * NQ;
        double t1[NQ], t2[NQ], lam[25], lam34[25];
        for (int i = 0; i < 25; ++i) {
            double id = (i % 6) == 0 ? 1.0 : 0.0;
            lam[i] = id - ImL[i];       /* Lambda         */
            lam34[i] = id - Ib[i];      /* 3/4 Lambda     */
        }
        /* f_hat^+ = (I - Lambda) f_hat + Lambda f^eq            (eq. 2.2.14) */
        mv5(ImL, fh, t1);
        mv5(lam, fe, t2);
        for (int j = 0; j < NQ; ++j) fhat_plus[a * NQ + j] = t1[j] + t2[j];
        /* f_bar^+ = (I - 3/4 Lambda) f_hat + 3/4 Lambda f^eq    (eq. 2.2.15) */
        mv5(Ib, fh, t1);
        mv5(lam34, fe, t2);
        for (int j = 0; j < NQ; ++j) fbar_plus[a * NQ + j] = t1[j] + t2[j];
    }
}

/* the same at a node without mass source */
void orc_collide_step1(const orc_state* st, const double* fhat, double* fhat_plus, double* fbar_plus)
{
    collide_step1(st, fhat, 0.0, fhat_plus, fbar_plus);
}

/* Step (3): f = (I + h/2 Lambda~)^-1 (f_bar + h/2 Lambda~ f^eq)   (eq. 2.2.16) */
static void collide_step3(const orc_state* st, const double* fbar, double R, double* f)
{
    double u, v, P, feq[NPL], scratch[125];
    node_state(st, fbar, FORM_BAR, R, &u, &v, &P);
    orc_feq(st->c, u, v, P, feq);
    double nu = node_nu(st, fbar, feq, st->cs2 * st->dt / 4.0);
    const double* mats = node_mats(st, nu, scratch);
    const double* Lt = mats;
    const double* Cinv = mats + 75;
    for (int a = 0; a < 2; ++a) {
        double lf[NQ], rhs[NQ], out[NQ];
        mv5(Lt, feq + a * NQ, lf);
        for (int j = 0; j < NQ; ++j) rhs[j] = fbar[a * NQ + j] + 0.5 * st->h * lf[j];
        mv5(Cinv, rhs, out);
        for (int j = 0; j < NQ; ++j) f[a * NQ + j] = out[j];
    }
}

/* ------------------------------------------------------------------ */
/* the alpha = 0 equation (rho0), tracked as a check of Remark 1        */
/* ------------------------------------------------------------------ */

/* Steps (1)-(4) for the alpha = 0 distributions: the same collision matrices
 * and stencils as the velocity sets, the equilibrium of feq_rho0 with the
 * velocity of the velocity sets at t (Step 1) and t + h (Step 3), and the
 * source F_{j,0} = w_j R (eq. 2.2.6 with F_bar_0 = R, eq. 2.1.2).  No pressure
 * enters (E_0 = 0).  Runs after the velocity sets' step, whose f_hat(t) and
 * f(t+h) it reads. */
static void rho0_step(orc_state* st)
{
    int nx = st->nx, ny = st->ny;
    size_t n = st->n;
    const double* Lt = st->mats;
    const double* ImL = st->mats + 25;
    const double* Ib = st->mats + 50;
    const double* Cinv = st->mats + 75;
    double lam[25], lam34[25];
    for (int k = 0; k < 25; ++k) {
        double id = (k % 6) == 0 ? 1.0 : 0.0;
        lam[k] = id - ImL[k];
        lam34[k] = id - Ib[k];
    }
    /* Step (1) */
    for (size_t i = 0; i < n; ++i) {
        double g[NQ], fe[NQ], t1[NQ], t2[NQ], rho = 0.0, u = 0.0, v = 0.0;
        for (int q = 0; q < NQ; ++q) {
            g[q] = st->r0hat[q * n + i];
            rho += g[q];
            u += st->fhat[q * n + i];
            v += st->fhat[(NQ + q) * n + i];
        }
        feq_rho0(st->c, st->cs2, rho, u, v, fe);
        mv5(ImL, g, t1);
        mv5(lam, fe, t2);
        for (int q = 0; q < NQ; ++q) st->r0hatp[q * n + i] = t1[q] + t2[q];
        mv5(Ib, g, t1);
        mv5(lam34, fe, t2);
        for (int q = 0; q < NQ; ++q) st->r0barp[q * n + i] = t1[q] + t2[q];
    }
    /* Step (2) */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            for (int q = 0; q < NQ; ++q) {
                const double* pl = st->r0barp + q * n;
                st->r0bar[q * n + i] = pl[i] - st->h * cdotgrad(st, pl, x, y, q) + st->h * WJ[q] * source_at(st, i);
            }
        }
    /* Step (3) */
    for (size_t i = 0; i < n; ++i) {
        double g[NQ], fe[NQ], lf[NQ], rhs[NQ], out[NQ], rho = 0.0, u = 0.0, v = 0.0;
        for (int q = 0; q < NQ; ++q) {
            g[q] = st->r0bar[q * n + i];
            rho += g[q];
            u += st->fmid[q * n + i];
            v += st->fmid[(NQ + q) * n + i];
        }
        feq_rho0(st->c, st->cs2, rho, u, v, fe);
        mv5(Lt, fe, lf);
        for (int q = 0; q < NQ; ++q) rhs[q] = g[q] + 0.5 * st->h * lf[q];
        mv5(Cinv, rhs, out);
        for (int q = 0; q < NQ; ++q) st->r0mid[q * n + i] = out[q];
    }
    /* Step (4) */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            for (int q = 0; q < NQ; ++q)
                st->r0new[q * n + i] = st->r0hatp[q * n + i] - st->dt * cdotgrad(st, st->r0mid + q * n, x, y, q)
                                     + st->dt * WJ[q] * source_at(st, i);
        }
    double* t = st->r0hat;
    st->r0hat = st->r0new;
    st->r0new = t;
}

int32_t orc_rho0(const orc_state* st, double* out)
{
    if (!st->r0hat) return -1;
    for (size_t i = 0; i < st->n; ++i) {
        double rho = 0.0;
        for (int q = 0; q < NQ; ++q) rho += st->r0hat[q * st->n + i];
        out[i] = rho;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* the sources G and G_bar (eqs. 2.2.7 and 2.2.10)                     */
/* ------------------------------------------------------------------ */

/* Momentum flux at every node at the start of the step: for alpha = 1 the
 * vector u_bar_1 u + P E_1 = (u u + P, u v), for alpha = 2 (v u, v v + P). */
static void flux_now(orc_state* st)
{
    for (size_t i = 0; i < st->n; ++i) {
        double phi[NPL], u, v, P;
        gather(st, st->fhat, i, phi);
        node_state(st, phi, FORM_HAT, source_at(st, i), &u, &v, &P);
        st->qn[4 * i + 0] = u * u + P;
        st->qn[4 * i + 1] = u * v;
        st->qn[4 * i + 2] = v * u;
        st->qn[4 * i + 3] = v * v + P;
    }
}

/* Source of distribution j of equation alpha at node i from the flux history:
 *   g  = w_j c_j . d_t(u_alpha u + P E_alpha) / c_s^2        (eq. 2.2.7)
 *   dg = w_j c_j . d_tt(u_alpha u + P E_alpha) / c_s^2       (its d_t)
 * with the backward differences (Q_n - Q_{n-1})/dt and
 * (Q_n - 2 Q_{n-1} + Q_{n-2})/dt^2, zero while the steps before are missing. */
static void flux_source_at(const orc_state* st, size_t i, int a, int j, double* g, double* dg)
{
    double d1[2] = {0.0, 0.0}, d2[2] = {0.0, 0.0};
    for (int b = 0; b < 2; ++b) {
        const double qn = st->qn[4 * i + 2 * a + b];
        if (st->nq >= 1) d1[b] = (qn - st->q1[4 * i + 2 * a + b]) / st->dt;
        if (st->nq >= 2) d2[b] = (qn - 2.0 * st->q1[4 * i + 2 * a + b] + st->q2[4 * i + 2 * a + b]) / (st->dt * st->dt);
    }
    *g = WJ[j] * st->c * (CX[j] * d1[0] + CY[j] * d1[1]) / st->cs2;
    *dg = WJ[j] * st->c * (CX[j] * d2[0] + CY[j] * d2[1]) / st->cs2;
}

/* ------------------------------------------------------------------ */
/* one time step                                                       */
/* ------------------------------------------------------------------ */

static void one_step(orc_state* st)
{
    int nx = st->nx, ny = st->ny;
    long n = (long)st->n;
    const double* Fa[2] = {st->Fx, st->Fy};
    /* time factor of the force at t = steps dt and its time derivative: F(x, t)
     * = F(x) m(t), d_t F = F(x) m'(t); m = 1, m' = 0 for a steady force */
    const double tn = (double)st->steps * st->dt;
    const int harmonic = st->p.force_harmonic != 0;
    const double m = harmonic ? cos(st->p.force_omega * tn + st->p.force_phase) : 1.0;
    const double dm = harmonic ? -st->p.force_omega * sin(st->p.force_omega * tn + st->p.force_phase) : 0.0;
    /* G_bar = (I + h/2 S~)^-1 G with S~ = s I (eq. 2.2.10) */
    const double gbar = st->qn ? 1.0 / (1.0 + 0.5 * st->h * st->cs2 / st->p.nu) : 0.0;
    if (st->qn) flux_now(st);

    /* Step (1): f_hat^+ and f_bar^+ at every node. */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double fh[NPL], fhp[NPL], fbp[NPL];
        gather(st, st->fhat, i, fh);
        collide_step1(st, fh, source_at(st, (size_t)i), fhp, fbp);
        scatter(st, st->fhat_plus, i, fhp);
        scatter(st, st->fbar_plus, i, fbp);
    }
    wall_update(st, st->fbar_plus, FORM_BARPLUS);

    /* Step (2): f_bar(t+h) = f_bar^+ - h c_j . grad f_bar^+ + h w_j F_alpha(t)
     * (eq. 2.3.25: eq. 2.2.11 with the G terms and the h^2/2 d_t F term dropped
     * per Remark 2; F_j = w_j F of eq. 2.2.6). */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (is_wall(st, x, y)) continue;
            size_t i = (size_t)y * nx + x;
            for (int a = 0; a < 2; ++a)
                for (int j = 0; j < NQ; ++j) {
                    const double* pl = st->fbar_plus + (size_t)(a * NQ + j) * n;
                    st->fbar[(size_t)(a * NQ + j) * n + i] =
                        pl[i] - st->h * cdotgrad(st, pl, x, y, j) + st->h * WJ[j] * Fa[a][i] * m;
                    if (st->qn) {
                        /* + h [G_bar + (h/2) d_t G_bar]   (eq. 2.2.11) */
                        double g, dg;
                        flux_source_at(st, i, a, j, &g, &dg);
                        st->fbar[(size_t)(a * NQ + j) * n + i] += st->h * gbar * (g + 0.5 * st->h * dg);
                    }
                }
        }

    /* Step (3): f(t+h) from f_bar(t+h) at every non-wall node, walls by rule. */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (is_wall(st, x, y)) continue;
            size_t i = (size_t)y * nx + x;
            double fb[NPL], f[NPL];
            gather(st, st->fbar, i, fb);
            collide_step3(st, fb, source_at(st, i), f);
            scatter(st, st->fmid, i, f);
        }
    wall_update(st, st->fmid, FORM_F);

    /* Step (4): f_hat(t+dt) = f_hat^+ - dt c_j . grad f(t+h) + dt w_j F_alpha(t)
     * + (dt^2/2) w_j d_t F_alpha(t)  (eq. 2.3.24; the last term vanishes for a
     * steady force). */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (is_wall(st, x, y)) continue;
            size_t i = (size_t)y * nx + x;
            for (int a = 0; a < 2; ++a)
                for (int j = 0; j < NQ; ++j) {
                    size_t k = (size_t)(a * NQ + j) * n;
                    st->fnew[k + i] = st->fhat_plus[k + i]
                                    - st->dt * cdotgrad(st, st->fmid + k, x, y, j)
                                    + st->dt * WJ[j] * Fa[a][i] * m
                                    + 0.5 * st->dt * st->dt * WJ[j] * Fa[a][i] * dm;
                    if (st->qn) {
                        /* + dt G + (dt^2/2) d_t G   (eq. 2.2.1) */
                        double g, dg;
                        flux_source_at(st, i, a, j, &g, &dg);
                        st->fnew[k + i] += st->dt * g + 0.5 * st->dt * st->dt * dg;
                    }
                }
        }
    wall_update(st, st->fnew, FORM_HAT);

    if (st->r0hat) rho0_step(st);
    if (st->qn) {
        double* t2 = st->q2;
        st->q2 = st->q1;
        st->q1 = st->qn;
        st->qn = t2;
        if (st->nq < 2) st->nq += 1;
    }

    double* t = st->fhat;
    st->fhat = st->fnew;
    st->fnew = t;
    st->steps += 1;
}

void orc_step(orc_state* st, int32_t nsteps)
{
    for (int32_t s = 0; s < nsteps; ++s) one_step(st);
}

int32_t orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return (int32_t)omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* life cycle                                                          */
/* ------------------------------------------------------------------ */

orc_state* orc_create(const orc_params* p, const double* u0, const double* v0, const double* p0)
{
    if (!p || p->nx < 5 || p->ny < 5 || !(p->c > 0.0) || !(p->cfl > 0.0)) return NULL;
    if (!(p->eta >= 0.0 && p->eta <= 1.0)) return NULL;
    if (!(p->pl_n == 1.0 || p->pl_n == 0.5 || p->pl_n == 1.5)) return NULL;
    if (!(p->nu > 0.0)) return NULL;
    if (p->pl_n != 1.0 && !(p->nu_min > 0.0 && p->nu_max >= p->nu_min)) return NULL;
    if ((p->inv_dx_x || p->inv_dx_y) && !(p->dx_min > 0.0)) return NULL;
    if (p->metric && (p->inv_dx_x || p->inv_dx_y || !(p->dx_min > 0.0))) return NULL;
    if (p->force_harmonic != 0 &&
        (p->force_harmonic != 1 || !isfinite(p->force_omega) || !isfinite(p->force_phase)))
        return NULL;
    if (p->mass_source) {
        if (p->pl_n != 1.0) return NULL;
        for (size_t i = 0; i < (size_t)p->nx * p->ny; ++i)
            if (!isfinite(p->mass_source[i])) return NULL;
    }
    if (p->track_rho0 != 0 &&
        (p->track_rho0 != 1 || p->pl_n != 1.0 || p->bc_x != ORC_PERIODIC || p->bc_y != ORC_PERIODIC))
        return NULL;
    if (p->flux_source != 0 && (p->flux_source != 1 || p->pl_n != 1.0)) return NULL;

    orc_state* st = (orc_state*)calloc(1, sizeof(orc_state));
    st->p = *p;
    st->nx = p->nx;
    st->ny = p->ny;
    st->n = (size_t)p->nx * p->ny;
    st->c = p->c;
    st->cs2 = lattice_cs2(p->c);

    /* node spacing: periodic x_i = i L/N, walls x_i = i L/(N-1) */
    double hx = p->bc_x == ORC_WALL ? p->lx / (p->nx - 1) : p->lx / p->nx;
    double hy = p->bc_y == ORC_WALL ? p->ly / (p->ny - 1) : p->ly / p->ny;
    st->gx = (double*)malloc(sizeof(double) * p->nx);
    st->gy = (double*)malloc(sizeof(double) * p->ny);
    /* body force per node: the uniform part plus the optional field */
    st->Fx = (double*)malloc(sizeof(double) * st->n);
    st->Fy = (double*)malloc(sizeof(double) * st->n);
    for (size_t i = 0; i < st->n; ++i) {
        st->Fx[i] = p->fx + (p->force_x ? p->force_x[i] : 0.0);
        st->Fy[i] = p->fy + (p->force_y ? p->force_y[i] : 0.0);
    }
    st->p.force_x = NULL;
    st->p.force_y = NULL;
    for (int i = 0; i < p->nx; ++i) st->gx[i] = p->inv_dx_x ? p->inv_dx_x[i] : 1.0 / hx;
    for (int i = 0; i < p->ny; ++i) st->gy[i] = p->inv_dx_y ? p->inv_dx_y[i] : 1.0 / hy;
    st->met = NULL;
    if (p->metric) {
        st->met = (double*)malloc(sizeof(double) * 4 * st->n);
        for (size_t k = 0; k < 4 * st->n; ++k) st->met[k] = p->metric[k];
    }
    st->p.metric = NULL;
    double dxmin = (p->inv_dx_x || p->inv_dx_y || p->metric) ? p->dx_min : (hx < hy ? hx : hy);
    /* eq. 3.1: dt = CFL dx_min / c; the half step is h = dt/2 (below eq. 2.2.8) */
    st->dt = p->cfl * dxmin / p->c;
    st->h = 0.5 * st->dt;

    if (p->pl_n == 1.0) {
        double s = st->cs2 / p->nu; /* nu = c_s^2 / s (eq. 2.3.14) */
        orc_collision_matrices(s, p->s_ratio * s, st->dt, st->mats);
    }
    st->R = NULL;
    if (p->mass_source) {
        st->R = (double*)malloc(sizeof(double) * st->n);
        for (size_t i = 0; i < st->n; ++i) st->R[i] = p->mass_source[i];
        for (int form = 0; form < 4; ++form) {
            st->kap[form] = form_kappa(st, form);
            form_inverse(st, form, st->kinv[form]);
        }
    }
    st->p.mass_source = NULL;

    size_t bytes = sizeof(double) * NPL * st->n;
    st->fhat = (double*)malloc(bytes);
    st->fhat_plus = (double*)malloc(bytes);
    st->fbar_plus = (double*)malloc(bytes);
    st->fbar = (double*)calloc(1, bytes);
    st->fmid = (double*)calloc(1, bytes);
    st->fnew = (double*)calloc(1, bytes);

    /* f_hat = f^eq(u0, P0) (Sec. 4), then the wall rule carries the wall velocity. */
    for (size_t i = 0; i < st->n; ++i) {
        double fe[NPL];
        orc_feq(st->c, u0[i], v0[i], p0[i], fe);
        scatter(st, st->fhat, i, fe);
    }
    orc_wall_update(st, st->fhat);
    /* walls of the intermediate fields start equal to the state */
    memcpy(st->fnew, st->fhat, bytes);

    if (p->flux_source) {
        st->q1 = (double*)calloc(4 * st->n, sizeof(double));
        st->q2 = (double*)calloc(4 * st->n, sizeof(double));
        st->qn = (double*)calloc(4 * st->n, sizeof(double));
        st->nq = 0;
    }

    /* rho0 = 1 at rest in the velocity field: f_hat_0 = f^eq_0(1, u0) */
    if (p->track_rho0) {
        size_t b0 = sizeof(double) * NQ * st->n;
        st->r0hat = (double*)malloc(b0);
        st->r0hatp = (double*)malloc(b0);
        st->r0barp = (double*)malloc(b0);
        st->r0bar = (double*)malloc(b0);
        st->r0mid = (double*)malloc(b0);
        st->r0new = (double*)malloc(b0);
        for (size_t i = 0; i < st->n; ++i) {
            double fe[NQ];
            feq_rho0(st->c, st->cs2, 1.0, u0[i], v0[i], fe);
            for (int q = 0; q < NQ; ++q) st->r0hat[q * st->n + i] = fe[q];
        }
    }
    return st;
}

void orc_destroy(orc_state* st)
{
    if (!st) return;
    free(st->gx);
    free(st->gy);
    free(st->met);
    free(st->Fx);
    free(st->Fy);
    free(st->fhat);
    free(st->fhat_plus);
    free(st->fbar_plus);
    free(st->fbar);
    free(st->fmid);
    free(st->fnew);
    free(st->R);
    free(st->r0hat);
    free(st->r0hatp);
    free(st->r0barp);
    free(st->r0bar);
    free(st->r0mid);
    free(st->r0new);
    free(st->q1);
    free(st->q2);
    free(st->qn);
    free(st);
}

double orc_dt(const orc_state* st) { return st->dt; }
int64_t orc_steps(const orc_state* st) { return st->steps; }

void orc_get_f(const orc_state* st, double* f) { memcpy(f, st->fhat, sizeof(double) * NPL * st->n); }

void orc_set_f(orc_state* st, const double* f) { memcpy(st->fhat, f, sizeof(double) * NPL * st->n); }

void orc_fields(const orc_state* st, int32_t which, double* out)
{
    const double* src = which == 0 ? st->fhat_plus : which == 1 ? st->fbar_plus : which == 2 ? st->fbar : st->fmid;
    memcpy(out, src, sizeof(double) * NPL * st->n);
}

void orc_moments(const orc_state* st, double* u, double* v, double* p)
{
    for (size_t i = 0; i < st->n; ++i) {
        double phi[NPL];
        gather(st, st->fhat, i, phi);
        node_state(st, phi, FORM_HAT, source_at(st, i), &u[i], &v[i], &p[i]);
    }
}

/* Local derived quantities of Sec. 2.4 at every node.  f^ne = f - f^eq is
 * recovered from the state through the inverse of eq. 2.2.2,
 * f - f^eq = (I + dt/2 Lambda~)^-1 (f_hat - f^eq), then
 *   grad_beta u_alpha = -(s/c_s^2) sum_i c_{i,beta} f^ne_{i,alpha}     (eq. 2.4.1)
 *   div u = sum_alpha grad_alpha u_alpha                               (eq. 2.4.2)
 *   S = (G + G^T)/2 (eq. 2.4.3 read as a sum), sigma = 2 rho0 nu S with rho0 = 1
 *   (eq. 2.4.4), Omega = (G - G^T)/2 (eq. 2.4.5), omega = dv/dx - du/dy. */
void orc_derived(const orc_state* st, double* out)
{
    size_t n = st->n;
    for (size_t i = 0; i < n; ++i) {
        double fh[NPL], feq[NPL], u, v, P, scratch[125];
        gather(st, st->fhat, i, fh);
        node_state(st, fh, FORM_HAT, source_at(st, i), &u, &v, &P);
        orc_feq(st->c, u, v, P, feq);
        double nu = node_nu(st, fh, feq, st->cs2 * st->dt / 2.0);
        const double* mats = node_mats(st, nu, scratch);
        const double* Ainv = mats + 100;
        double s = st->cs2 / nu;
        double G[2][2];
        for (int a = 0; a < 2; ++a) {
            double g[NQ], fne[NQ];
            for (int j = 0; j < NQ; ++j) g[j] = fh[a * NQ + j] - feq[a * NQ + j];
            mv5(Ainv, g, fne);
            double mx = 0.0, my = 0.0;
            for (int j = 0; j < NQ; ++j) {
                mx += st->c * CX[j] * fne[j];
                my += st->c * CY[j] * fne[j];
            }
            G[a][0] = -(s / st->cs2) * mx;
            G[a][1] = -(s / st->cs2) * my;
        }
        double Sxx = G[0][0], Syy = G[1][1], Sxy = 0.5 * (G[0][1] + G[1][0]);
        double vals[14] = {
            G[0][0], G[0][1], G[1][0], G[1][1],
            G[0][0] + G[1][1],
            Sxx, Sxy, Syy,
            2.0 * nu * Sxx, 2.0 * nu * Sxy, 2.0 * nu * Syy,
            0.5 * (G[0][1] - G[1][0]),
            G[1][0] - G[0][1],
            nu,
        };
        for (int k = 0; k < 14; ++k) out[(size_t)k * n + i] = vals[k];
    }
}

/* Diagnostics: sum u, sum v, KE = 1/2 sum |u|^2 dA, enstrophy = 1/2 sum omega^2 dA
 * (omega from the local scheme of Sec. 2.4), max |u|, max |div u| by central
 * differences over non-wall nodes, number of non-finite state entries, and
 * sum dA, with dA = 1/(g_x g_y) the area of a node (under a general mapping
 * dA = 1/|det| of the node's inverse Jacobian, and the divergence takes both
 * index differences of each velocity component by the chain rule). */
void orc_diagnostics(const orc_state* st, double* out)
{
    int nx = st->nx, ny = st->ny;
    size_t n = st->n;
    double* u = (double*)malloc(sizeof(double) * n);
    double* v = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* d = (double*)malloc(sizeof(double) * 14 * n);
    orc_moments(st, u, v, p);
    orc_derived(st, d);
    double su = 0, sv = 0, ke = 0, ens = 0, umax = 0, dmax = 0, bad = 0, area = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            double dA = 1.0 / (st->gx[x] * st->gy[y]);
            if (st->met) {
                double det = st->met[i] * st->met[3 * n + i] - st->met[n + i] * st->met[2 * n + i];
                dA = 1.0 / fabs(det);
            }
            double om = d[12 * n + i];
            su += u[i];
            sv += v[i];
            ke += 0.5 * (u[i] * u[i] + v[i] * v[i]) * dA;
            ens += 0.5 * om * om * dA;
            double sp = sqrt(u[i] * u[i] + v[i] * v[i]);
            if (sp > umax) umax = sp;
            area += dA;
            if (!is_wall(st, x, y)) {
                int xp = (x + 1) % nx, xm = (x - 1 + nx) % nx;
                int yp = (y + 1) % ny, ym = (y - 1 + ny) % ny;
                double div = (u[(size_t)y * nx + xp] - u[(size_t)y * nx + xm]) * st->gx[x] / 2.0
                           + (v[(size_t)yp * nx + x] - v[(size_t)ym * nx + x]) * st->gy[y] / 2.0;
                if (st->met) {
                    /* du/dx + dv/dy = (di/dx) u_i + (dj/dx) u_j + (di/dy) v_i + (dj/dy) v_j */
                    double ui = (u[(size_t)y * nx + xp] - u[(size_t)y * nx + xm]) / 2.0;
                    double uj = (u[(size_t)yp * nx + x] - u[(size_t)ym * nx + x]) / 2.0;
                    double vi = (v[(size_t)y * nx + xp] - v[(size_t)y * nx + xm]) / 2.0;
                    double vj = (v[(size_t)yp * nx + x] - v[(size_t)ym * nx + x]) / 2.0;
                    div = st->met[i] * ui + st->met[2 * n + i] * uj + st->met[n + i] * vi + st->met[3 * n + i] * vj;
                }
                if (fabs(div) > dmax) dmax = fabs(div);
            }
        }
    for (size_t k = 0; k < NPL * n; ++k)
        if (!isfinite(st->fhat[k])) bad += 1.0;
    out[0] = su;
    out[1] = sv;
    out[2] = ke;
    out[3] = ens;
    out[4] = umax;
    out[5] = dmax;
    out[6] = bad;
    out[7] = area;
    free(u);
    free(v);
    free(p);
    free(d);
}
