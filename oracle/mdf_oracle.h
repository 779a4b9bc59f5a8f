/*
 * MDF-FDLBM CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential FP64 implementation of the time step of the
 * multiple-distribution-function finite-difference lattice Boltzmann method
 * (Chen, Chai, Zhao & Shi, "Multiple-distribution-function finite-difference
 * lattice Boltzmann method for incompressible Navier-Stokes equation").
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source, header, table or
 * constant with the HIP library; both sides see only the same raw inputs
 * (problem parameters, initial fields, grid metric arrays).
 *
 * Layout of every distribution array exchanged with this library:
 *   f[(alpha*5 + j)*ny*nx + y*nx + x],  alpha in {0 (u), 1 (v)}, j in 0..4,
 *   D2Q5 velocities c_j = c*{(0,0),(1,0),(0,1),(-1,0),(0,-1)}  (Sec. 3.1, eq. 3.1.0).
 */
#ifndef MDF_ORACLE_H
#define MDF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_WALL = 1 };

typedef struct {
    int32_t nx, ny;          /* nodes per axis (wall axes include both wall nodes)   */
    double  lx, ly;          /* domain lengths                                       */
    double  nu;              /* Newtonian viscosity, or consistency K if pl_n != 1   */
    double  pl_n;            /* power-law index (1 = Newtonian)                      */
    double  nu_min, nu_max;  /* clamp of the local power-law viscosity              */
    double  cfl, c, eta, s_ratio;
    int32_t bc_x, bc_y;      /* ORC_PERIODIC or ORC_WALL                             */
    double  lid_u;           /* tangential velocity of the top (y = ly) wall         */
    double  fx, fy;          /* uniform body force                                   */
    const double* inv_dx_x;  /* nx entries: d(xi)/dx / d(xi), i.e. 1/(X'(xi_i) dxi); NULL = uniform */
    const double* inv_dx_y;  /* ny entries, same meaning for y                        */
    double  dx_min;          /* smallest node spacing; used for dt when metrics are given */
    const double* force_x;   /* ny*nx entries added to fx at each node (F(x), eq. 2.2.6); NULL = none */
    const double* force_y;   /* same for fy                                           */
    /* time dependence of the force: 0 = steady; 1 = F(x, t) = F(x) cos(force_omega t + force_phase),
     * with F(x) the uniform part plus the field above, t = steps * dt */
    double  force_omega, force_phase;
    int32_t force_harmonic;
    /* general (non-separable) coordinate transformation x = X(i, j), y = Y(i, j) of the
     * node indices: 4 planes of ny*nx entries, d i/dx, d i/dy, d j/dx, d j/dy at each node
     * (the inverse Jacobian in node units), or NULL.  Excludes inv_dx_x / inv_dx_y; needs
     * dx_min.  Walls, when given, lie on the index lines i = 0, nx-1 / j = 0, ny-1. */
    const double* metric;
    /* mass source R of eq. 2.1.1 (the alpha = 0 source of eq. 2.1.2): ny*nx entries, or NULL
     * for R = 0.  Enters the pressure of eq. 2.3.23; needs a Newtonian fluid (pl_n = 1). */
    const double* mass_source;
    /* 1: also advance the alpha = 0 distributions (rho0 of eq. 2.1.2), which Remark 1 says
     * the velocity equations do not need; a check of that remark.  Periodic axes and a
     * Newtonian fluid only.  0: not carried. */
    int32_t track_rho0;
    /* 1: add the sources G and G_bar of eqs. 2.2.7 and 2.2.10 with their time-derivative
     * terms (eqs. 2.2.1 and 2.2.11), which Remark 2 drops, taking d_t of the momentum flux
     * u_alpha u + P E_alpha by backward differences over the previous steps (zero until
     * those steps exist).  Newtonian fluid only.  0: dropped, as in every computation of
     * the paper. */
    int32_t flux_source;
} orc_params;

typedef struct orc_state orc_state;

/* Create a state initialised with f_hat = f^eq(u0, v0, p0) (Sec. 4, first
 * paragraph), then the wall rule applied to it.  Returns NULL on bad input. */
orc_state* orc_create(const orc_params* p, const double* u0, const double* v0, const double* p0);
void       orc_destroy(orc_state* st);
void       orc_step(orc_state* st, int32_t nsteps);
double     orc_dt(const orc_state* st);
int64_t    orc_steps(const orc_state* st);
void       orc_get_f(const orc_state* st, double* f);
void       orc_set_f(orc_state* st, const double* f);
/* intermediate fields of the last step: 0 f_hat^+(t), 1 f_bar^+(t), 2 f_bar(t+h), 3 f(t+h) */
void       orc_fields(const orc_state* st, int32_t which, double* out);
void       orc_moments(const orc_state* st, double* u, double* v, double* p);
/* 14 planes, each ny*nx: ux uy vx vy div Sxx Sxy Syy sig_xx sig_xy sig_yy Omega_xy omega nu */
void       orc_derived(const orc_state* st, double* out);
/* 8 scalars: sum u, sum v, KE, enstrophy, max|u|, max|FD div u|, non-finite count, area */
void       orc_diagnostics(const orc_state* st, double* out);
/* rho0 = sum_j f_hat_{j,0} at every node (ny*nx); needs track_rho0 */
int32_t    orc_rho0(const orc_state* st, double* out);
/* threads of the OpenMP build (no effect in the sequential build); returns the count in use */
int32_t    orc_set_threads(int32_t n);

/* ---- pieces exposed so that tests can pin them one by one ---- */
/* f^eq for one node (eq. 2.2.5): out[alpha*5+j] */
void   orc_feq(double c, double u, double v, double P, double* out);
/* moments of any stored form: u, v, P (eq. 2.3.23 with R = 0) */
void   orc_node_moments(double c, const double* phi, double* u, double* v, double* P);
/* pressure of eq. 2.3.23 with a mass source R at a node whose stored form is
 * phi = f + kappa Lambda~ (f - f^eq) of the state's Newtonian collision matrix, by solving
 * the definition for P; form 0: kappa = dt/2 (f_hat), 1: h/2 (f_bar), 2: -h/2 (f_bar^+),
 * 3: 0 (f).  Returns NaN for a form outside 0..3 or a power-law state. */
double orc_form_pressure(const orc_state* st, const double* phi, int32_t form, double R);
/* collision matrices for rates (s, s'), time step dt (5x5, row-major):
 *   out[0]  = Lambda~                        (eq. 2.2.4 MRT matrix)
 *   out[25] = I - Lambda                     (eq. 2.2.14)
 *   out[50] = I - 3/4 Lambda                 (eq. 2.2.15)
 *   out[75] = (I + h/2 Lambda~)^-1           (eq. 2.2.16, h = dt/2)
 *   out[100]= (I + dt/2 Lambda~)^-1          (inverse of eq. 2.2.2)     */
void   orc_collision_matrices(double s, double sp, double dt, double* out);
/* one full collision of Step (1) at a node: fhat -> (fhat_plus, fbar_plus) */
void   orc_collide_step1(const orc_state* st, const double* fhat, double* fhat_plus, double* fbar_plus);
/* mixed-difference derivative (eqs. 2.2.12-2.2.13) of one plane along an
 * axis (0 = x, 1 = y) for a velocity sign (+1 or -1) at every node where the
 * stencil is evaluated; out is ny*nx. */
void   orc_mixed_derivative(const orc_state* st, const double* field, int32_t axis, int32_t sign, double* out);
/* wall rule applied in place to a 10-plane field */
void   orc_wall_update(const orc_state* st, double* field);
/* local power-law viscosity for a non-equilibrium strain magnitude gam_hat and offset theta */
double orc_powerlaw_nu(const orc_state* st, double gam_hat, double theta);

#ifdef __cplusplus
}
#endif
#endif
