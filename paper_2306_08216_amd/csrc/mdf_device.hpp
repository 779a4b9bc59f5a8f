// Device-side building blocks of the MDF-FDLBM step for gfx950.
//
// Everything here is per node and register-resident.  The collision is the
// O(q) closed form of the MRT operator: with rates s_0 = s_3 = s_4 = s' and
// s_1 = s_2 = s (Sec. 3.1) and an orthogonal moment basis, the constraints of
// eq. 2.2.4 give Lambda~ = s' I + (s - s') P_c with P_c the projector onto the
// first moments, (P_c g)_1 = -(P_c g)_3 = (g_1 - g_3)/2 and likewise for 2/4.
// Any function r(Lambda~) then acts as r(s') g + (r(s) - r(s')) P_c g, so each
// matrix of Steps (1)-(3) reduces to a pair of scalars per rate:
//   a(sig) = (1 - sig dt/2)/(1 + sig dt/2)   I - Lambda            (eq. 2.2.14)
//   b(sig) = (1 + 3 a(sig))/4                I - 3/4 Lambda        (eq. 2.2.15)
//   q(sig) = 1/(1 + sig dt/4)                (I + h/2 Lambda~)^-1  (eq. 2.2.16)
// and the mid-step collision (I + h/2 L~)^-1 (f_bar + h/2 L~ f^eq) equals
// f^eq + R_q(f_bar - f^eq) because the moments of f_bar equal those of f.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mdf {

enum : int { PL_NEWTON = 0, PL_HALF = 1, PL_THREE_HALVES = 2 };

// Checking build (libmdf_poison.so, compiled with MDF_POISON_LDS=1): every
// LDS slot a kernel is about to publish in is first set to NaN, so a read of a
// slot that no thread wrote for this row or tile carries a NaN into the
// state, where the parity tests see it.  The released library has it off.
#ifndef MDF_POISON_LDS
#define MDF_POISON_LDS 0
#endif
constexpr bool kPoisonLds = MDF_POISON_LDS != 0;
__device__ __forceinline__ double lds_poison_value() { return __builtin_nan(""); }

// Constants of one run, computed on the host at mdf_init and passed by value.
struct StepConsts {
    int nx, ny;
    int bcx, bcy;            // 0 periodic, 1 wall
    int pl;                  // PL_*
    int pitch;               // nodes per row of the node-major state (>= nx)
    double c, w, kf;         // lattice speed, weight 1/5, w c / c_s^2
    double cs2, dt, h;
    double eta, one_m_eta;
    double st_a, st_b, st_c, st_d;   // mixed-difference weights (see transport_pos)
    int uniform;                     // both axes uniform: stencil coefficients below are valid
    double sh[2][4], sd[2][4];       // folded stencils per axis for the half (tau = h, centre + 1)
                                     // and full (tau = dt) updates, see make_stencil
    double lid_u;
    // Newtonian relaxation factors for (s, s')
    double a_s, a_p, b_s, b_p, q_s, q_p;
    double nu;               // Newtonian viscosity or power-law K
    double nu_min, nu_max, s_ratio;
    double theta1, theta3;   // c_s^2 dt/2 and c_s^2 dt/4
    // transport coefficients: tau * c / 2 for tau = h and tau = dt
    double lam_h, lam_dt;
    // body force terms h w F_alpha and dt w F_alpha of a uniform force
    double hwf[2], dwf[2];
    const double* gx;        // nx derivative scales 1/(X' dxi), or null on a uniform grid
    const double* gy;        // ny derivative scales, or null
    double ginv[2];          // 1/dx and 1/dy of the uniform spacing (used where gx, gy are null)
    // steady force field (eq. 2.2.6 with F depending on x): (F_x, F_y) per node,
    // rows of pitch nodes, uniform part included; null for a uniform force.
    // Steps (2) and (4) then add hw F and dw F with hw = h w, dw = dt w.
    const double* ff;
    // general mapping: 4 planes of nx*ny (d i/dx, d i/dy, d j/dx, d j/dy per node), or null
    const double* met;
    double hw, dw;
    // mass source R of eq. 2.1.1: nx*ny values (row y at y*nx), or null for R = 0.
    // The pressure of eq. 2.3.23 is defined on f; a stored form phi = f + kappa
    // Lambda~ (f - f^eq) has the first-moment trace of f shifted by kappa c_s^2 R
    // (the collision scales first moments by s and s nu = c_s^2), so its pressure
    // is the plain sum of node_moments plus R (nu + kappa c_s^2)/2.  Per unit R:
    // r_hat (f_hat, kappa = dt/2), r_bar (f_bar, h/2), r_bp (f_bar^+, -h/2), r_f (f).
    const double* rsrc;
    double r_hat, r_bar, r_bp, r_f;
};

// State layout (row-split).  Row y occupies 80*pitch contiguous bytes: first
// the x-part block, pitch nodes x 6 doubles holding the components streamed
// along x or not at all (j = 0, 1, 3 of the u set, then of the v set), then the
// y-part block, pitch nodes x 4 doubles holding the components streamed along
// y (j = 2, 4 of the u set, then of the v set).  A fused step writes the x
// part and the y part of a node at different times (the y stencil needs two
// more rows); with this split each write covers whole cache lines of one
// block.  Components are numbered q = alpha*5 + j as in the method.
__host__ __device__ constexpr int comp_slot(int q)   // slot within its block
{
    return (q % 5 == 2 || q % 5 == 4) ? 2 * (q / 5) + (q % 5 == 4) : 3 * (q / 5) + (q % 5 == 0 ? 0 : (q % 5 == 1 ? 1 : 2));
}
__host__ __device__ constexpr bool comp_in_xpart(int q) { return !(q % 5 == 2 || q % 5 == 4); }

__device__ __forceinline__ size_t xpart_off(int pitch, int x, int y) { return (size_t)y * pitch * 10 + (size_t)x * 6; }
__device__ __forceinline__ size_t ypart_off(int pitch, int x, int y)
{
    return (size_t)y * pitch * 10 + (size_t)pitch * 6 + (size_t)x * 4;
}
__device__ __forceinline__ size_t comp_off(int pitch, int x, int y, int q)
{
    return comp_in_xpart(q) ? xpart_off(pitch, x, y) + comp_slot(q) : ypart_off(pitch, x, y) + comp_slot(q);
}

__device__ __forceinline__ void load_node(const double* __restrict__ f, int pitch, int x, int y, double* phi)
{
    const double2* px = reinterpret_cast<const double2*>(f + xpart_off(pitch, x, y));
    const double2* py = reinterpret_cast<const double2*>(f + ypart_off(pitch, x, y));
    const double2 a = px[0], b = px[1], c = px[2], d = py[0], e = py[1];
    phi[0] = a.x; phi[1] = a.y; phi[3] = b.x;   // u set j = 0, 1, 3
    phi[5] = b.y; phi[6] = c.x; phi[8] = c.y;   // v set j = 0, 1, 3
    phi[2] = d.x; phi[4] = d.y;                 // u set j = 2, 4
    phi[7] = e.x; phi[9] = e.y;                 // v set j = 2, 4
}

__device__ __forceinline__ void store_node(double* __restrict__ f, int pitch, int x, int y, const double* phi)
{
    double2* px = reinterpret_cast<double2*>(f + xpart_off(pitch, x, y));
    double2* py = reinterpret_cast<double2*>(f + ypart_off(pitch, x, y));
    px[0] = make_double2(phi[0], phi[1]);
    px[1] = make_double2(phi[3], phi[5]);
    px[2] = make_double2(phi[6], phi[8]);
    py[0] = make_double2(phi[2], phi[4]);
    py[1] = make_double2(phi[7], phi[9]);
}

// Workgroup barrier that orders LDS traffic only.  __syncthreads() also
// fences global memory, which makes every wave drain its outstanding global
// loads (vmcnt 0) at the barrier and so cancels any row prefetch in flight.
// The fused kernels exchange data between waves through LDS alone, so the
// barrier only needs LDS (lgkm) completion.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Exchange barrier for a workgroup of NW waves.  One wave needs no hardware
// barrier: LDS executes a wave's accesses in issue order, so only the compiler
// must be kept from moving LDS accesses across the exchange point.
template <int NW>
__device__ __forceinline__ void exchange_barrier()
{
    if constexpr (NW == 1) {
        __builtin_amdgcn_wave_barrier();
    } else {
        lds_barrier();
    }
}

// Raw buffer access to one row of the state.  The descriptor lives in scalar
// registers; with stride 0 the hardware checks each access against
// num_records: loads past it return zero and stores past it are dropped.
typedef __amdgpu_buffer_rsrc_t BufRes;
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef int ivec4 __attribute__((ext_vector_type(4)));
typedef int ivec2 __attribute__((ext_vector_type(2)));
constexpr int kBufWord3 = 0x00020000;   // 32-bit data format for gfx9 raw buffers

// descriptor of row `row` (row_bytes bytes) of f; `on` false gives no records
__device__ __forceinline__ BufRes row_res(const double* f, int row_bytes, int row, bool on)
{
    const char* p = reinterpret_cast<const char*>(f) + (size_t)row * (size_t)row_bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), 0, on ? row_bytes : 0, kBufWord3);
}

__device__ __forceinline__ dvec2 buf_load2(BufRes r, unsigned off)
{
    return __builtin_bit_cast(dvec2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

__device__ __forceinline__ void buf_store2(BufRes r, unsigned off, dvec2 v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(ivec4, v), r, off, 0, 0);
}

__device__ __forceinline__ void buf_store1(BufRes r, unsigned off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(ivec2, v), r, off, 0, 0);
}

struct Relax {               // a relaxation pair kappa (rate s), kappa' (rate s')
    double k, kp;
};

__device__ __forceinline__ void node_moments(const double* phi, double c, double& u, double& v, double& P)
{
    u = ((phi[0] + phi[1]) + (phi[2] + phi[3])) + phi[4];
    v = ((phi[5] + phi[6]) + (phi[7] + phi[8])) + phi[9];
    // sum_alpha sum_j c_{j,alpha} phi_{j,alpha}: x-moment of the u set plus y-moment of the v set
    const double q = c * ((phi[1] - phi[3]) + (phi[7] - phi[9]));
    P = 0.5 * (q - (u * u + v * v));
}

// Linear equilibrium of eq. 2.2.5 for both velocity components.
__device__ __forceinline__ void equilibrium(double u, double v, double P, const StepConsts& K, double* fe)
{
    const double fxu = u * u + P, fyu = u * v;   // flux of the u equation
    const double fxv = v * u, fyv = v * v + P;   // flux of the v equation
    const double bu = K.w * u, bv = K.w * v;
    fe[0] = bu;
    fe[1] = bu + K.kf * fxu;
    fe[2] = bu + K.kf * fyu;
    fe[3] = bu - K.kf * fxu;
    fe[4] = bu - K.kf * fyu;
    fe[5] = bv;
    fe[6] = bv + K.kf * fxv;
    fe[7] = bv + K.kf * fyv;
    fe[8] = bv - K.kf * fxv;
    fe[9] = bv - K.kf * fyv;
}

// out = f^eq + R_{k,k'}(phi - f^eq)
__device__ __forceinline__ void relax(const double* phi, const double* fe, Relax r, double* out)
{
    const double dk = 0.5 * (r.k - r.kp);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const double* p = phi + 5 * a;
        const double* e = fe + 5 * a;
        double* o = out + 5 * a;
        const double g0 = p[0] - e[0], g1 = p[1] - e[1], g2 = p[2] - e[2], g3 = p[3] - e[3], g4 = p[4] - e[4];
        const double dx = dk * (g1 - g3), dy = dk * (g2 - g4);
        o[0] = e[0] + r.kp * g0;
        o[1] = e[1] + (r.kp * g1 + dx);
        o[3] = e[3] + (r.kp * g3 - dx);
        o[2] = e[2] + (r.kp * g2 + dy);
        o[4] = e[4] + (r.kp * g4 - dy);
    }
}

// 2 S^:S^ (the square of the non-equilibrium strain magnitude) with
// S^ = -sym(M^ne), M^ne_{ab} = sum_j c_{j,b} (phi - f^eq)_{j,a}.
__device__ __forceinline__ double noneq_shear_sq(const double* phi, const double* fe, double c)
{
    const double mxx = c * ((phi[1] - fe[1]) - (phi[3] - fe[3]));
    const double mxy = c * ((phi[2] - fe[2]) - (phi[4] - fe[4]));
    const double myx = c * ((phi[6] - fe[6]) - (phi[8] - fe[8]));
    const double myy = c * ((phi[7] - fe[7]) - (phi[9] - fe[9]));
    const double s12 = 0.5 * (mxy + myx);
    return 2.0 * (mxx * mxx + myy * myy + 2.0 * s12 * s12);
}

// 1/x for a positive normal x: the hardware reciprocal after two Newton
// refinements, each of which squares its relative error, so the result is
// within rounding of 1/x at a third of the cost of an IEEE division.
__device__ __forceinline__ double rcp_refined(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// 1/sqrt(x) for a positive normal x: the hardware estimate after two Newton
// steps y <- y (3/2 - x y^2 / 2), each of which roughly squares the relative
// error; sqrt(x) from it with one more correction s <- s + y (x - s^2)/2.
// The general library routines also handle zero, infinities and subnormal
// arguments with scaling and class tests; the power-law solve never passes
// those (a zero strain rate takes its own branch), and the refined estimates
// agree with the correctly rounded values to an ulp or two.
__device__ __forceinline__ double rsqrt_refined(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    return y * fma(-hx * y, y, 1.5);
}

__device__ __forceinline__ double sqrt_refined(double x)
{
    const double y = rsqrt_refined(x);
    const double s = x * y;
    return fma(0.5 * y, fma(-s, s, x), s);
}

// Local power-law viscosity nu = K (g/(nu + theta))^(n-1), clamped, from the
// squared strain magnitude q = g^2:
//  n = 1/2: positive root of nu^2 - b nu - b theta = 0 with b = K^2/g, i.e.
//           nu = (b + sqrt(b (b + 4 theta)))/2;
//  n = 3/2: root of nu^3 + theta nu^2 - K^2 g = 0 by three Halley steps from
//           an upper bound of the root: nu^3 and theta nu^2 each stay below
//           r = K^2 g, so nu <= min(r^(1/3), sqrt(r/theta)).  The cube root is
//           read from the exponent bits: a third of r's bit pattern plus two
//           thirds of the exponent bias is 2^(log2(r)/3) with the mantissa
//           interpolated linearly, which overestimates r^(1/3) by 0-5.9 %.
//           The start is then within 34 % of the root for every g and theta,
//           and Halley's cubic convergence takes that to a 1-ulp root in three
//           steps; a fixed count keeps every lane of a wave on the same
//           instructions.  The first two steps divide by the raw hardware
//           reciprocal: its error perturbs only their corrections, which the
//           next step's cubic convergence removes.  The last step, whose
//           correction is below 1e-6 of the root, refines the reciprocal once.
//           A root beyond the clamp range is clamped like the n = 1/2 one.
template <int PL>
__device__ __forceinline__ double powerlaw_nu_sq_t(const StepConsts& K, double q, double theta)
{
    const double Kc = K.nu;
    // A node at rest (q = 0) takes the clamp bound its index gives; it runs the
    // same instructions on a stand-in q = 1 and selects, so that no lane
    // branches and the collisions around stay one basic block.
    const bool rest = q == 0.0;
    q = rest ? 1.0 : q;
    double nu;
    if constexpr (PL == PL_HALF) {
        const double b = Kc * Kc * rsqrt_refined(q);
        nu = 0.5 * (b + sqrt_refined(b * (b + 4.0 * theta)));
        nu = rest ? K.nu_max : nu;
    } else {
        const double r = Kc * Kc * sqrt_refined(q);
        const unsigned long long rb = static_cast<unsigned long long>(__double_as_longlong(r));
        const double cb = __longlong_as_double(static_cast<long long>(rb / 3ull + (682ull << 52)));
        // the start needs no accuracy (the steps absorb a relative error of
        // 2^-8 in it), so sqrt(r/theta) is the raw estimate
        const double rt = r * (1.0 / theta);
        double x = fmin(cb, rt * __builtin_amdgcn_rsq(rt));
#pragma unroll
        for (int it = 0; it < 3; ++it) {
            const double f = x * x * (x + theta) - r;
            const double d1 = x * (3.0 * x + 2.0 * theta);
            const double d2 = 6.0 * x + 2.0 * theta;
            const double den = 2.0 * d1 * d1 - f * d2;
            double y = __builtin_amdgcn_rcp(den);
            // an error in the first two corrections is absorbed by the next
            // step; only the last one needs the refined reciprocal
            if (it == 2) y = fma(y, fma(-den, y, 1.0), y);
            x -= 2.0 * f * d1 * y;
        }
        nu = rest ? K.nu_min : x;
    }
    return fmin(fmax(nu, K.nu_min), K.nu_max);
}

// The same with the index read from the constants at run time.
__device__ __forceinline__ double powerlaw_nu_sq(const StepConsts& K, double q, double theta)
{
    if (K.pl == PL_HALF) return powerlaw_nu_sq_t<PL_HALF>(K, q, theta);
    return powerlaw_nu_sq_t<PL_THREE_HALVES>(K, q, theta);
}

// Relaxation factors at a local viscosity nu, with s = c_s^2/nu and
// s' = s_ratio s.  a(s) = (1 - s dt/2)/(1 + s dt/2) = (nu - t1)/(nu + t1) and
// q(s) = 1/(1 + s dt/4) = nu/(nu + t3) with t1 = c_s^2 dt/2, t3 = c_s^2 dt/4;
// the two rates of a pair share one reciprocal.
__device__ __forceinline__ void relax_ab_nu(const StepConsts& K, double nu, Relax& ra, Relax& rb)
{
    const double t = K.theta1, tp = K.s_ratio * K.theta1;
    const double d = nu + t, dp = nu + tp, inv = rcp_refined(d * dp);
    const double as = (nu - t) * dp * inv, ap = (nu - tp) * d * inv;
    ra = Relax{as, ap};
    rb = Relax{0.25 * (1.0 + 3.0 * as), 0.25 * (1.0 + 3.0 * ap)};
}

__device__ __forceinline__ Relax relax_q_nu(const StepConsts& K, double nu)
{
    const double t = K.theta3, tp = K.s_ratio * K.theta3;
    const double d = nu + t, dp = nu + tp, inv = nu * rcp_refined(d * dp);
    return Relax{dp * inv, d * inv};
}

// Step (1) factors for a node: a(s), a(s') (f_hat^+) and b(s), b(s') (f_bar^+).
template <int PL>
__device__ __forceinline__ void step1_factors_t(const StepConsts& K, const double* fh, const double* fe, Relax& ra,
                                                Relax& rb)
{
    if (PL == PL_NEWTON) {
        ra = Relax{K.a_s, K.a_p};
        rb = Relax{K.b_s, K.b_p};
        return;
    }
    relax_ab_nu(K, powerlaw_nu_sq_t<PL>(K, noneq_shear_sq(fh, fe, K.c), K.theta1), ra, rb);
}

// Step (3) factors q(s), q(s') for the collision of f_bar.
template <int PL>
__device__ __forceinline__ Relax step3_factors_t(const StepConsts& K, const double* fb, const double* fe)
{
    if (PL == PL_NEWTON) return Relax{K.q_s, K.q_p};
    return relax_q_nu(K, powerlaw_nu_sq_t<PL>(K, noneq_shear_sq(fb, fe, K.c), K.theta3));
}

__device__ __forceinline__ void step1_factors(const StepConsts& K, const double* fh, const double* fe, Relax& ra,
                                              Relax& rb)
{
    if (K.pl == PL_NEWTON)
        step1_factors_t<PL_NEWTON>(K, fh, fe, ra, rb);
    else if (K.pl == PL_HALF)
        step1_factors_t<PL_HALF>(K, fh, fe, ra, rb);
    else
        step1_factors_t<PL_THREE_HALVES>(K, fh, fe, ra, rb);
}

__device__ __forceinline__ Relax step3_factors(const StepConsts& K, const double* fb, const double* fe)
{
    if (K.pl == PL_NEWTON) return step3_factors_t<PL_NEWTON>(K, fb, fe);
    if (K.pl == PL_HALF) return step3_factors_t<PL_HALF>(K, fb, fe);
    return step3_factors_t<PL_THREE_HALVES>(K, fb, fe);
}

// The node-level updates below take the pressure offset dP of a mass source
// (R times the stored form's coefficient in StepConsts) when SRC is set; with
// SRC unset they are the plain updates of a run without source.
template <bool SRC>
__device__ __forceinline__ void moments_equilibrium(const StepConsts& K, const double* phi, double dP, double& u,
                                                    double& v, double& P, double* fe)
{
    node_moments(phi, K.c, u, v, P);
    if constexpr (SRC) P += dP;
    equilibrium(u, v, P, K, fe);
}

// Step (1): f_hat -> f_hat^+ (eq. 2.2.14) and f_bar^+ (eq. 2.2.15).
template <bool SRC = false>
__device__ __forceinline__ void collide1(const StepConsts& K, const double* fh, double* fhp, double* fbp,
                                         double dP = 0.0)
{
    double u, v, P, fe[10];
    moments_equilibrium<SRC>(K, fh, dP, u, v, P, fe);
    Relax ra, rb;
    step1_factors(K, fh, fe, ra, rb);
    relax(fh, fe, ra, fhp);
    relax(fh, fe, rb, fbp);
}

template <bool SRC = false>
__device__ __forceinline__ void collide1_bar(const StepConsts& K, const double* fh, double* fbp, double dP = 0.0)
{
    double u, v, P, fe[10];
    moments_equilibrium<SRC>(K, fh, dP, u, v, P, fe);
    Relax ra, rb;
    step1_factors(K, fh, fe, ra, rb);
    relax(fh, fe, rb, fbp);
}

template <bool SRC = false>
__device__ __forceinline__ void collide1_hat(const StepConsts& K, const double* fh, double* fhp, double dP = 0.0)
{
    double u, v, P, fe[10];
    moments_equilibrium<SRC>(K, fh, dP, u, v, P, fe);
    Relax ra, rb;
    step1_factors(K, fh, fe, ra, rb);
    relax(fh, fe, ra, fhp);
}

// Step (3): f(t+h) = f^eq + R_q(f_bar - f^eq) (eq. 2.2.16).
template <bool SRC = false>
__device__ __forceinline__ void collide3(const StepConsts& K, const double* fb, double* f, double dP = 0.0)
{
    double u, v, P, fe[10];
    moments_equilibrium<SRC>(K, fb, dP, u, v, P, fe);
    const Relax rq = step3_factors(K, fb, fe);
    relax(fb, fe, rq, f);
}

// Wall rule: Pi(w) = f^eq(u_w, P_1) + 2 [Pi(1) - f^eq(1)] - [Pi(2) - f^eq(2)]
// (dP1, dP2: the pressure offsets of a mass source at the two neighbours).
template <bool SRC = false>
__device__ __forceinline__ void wall_extrapolate(const StepConsts& K, const double* p1, const double* p2, double uw,
                                                 double* out, double dP1 = 0.0, double dP2 = 0.0)
{
    double u1, v1, P1, u2, v2, P2, e1[10], e2[10], ew[10];
    moments_equilibrium<SRC>(K, p1, dP1, u1, v1, P1, e1);
    moments_equilibrium<SRC>(K, p2, dP2, u2, v2, P2, e2);
    equilibrium(uw, 0.0, P1, K, ew);
#pragma unroll
    for (int k = 0; k < 10; ++k) out[k] = ew[k] + 2.0 * (p1[k] - e1[k]) - (p2[k] - e2[k]);
}

// mass source at node (x, y) (StepConsts::rsrc must be set)
__device__ __forceinline__ double source_at(const StepConsts& K, int x, int y)
{
    return K.rsrc[(size_t)y * K.nx + x];
}

// tau c_j . grad Pi for the velocity of sign sg along one axis with the mixed
// scheme; lam = tau c / 2 and g = 1/(X' dxi) at the node, lamg = lam g.
//   c > 0: lamg [eta (P1 - Pm1) + (1-eta)(3 P0 - 4 Pm1 + Pm2)]
//   c < 0: -lamg [eta (P1 - Pm1) - (1-eta)(3 P0 - 4 P1 + P2)]
// written as four-point weighted sums with w_a = 1-eta, w_b = -(4-3 eta),
// w_c = 3(1-eta), w_d = eta (the c < 0 branch is the mirror image).
__device__ __forceinline__ double transport_pos(const StepConsts& K, double lamg, double pm2, double pm1, double p0,
                                                double p1)
{
    return lamg * (K.st_a * pm2 + K.st_b * pm1 + K.st_c * p0 + K.st_d * p1);
}

__device__ __forceinline__ double transport_neg(const StepConsts& K, double lamg, double pm1, double p0, double p1,
                                                double p2)
{
    return lamg * (K.st_d * pm1 + K.st_c * p0 + K.st_b * p1 + K.st_a * p2);
}

// Folded stencil of one axis: new = base + k_a Pm2 + k_b Pm1 + k_c P0 + k_d P1
// for c > 0 (mirror order for c < 0), with k_x = -lamg w_x, plus 1 on the
// centre weight when the stenciled field itself is the one being advanced
// (the half step f_bar = f_bar^+ - h c.grad f_bar^+).  Four FMAs per update.
struct Stencil {
    double a, b, c, d;
};

__host__ __device__ inline Stencil make_stencil(const StepConsts& K, double lamg, bool centre_one)
{
    return Stencil{-lamg * K.st_a, -lamg * K.st_b, (centre_one ? 1.0 : 0.0) - lamg * K.st_c, -lamg * K.st_d};
}

__device__ __forceinline__ Stencil stencil_of(const double* s4) { return Stencil{s4[0], s4[1], s4[2], s4[3]}; }

__device__ __forceinline__ double upd_pos(const Stencil& k, double base, double pm2, double pm1, double p0, double p1)
{
    return fma(k.d, p1, fma(k.c, p0, fma(k.b, pm1, fma(k.a, pm2, base))));
}

__device__ __forceinline__ double upd_neg(const Stencil& k, double base, double pm1, double p0, double p1, double p2)
{
    return fma(k.a, p2, fma(k.b, p1, fma(k.c, p0, fma(k.d, pm1, base))));
}

__device__ __forceinline__ double ghost(double p0, double p1, double p2) { return 3.0 * p0 - 3.0 * p1 + p2; }

// derivative scale of column x and row y: the metric arrays where the run has
// them, else the uniform 1/dx, 1/dy (batch instances carry no arrays)
__device__ __forceinline__ double gx_at(const StepConsts& K, int x) { return K.gx ? K.gx[x] : K.ginv[0]; }
__device__ __forceinline__ double gy_at(const StepConsts& K, int y) { return K.gy ? K.gy[y] : K.ginv[1]; }

// h w F_alpha and dt w F_alpha at node (x, y) for alpha index a: the force
// field when one is set, else the uniform force
__device__ __forceinline__ double hwf_at(const StepConsts& K, int x, int y, int a)
{
    return K.ff ? K.hw * K.ff[((size_t)y * K.pitch + x) * 2 + a] : K.hwf[a];
}

__device__ __forceinline__ double dwf_at(const StepConsts& K, int x, int y, int a)
{
    return K.ff ? K.dw * K.ff[((size_t)y * K.pitch + x) * 2 + a] : K.dwf[a];
}

__device__ __forceinline__ bool is_wall(const StepConsts& K, int x, int y)
{
    return (K.bcx && (x == 0 || x == K.nx - 1)) || (K.bcy && (y == 0 || y == K.ny - 1));
}

}  // namespace mdf
