// C ABI of the MDF-FDLBM library: parameter validation, constants of the
// method, workspace carving and kernel launches.  See include/mdf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mdf.h"
#include "mdf_internal.hpp"

using mdf::StepConsts;

struct mdf_ctx {
    mdf_params p;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    double* f[2] = {nullptr, nullptr};
    double* fbp = nullptr;
    double* fmid = nullptr;
    double* gx = nullptr;
    double* gy = nullptr;
    double* diag_part = nullptr;
    double* diag_out = nullptr;
    int cur = 0;
    int64_t steps = 0;
    int variant = 2;
    mdf::FusedShape shape{64, -1, 2, nullptr, 0};
    int4* seg = nullptr;          // segment table of the balanced partition (device)
    int slots = 1024;             // 64-lane waves one round of the fused step holds (one per SIMD)
    int rounds = 1;               // rounds of workgroups the balanced table fills
    double cx_scale = 1.0, cy_scale = 1.0;   // autotuned scalings of the wall-row cost factors
    StepConsts K;
    std::string err;
};

namespace {

thread_local std::string g_err;

mdf_status fail(mdf_ctx* c, mdf_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    g_err = buf;
    return s;
}

mdf_status hip_check(mdf_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return MDF_OK;
    return fail(c, MDF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

struct Layout {
    size_t pitch;                 // nodes per row
    size_t off_f0, off_f1, off_fbp, off_fmid, off_gx, off_gy, off_dp, off_do, off_seg, off_ff, off_met, off_rs,
        total;  // bytes
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr int kSegCap = 4096;   // entries of the segment table (one per workgroup)

bool has_force_field(const mdf_params* p) { return p->force_x != nullptr || p->force_y != nullptr; }

Layout layout_for(int nx, int ny, bool force_field, bool metric, bool source)
{
    Layout L;
    // rows of 80 bytes per node (x-part block, then y-part block); 16-node multiples keep
    // rows and both blocks 256-byte aligned
    L.pitch = ((size_t)nx + 15) & ~size_t(15);
    const size_t fbytes = align256(10 * L.pitch * (size_t)ny * sizeof(double));
    size_t o = 0;
    L.off_f0 = o;   o += fbytes;
    L.off_f1 = o;   o += fbytes;
    L.off_fbp = o;  o += fbytes;
    L.off_fmid = o; o += fbytes;
    L.off_gx = o;   o += align256((size_t)nx * sizeof(double));
    L.off_gy = o;   o += align256((size_t)ny * sizeof(double));
    L.off_dp = o;   o += align256(8 * (size_t)mdf::kDiagMaxBlocks * sizeof(double));
    L.off_do = o;   o += align256(16 * sizeof(double));   // diagnostics result (8), closure guard state (4)
    L.off_seg = o;  o += align256(kSegCap * sizeof(int4));
    // force field: (F_x, F_y) per node in rows of pitch nodes
    L.off_ff = o;   o += force_field ? align256(2 * L.pitch * (size_t)ny * sizeof(double)) : 0;
    // general mapping: 4 planes of nx*ny metric values
    L.off_met = o;  o += metric ? align256(4 * (size_t)nx * (size_t)ny * sizeof(double)) : 0;
    // mass source: one plane of nx*ny values
    L.off_rs = o;   o += source ? align256((size_t)nx * (size_t)ny * sizeof(double)) : 0;
    L.total = o;
    return L;
}

const char* validate(const mdf_params* p)
{
    if (!p) return "params is NULL";
    if (p->nx < 5 || p->ny < 5) return "nx and ny must be >= 5";
    if (p->nx > 32768 || p->ny > 32768) return "nx and ny must be <= 32768";
    if (!(p->lx > 0.0) || !(p->ly > 0.0)) return "lx and ly must be > 0";
    if (!(p->nu > 0.0)) return "nu must be > 0";
    if (!(p->cfl > 0.0)) return "cfl must be > 0";
    if (!(p->c > 0.0)) return "c must be > 0";
    if (!(p->eta >= 0.0 && p->eta <= 1.0)) return "eta must lie in [0, 1]";
    if (!(p->s_ratio > 0.0)) return "s_ratio must be > 0";
    if (p->bc_x != MDF_BC_PERIODIC && p->bc_x != MDF_BC_WALL) return "bc_x must be MDF_BC_PERIODIC or MDF_BC_WALL";
    if (p->bc_y != MDF_BC_PERIODIC && p->bc_y != MDF_BC_WALL) return "bc_y must be MDF_BC_PERIODIC or MDF_BC_WALL";
    if (!(p->pl_n == 1.0 || p->pl_n == 0.5 || p->pl_n == 1.5)) return "pl_n must be 1, 0.5 or 1.5";
    if (p->pl_n != 1.0 && !(p->nu_min > 0.0 && p->nu_max >= p->nu_min)) return "power law needs 0 < nu_min <= nu_max";
    if ((p->inv_dx_x || p->inv_dx_y) && !(p->dx_min > 0.0)) return "metric arrays need dx_min > 0";
    if (!std::isfinite(p->fx) || !std::isfinite(p->fy) || !std::isfinite(p->lid_u)) return "non-finite force or lid speed";
    if (p->force_harmonic != 0 && p->force_harmonic != 1) return "force_harmonic must be 0 or 1";
    if (p->force_harmonic && !(std::isfinite(p->force_omega) && std::isfinite(p->force_phase)))
        return "non-finite force_omega or force_phase";
    if (p->metric && (p->inv_dx_x || p->inv_dx_y)) return "a general mapping (metric) excludes inv_dx_x and inv_dx_y";
    if (p->metric && !(p->dx_min > 0.0)) return "a general mapping needs dx_min > 0";
    if (p->mass_source && p->pl_n != 1.0) return "a mass source needs a Newtonian fluid (pl_n = 1)";
    return nullptr;
}

Layout layout_of(const mdf_params* p)
{
    return layout_for(p->nx, p->ny, has_force_field(p), p->metric != nullptr, p->mass_source != nullptr);
}

// Force terms of the step that starts at time t = step * dt for a force
// F(x) cos(omega t + phase): the half step adds h w F(t) (eq. 2.3.25), the full
// step dt w F(t) + (dt^2/2) w d_t F(t) (eq. 2.3.24).  The kernels read them as
// the scalars h w F_alpha and dt w F_alpha of the uniform force, and h w and
// dt w that multiply a force field node by node.
void set_force_time(StepConsts& K, const mdf_params& p, int64_t step)
{
    const double t = (double)step * K.dt;
    const double m = std::cos(p.force_omega * t + p.force_phase);
    const double dm = -p.force_omega * std::sin(p.force_omega * t + p.force_phase);
    const double F[2] = {p.fx, p.fy};
    for (int a = 0; a < 2; ++a) {
        K.hwf[a] = K.h * K.w * F[a] * m;
        K.dwf[a] = K.dt * K.w * F[a] * m + 0.5 * K.dt * K.dt * K.w * F[a] * dm;
    }
    K.hw = K.h * K.w * m;
    K.dw = K.dt * K.w * m + 0.5 * K.dt * K.dt * K.w * dm;
}

// Constants of the method for one run (Sec. 2.2; eq. 3.1 for dt).
StepConsts make_consts(const mdf_params& p, const Layout& L)
{
    StepConsts K{};
    K.nx = p.nx;
    K.ny = p.ny;
    K.bcx = p.bc_x;
    K.bcy = p.bc_y;
    K.pl = p.pl_n == 1.0 ? mdf::PL_NEWTON : (p.pl_n == 0.5 ? mdf::PL_HALF : mdf::PL_THREE_HALVES);
    K.pitch = (int)L.pitch;
    K.c = p.c;
    K.w = 0.2;                                  // D2Q5 weights 1/5
    K.cs2 = 0.4 * p.c * p.c;                    // sum_j w_j c_jx^2 = 2c^2/5
    K.kf = K.w * p.c / K.cs2;
    const double hx = p.bc_x == MDF_BC_WALL ? p.lx / (p.nx - 1) : p.lx / p.nx;
    const double hy = p.bc_y == MDF_BC_WALL ? p.ly / (p.ny - 1) : p.ly / p.ny;
    const double dxmin = (p.inv_dx_x || p.inv_dx_y || p.metric) ? p.dx_min : (hx < hy ? hx : hy);
    K.dt = p.cfl * dxmin / p.c;
    K.h = 0.5 * K.dt;
    K.eta = p.eta;
    K.one_m_eta = 1.0 - p.eta;
    K.st_a = 1.0 - p.eta;
    K.st_b = -(4.0 - 3.0 * p.eta);
    K.st_c = 3.0 * (1.0 - p.eta);
    K.st_d = p.eta;
    K.lid_u = p.lid_u;
    K.nu = p.nu;
    K.nu_min = p.nu_min;
    K.nu_max = p.nu_max;
    K.s_ratio = p.s_ratio;
    K.theta1 = 0.5 * K.cs2 * K.dt;
    K.theta3 = 0.25 * K.cs2 * K.dt;
    const double s = K.cs2 / p.nu, sp = p.s_ratio * s;
    auto a = [&](double sig) { return (1.0 - 0.5 * sig * K.dt) / (1.0 + 0.5 * sig * K.dt); };
    K.a_s = a(s);
    K.a_p = a(sp);
    K.b_s = 0.25 * (1.0 + 3.0 * K.a_s);
    K.b_p = 0.25 * (1.0 + 3.0 * K.a_p);
    K.q_s = 1.0 / (1.0 + 0.25 * s * K.dt);
    K.q_p = 1.0 / (1.0 + 0.25 * sp * K.dt);
    K.lam_h = 0.5 * K.h * p.c;
    K.lam_dt = 0.5 * K.dt * p.c;
    K.uniform = (p.inv_dx_x == nullptr && p.inv_dx_y == nullptr && p.metric == nullptr) ? 1 : 0;
    K.ginv[0] = 1.0 / hx;
    K.ginv[1] = 1.0 / hy;
    K.gx = nullptr;
    K.gy = nullptr;
    {
        const double g[2] = {1.0 / hx, 1.0 / hy};
        for (int ax = 0; ax < 2; ++ax) {
            const mdf::Stencil a = mdf::make_stencil(K, K.lam_h * g[ax], true);
            const mdf::Stencil b = mdf::make_stencil(K, K.lam_dt * g[ax], false);
            K.sh[ax][0] = a.a; K.sh[ax][1] = a.b; K.sh[ax][2] = a.c; K.sh[ax][3] = a.d;
            K.sd[ax][0] = b.a; K.sd[ax][1] = b.b; K.sd[ax][2] = b.c; K.sd[ax][3] = b.d;
        }
    }
    K.hwf[0] = K.h * K.w * p.fx;
    K.hwf[1] = K.h * K.w * p.fy;
    K.dwf[0] = K.dt * K.w * p.fx;
    K.dwf[1] = K.dt * K.w * p.fy;
    K.hw = K.h * K.w;
    K.dw = K.dt * K.w;
    K.ff = nullptr;
    K.met = nullptr;
    // pressure offsets per unit mass source of the stored forms (eq. 2.3.23
    // with c_s^2/s = nu): R (nu + kappa c_s^2)/2 for f_hat (kappa = dt/2),
    // f_bar (h/2), f_bar^+ (-h/2) and f (0)
    K.rsrc = nullptr;
    K.r_hat = 0.5 * (p.nu + 0.5 * K.dt * K.cs2);
    K.r_bar = 0.5 * (p.nu + 0.5 * K.h * K.cs2);
    K.r_bp = 0.5 * (p.nu - 0.5 * K.h * K.cs2);
    K.r_f = 0.5 * p.nu;
    return K;
}

// Greedy segmentation of every strip of every grid at cost budget T (row
// units); returns the number of segments, or -1 if some segment cannot hold a
// single row.  A segment of h rows marches h + 8 rows rounded up to whole
// groups of 4 (the kernels' unrolled loop), so its height is chosen with
// h + 8 a multiple of 4 where the budget allows.
int segment_strips(const mdf::PlanGrid* grids, int count, int tile_w, double cx, double cy, double T, int4* out,
                   int cap)
{
    auto rows_for = [](double budget) { return ((int)std::floor(budget) & ~3) - 8; };
    int n = 0;
    for (int g = 0; g < count; ++g) {
        const int nx = grids[g].nx, ny = grids[g].ny;
        const bool wall_x = grids[g].wall_x, wall_y = grids[g].wall_y;
        const int nstrips = (nx + tile_w - 9) / (tile_w - 8);
        for (int s = 0; s < nstrips; ++s) {
            // the strip bounds and wall tests the fused kernels use
            const int xs0 = (int)((unsigned)(s * nx) / (unsigned)nstrips);
            const int xs1 = (int)((unsigned)((s + 1) * nx) / (unsigned)nstrips);
            const double fx = (wall_x && (xs0 <= 8 || xs1 >= nx - 8)) ? cx : 1.0;
            int y = 0;
            while (y < ny) {
                double f = fx * ((wall_y && y <= 8) ? cy : 1.0);
                int h = rows_for(T / f);
                if (wall_y && y + h >= ny - 8) h = rows_for(T / (fx * cy));   // ends next to the top wall
                if (h < 1) return -1;
                if (y + h > ny) h = ny - y;
                if (out && n < cap) out[n] = make_int4(s, y, y + h, g);
                ++n;
                y += h;
            }
        }
    }
    return n;
}

}  // namespace

namespace mdf {

int balanced_partition_multi(const PlanGrid* grids, int count, int tile_w, int slots, double cx, double cy, int4* out,
                             int cap)
{
    int maxny = 0;
    for (int g = 0; g < count; ++g) maxny = grids[g].ny > maxny ? grids[g].ny : maxny;
    const double fmax = cx * cy;
    double lo = 9.0, hi = fmax * (maxny + 12) + 1.0;   // hi: one segment per strip always fits
    if (segment_strips(grids, count, tile_w, cx, cy, hi, nullptr, 0) > slots) {
        lo = hi;   // more strips than slots: one segment each
    } else {
        while (hi - lo > 0.25) {
            const double mid = 0.5 * (lo + hi);
            const int n = segment_strips(grids, count, tile_w, cx, cy, mid, nullptr, 0);
            if (n > 0 && n <= slots)
                hi = mid;
            else
                lo = mid;
        }
        lo = hi;
    }
    const int n = segment_strips(grids, count, tile_w, cx, cy, lo, out, cap);
    return (n > 0 && n <= cap) ? n : 0;
}

int balanced_partition(int nx, int ny, bool wall_x, bool wall_y, int tile_w, int slots, double cx, double cy,
                       int4* out, int cap)
{
    const PlanGrid g{nx, ny, wall_x, wall_y};
    return balanced_partition_multi(&g, 1, tile_w, slots, cx, cy, out, cap);
}

bool wall_tasks_apply(int nx, bool wall_x, int tile_w)
{
    return wall_x && tile_w > 64 && nx - 2 * kWallCols >= 16;
}

namespace {
// Plan at budget T with wall tasks: the columns [W, nx - W) (W = kWallCols) cut
// into strips of tile_w lanes, each segmented at cost 1 (cy next to a y wall),
// and the two W-column strips at the x walls cut into single-wave tasks at
// cost cx.  Writes the workgroup entries to out[0, nwg) -- interior segments
// (strip, ys0, ys1, 0), then (-1 - j, 0, 0, 0) for each group j of tile_w/64
// tasks -- and the tasks (xs0, xs1, ys0, ys1) to out[nwg + j tile_w/64 + w],
// empty ones (0, 0, 0, 0).  Returns nwg (entries nwg + groups*tile_w/64 in
// *total), or -1 if some segment cannot hold a row.
int plan_wall_tasks(int nx, int ny, bool wall_y, int tile_w, double cx, double cy, double T, int4* out, int cap,
                    int* total)
{
    constexpr int W = kWallCols;
    auto rows_for = [](double budget) { return ((int)std::floor(budget) & ~3) - 8; };
    const int span = nx - 2 * W, tpw = tile_w / 64;
    const int nstrips = (span + tile_w - 9) / (tile_w - 8);
    // segments of one column range at factor fx: calls emit(ys0, ys1)
    auto cut = [&](double fx, auto emit) -> bool {
        int y = 0;
        while (y < ny) {
            int h = rows_for(T / (fx * ((wall_y && y <= 8) ? cy : 1.0)));
            if (wall_y && y + h >= ny - 8) h = rows_for(T / (fx * cy));   // ends next to the top wall
            if (h < 1) return false;
            if (y + h > ny) h = ny - y;
            emit(y, y + h);
            y += h;
        }
        return true;
    };
    int nint = 0;
    for (int st = 0; st < nstrips; ++st)
        if (!cut(1.0, [&](int a, int b) {
                if (out && nint < cap) out[nint] = make_int4(st, a, b, 0);
                ++nint;
            }))
            return -1;
    // the tasks, in order: left wall strip, then right
    int ntask = 0;
    int4* tasks = nullptr;
    const int tcap = 2 * (ny + 1);
    if (out) tasks = new (std::nothrow) int4[tcap];
    if (out && !tasks) return -1;
    for (int side = 0; side < 2; ++side) {
        const int x0 = side == 0 ? 0 : nx - W, x1 = side == 0 ? W : nx;
        if (!cut(cx, [&](int a, int b) {
                if (tasks && ntask < tcap) tasks[ntask] = make_int4(x0, x1, a, b);
                ++ntask;
            })) {
            delete[] tasks;
            return -1;
        }
    }
    const int groups = (ntask + tpw - 1) / tpw, nwg = nint + groups;
    *total = nwg + groups * tpw;
    if (out && *total <= cap) {
        for (int j = 0; j < groups; ++j) {
            out[nint + j] = make_int4(-1 - j, 0, 0, 0);
            for (int w = 0; w < tpw; ++w) {
                const int i = j * tpw + w;
                out[nwg + i] = i < ntask ? tasks[i] : make_int4(0, 0, 0, 0);
            }
        }
    }
    delete[] tasks;
    return nwg;
}
}  // namespace

int balanced_partition_wall_tasks(int nx, int ny, bool wall_y, int tile_w, int slots, double cx, double cy, int4* out,
                                  int cap, int* total)
{
    double lo = 9.0, hi = cx * cy * (ny + 12) + 1.0;   // hi: one segment per strip and wall strip
    int tot = 0;
    if (plan_wall_tasks(nx, ny, wall_y, tile_w, cx, cy, hi, nullptr, 0, &tot) > slots) {
        lo = hi;
    } else {
        while (hi - lo > 0.25) {
            const double mid = 0.5 * (lo + hi);
            const int n = plan_wall_tasks(nx, ny, wall_y, tile_w, cx, cy, mid, nullptr, 0, &tot);
            if (n > 0 && n <= slots)
                hi = mid;
            else
                lo = mid;
        }
        lo = hi;
    }
    const int n = plan_wall_tasks(nx, ny, wall_y, tile_w, cx, cy, lo, out, cap, &tot);
    if (n <= 0 || tot > cap) return 0;
    *total = tot;
    return n;
}

}  // namespace mdf

namespace {

mdf::FusedShape default_shape()
{
    // One wave per strip of 64 columns (56 outputs), rows from the balanced table.
    mdf::FusedShape sh{64, -1, 2, nullptr, 0};
    return sh;
}

// Relative cost per row of a segment next to an x wall (cx) and next to a y
// wall (cy), measured on MI355X for each fused kernel against its wall-free
// march (lid-driven cavity 1024^2): the wall rule, the ghost nodes and the
// divergent lanes of the x-wall strips make those rows dearer.
constexpr double kWallTaskCost = 2.48;   // row cost of a single-wave task at an x wall

void segment_costs(int variant, double& cx, double& cy)
{
    if (variant == 1) {
        cx = 1.53;
        cy = 1.19;
    } else {
        cx = 1.19;
        cy = 1.08;
    }
}

// Build and upload the balanced segment table when the shape asks for it.
mdf_status prepare_shape(mdf_ctx* c)
{
    mdf::FusedShape& sh = c->shape;
    if (c->variant == 0 || sh.seg_h > 0) {
        sh.table = nullptr;
        sh.nwg = 0;
        sh.wall_tasks = 0;
        return MDF_OK;
    }
    // the per-component kernel always runs 64-lane strips; a 128-lane strip
    // takes two waves, so a round holds half as many of its workgroups
    const int tw = c->variant == 2 ? 64 : sh.tile_w;
    const bool tasks = c->variant == 1 && mdf::wall_tasks_apply(c->p.nx, c->p.bc_x == MDF_BC_WALL, tw);
    double cx, cy;
    segment_costs(c->variant, cx, cy);
    // a single-wave task at an x wall: one wave (64 lanes, 8 of them halo) per
    // row instead of four, so it takes longer per row than a wall strip of
    // four waves (2.48x an interior row; measured over scales of the factor)
    if (tasks) cx = kWallTaskCost;
    cx = 1.0 + (cx - 1.0) * c->cx_scale;
    cy = 1.0 + (cy - 1.0) * c->cy_scale;
    int4* host = new (std::nothrow) int4[kSegCap];
    if (!host) return fail(c, MDF_EDEVICE, "out of host memory");
    const int want = c->slots * c->rounds / (tw / 64);
    const int slots = want < kSegCap ? want : kSegCap;
    int total = 0;
    const int n = tasks ? mdf::balanced_partition_wall_tasks(c->p.nx, c->p.ny, c->p.bc_y == MDF_BC_WALL, tw, slots, cx,
                                                             cy, host, kSegCap, &total)
                        : mdf::balanced_partition(c->p.nx, c->p.ny, c->p.bc_x == MDF_BC_WALL,
                                                  c->p.bc_y == MDF_BC_WALL, tw, slots, cx, cy, host, kSegCap);
    if (!tasks) total = n;
    hipError_t e = hipSuccess;
    if (n > 0) {
        e = hipMemcpyAsync(c->seg, host, sizeof(int4) * total, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    delete[] host;
    if (n <= 0) return fail(c, MDF_EINVAL, "grid too wide for the segment table");
    if (e != hipSuccess) return hip_check(c, e, "segment table upload");
    sh.table = c->seg;
    sh.nwg = n;
    sh.wall_tasks = tasks ? 1 : 0;
    return MDF_OK;
}

bool check_ctx(mdf_ctx* c) { return c != nullptr; }

}  // namespace

// ---------------------------------------------------------------------------
// Batches of independent periodic instances (one launch per step for all).

struct mdf_batch {
    int count = 0;
    hipStream_t stream = nullptr;   // the caller's stream
    hipStream_t gstream = nullptr;  // private stream the captured step graphs replay on
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    double* f[2] = {nullptr, nullptr};
    double* backup = nullptr;       // copy of the state while the autotuner runs
    double* diag_part = nullptr;    // diagnostics partials and result
    double* diag_out = nullptr;
    size_t state_doubles = 0;       // doubles of one state buffer (all instances)
    mdf::BatchInst* d_insts = nullptr;
    int4* d_table = nullptr;
    int table_cap = 0;
    std::vector<mdf::BatchInst> insts;
    bool powerlaw = false;
    int pl = mdf::PL_NEWTON;      // viscosity law every instance shares
    int variant = 2, tile_w = 64, prefetch = 2, rounds = 1, slots = 1024, nwg = 0;
    int cur = 0;
    int64_t steps = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // by starting buffer
    int64_t gn[2] = {0, 0};
    std::string err;
};

namespace {

struct BatchLayout {
    size_t off_insts, off_table, off_f0, off_f1, off_backup, off_dp, off_do, total;
    size_t state_doubles;
    int table_cap;
    std::vector<long long> offs;   // per instance, doubles
    std::vector<int> pitch;
};

const char* validate_batch(const mdf_params* ps, int count)
{
    if (!ps) return "params is NULL";
    if (count < 1 || count > 65536) return "count must lie in 1..65536";
    for (int i = 0; i < count; ++i) {
        if (const char* e = validate(&ps[i])) return e;
        if (ps[i].bc_x != MDF_BC_PERIODIC || ps[i].bc_y != MDF_BC_PERIODIC)
            return "batched instances must be periodic on both axes";
        if (ps[i].inv_dx_x || ps[i].inv_dx_y) return "batched instances must use uniform grids";
        if (has_force_field(&ps[i])) return "batched instances take a uniform force only";
        if (ps[i].force_harmonic) return "batched instances take a steady force only";
        if (ps[i].metric) return "batched instances take no general mapping";
        if (ps[i].mass_source) return "batched instances take no mass source";
        if (ps[i].pl_n != ps[0].pl_n) return "batched instances must share the fluid model (pl_n)";
    }
    return nullptr;
}

BatchLayout batch_layout(const mdf_params* ps, int count)
{
    BatchLayout B;
    long long nstrips = 0;
    size_t o = 0;
    B.offs.resize(count);
    B.pitch.resize(count);
    for (int i = 0; i < count; ++i) {
        B.pitch[i] = (ps[i].nx + 15) & ~15;
        B.offs[i] = (long long)(o / sizeof(double));
        o += align256(10 * (size_t)B.pitch[i] * (size_t)ps[i].ny * sizeof(double));
        nstrips += (ps[i].nx + 55) / 56;
    }
    B.state_doubles = o / sizeof(double);
    const long long cap = nstrips + 64 > 16384 ? nstrips + 64 : 16384;
    B.table_cap = (int)cap;
    size_t t = 0;
    B.off_insts = t;  t += align256((size_t)count * sizeof(mdf::BatchInst));
    B.off_table = t;  t += align256((size_t)B.table_cap * sizeof(int4));
    B.off_f0 = t;     t += o;
    B.off_f1 = t;     t += o;
    B.off_backup = t; t += o;
    B.off_dp = t;     t += align256(8 * (size_t)mdf::kDiagMaxBlocks * sizeof(double));   // diagnostics partials
    B.off_do = t;     t += align256(8 * sizeof(double));
    B.total = t;
    return B;
}

mdf_status bfail(mdf_batch* b, mdf_status s, const char* msg)
{
    if (b) b->err = msg;
    return fail(nullptr, s, "%s", msg);
}

mdf_status bhip(mdf_batch* b, hipError_t e, const char* what)
{
    if (e == hipSuccess) return MDF_OK;
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return bfail(b, MDF_EDEVICE, buf);
}

void batch_drop_graphs(mdf_batch* b)
{
    for (int i = 0; i < 2; ++i) {
        if (b->gexec[i]) (void)hipGraphExecDestroy(b->gexec[i]);
        b->gexec[i] = nullptr;
        b->gn[i] = 0;
    }
}

// Balanced partition of all instances' strips over `rounds` rounds of waves
// (a strip of tile_w lanes takes tile_w / 64 of them).
mdf_status batch_plan(mdf_batch* b)
{
    std::vector<mdf::PlanGrid> g(b->count);
    for (int i = 0; i < b->count; ++i) g[i] = mdf::PlanGrid{b->insts[i].K.nx, b->insts[i].K.ny, false, false};
    std::vector<int4> host(b->table_cap);
    const int tw = b->variant == 2 ? 64 : b->tile_w;
    const int n = mdf::balanced_partition_multi(g.data(), b->count, tw, b->slots * b->rounds / (tw / 64), 1.0, 1.0,
                                                host.data(), b->table_cap);
    if (n <= 0) return bfail(b, MDF_EINVAL, "batch too large for its segment table");
    hipError_t e = hipMemcpyAsync(b->d_table, host.data(), sizeof(int4) * n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "batch segment table upload");
    b->nwg = n;
    batch_drop_graphs(b);
    return MDF_OK;
}

hipError_t batch_launch(mdf_batch* b, const double* fin, double* fout, hipStream_t s)
{
    if (b->variant == 1)
        return mdf::launch_fused_batch(b->d_insts, b->d_table, b->nwg, b->pl, b->tile_w, b->prefetch, fin, fout,
                                       s);
    return mdf::launch_fused2_batch(b->d_insts, b->d_table, b->nwg, b->powerlaw, b->prefetch, fin, fout, s);
}

}  // namespace

extern "C" {


size_t mdf_workspace_size(const mdf_params* p)
{
    if (validate(p)) return 0;
    return layout_of(p).total;
}

mdf_status mdf_init(const mdf_params* p, const double* u0, const double* v0, const double* p0, void* workspace,
                    size_t ws_bytes, void* hip_stream, mdf_ctx** out)
{
    if (!out) return fail(nullptr, MDF_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char* why = validate(p)) return fail(nullptr, MDF_EINVAL, "%s", why);
    if (!u0 || !v0 || !p0) return fail(nullptr, MDF_EINVAL, "initial fields must be non-NULL device pointers");
    const Layout L = layout_of(p);
    if (!workspace || ws_bytes < L.total)
        return fail(nullptr, MDF_EINVAL, "workspace too small: need %zu bytes, got %zu", L.total, ws_bytes);
    if (((uintptr_t)workspace & 255u) != 0) return fail(nullptr, MDF_EINVAL, "workspace must be 256-byte aligned");

    mdf_ctx* c = new (std::nothrow) mdf_ctx();
    if (!c) return fail(nullptr, MDF_EDEVICE, "out of host memory");
    c->p = *p;
    c->p.inv_dx_x = nullptr;
    c->p.inv_dx_y = nullptr;
    c->p.force_x = nullptr;
    c->p.force_y = nullptr;
    c->p.metric = nullptr;
    c->p.mass_source = nullptr;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)workspace;
    c->ws_bytes = ws_bytes;
    c->f[0] = (double*)(c->ws + L.off_f0);
    c->f[1] = (double*)(c->ws + L.off_f1);
    c->fbp = (double*)(c->ws + L.off_fbp);
    c->fmid = (double*)(c->ws + L.off_fmid);
    c->gx = (double*)(c->ws + L.off_gx);
    c->gy = (double*)(c->ws + L.off_gy);
    c->diag_part = (double*)(c->ws + L.off_dp);
    c->diag_out = (double*)(c->ws + L.off_do);
    c->seg = (int4*)(c->ws + L.off_seg);
    c->K = make_consts(*p, L);
    c->K.gx = c->gx;
    c->K.gy = c->gy;
    // both fused kernels hold four workgroups per compute unit
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    c->slots = 4 * (cus > 0 ? cus : 256);
    c->shape = default_shape();
    // one wave per velocity component fits two waves per SIMD for a Newtonian
    // fluid; the power-law viscosity solve needs more registers than that
    // allows, and there one wave per strip is faster.  A force field has
    // kernels of the second kind only.
    c->variant = (p->pl_n == 1.0 && !has_force_field(p)) ? 2 : 1;
    // a general mapping and a mass source run on the tiled step
    if (p->metric || p->mass_source) c->variant = 0;

    // derivative scales 1/(X' dxi) per node (uniform: 1/dx)
    std::string hbuf;
    {
        const double hx = p->bc_x == MDF_BC_WALL ? p->lx / (p->nx - 1) : p->lx / p->nx;
        const double hy = p->bc_y == MDF_BC_WALL ? p->ly / (p->ny - 1) : p->ly / p->ny;
        double* gxh = new (std::nothrow) double[(size_t)p->nx + p->ny];
        if (!gxh) {
            delete c;
            return fail(nullptr, MDF_EDEVICE, "out of host memory");
        }
        for (int i = 0; i < p->nx; ++i) gxh[i] = p->inv_dx_x ? p->inv_dx_x[i] : 1.0 / hx;
        for (int i = 0; i < p->ny; ++i) gxh[p->nx + i] = p->inv_dx_y ? p->inv_dx_y[i] : 1.0 / hy;
        for (int i = 0; i < p->nx + p->ny; ++i)
            if (!(gxh[i] > 0.0) || !std::isfinite(gxh[i])) {
                delete[] gxh;
                delete c;
                return fail(nullptr, MDF_EINVAL, "metric arrays must be finite and > 0");
            }
        hipError_t e = hipMemcpyAsync(c->gx, gxh, sizeof(double) * p->nx, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->gy, gxh + p->nx, sizeof(double) * p->ny, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        delete[] gxh;
        if (e != hipSuccess) {
            mdf_status s = hip_check(nullptr, e, "metric upload");
            delete c;
            return s;
        }
    }
    // force field: the uniform force plus the given field, (F_x, F_y) per node
    if (has_force_field(p)) {
        const size_t pitch = L.pitch, n2 = 2 * pitch * (size_t)p->ny;
        std::vector<double> ffh;
        try {
            ffh.assign(n2, 0.0);
        } catch (...) {
            delete c;
            return fail(nullptr, MDF_EDEVICE, "out of host memory");
        }
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const size_t i = (size_t)y * p->nx + x, o = ((size_t)y * pitch + x) * 2;
                ffh[o] = p->fx + (p->force_x ? p->force_x[i] : 0.0);
                ffh[o + 1] = p->fy + (p->force_y ? p->force_y[i] : 0.0);
                if (!std::isfinite(ffh[o]) || !std::isfinite(ffh[o + 1])) {
                    delete c;
                    return fail(nullptr, MDF_EINVAL, "force field values must be finite");
                }
            }
        double* dff = (double*)(c->ws + L.off_ff);
        hipError_t e = hipMemcpyAsync(dff, ffh.data(), sizeof(double) * n2, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            mdf_status s = hip_check(nullptr, e, "force field upload");
            delete c;
            return s;
        }
        c->K.ff = dff;
    }
    // general mapping: the inverse Jacobian's four planes, finite and invertible at every node
    if (p->metric) {
        const size_t n = (size_t)p->nx * p->ny;
        for (size_t i = 0; i < n; ++i) {
            const double a = p->metric[i], b = p->metric[n + i], cc = p->metric[2 * n + i], d = p->metric[3 * n + i];
            const double det = a * d - b * cc;
            if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(cc) || !std::isfinite(d) || !(det != 0.0) ||
                !std::isfinite(det)) {
                delete c;
                return fail(nullptr, MDF_EINVAL, "metric values must be finite with a non-zero Jacobian");
            }
        }
        double* dmet = (double*)(c->ws + L.off_met);
        hipError_t e = hipMemcpyAsync(dmet, p->metric, sizeof(double) * 4 * n, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            mdf_status s = hip_check(nullptr, e, "metric upload");
            delete c;
            return s;
        }
        c->K.met = dmet;
    }
    // mass source: one finite value per node
    if (p->mass_source) {
        const size_t n = (size_t)p->nx * p->ny;
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(p->mass_source[i])) {
                delete c;
                return fail(nullptr, MDF_EINVAL, "mass source values must be finite");
            }
        double* drs = (double*)(c->ws + L.off_rs);
        hipError_t e = hipMemcpyAsync(drs, p->mass_source, sizeof(double) * n, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            mdf_status s = hip_check(nullptr, e, "mass source upload");
            delete c;
            return s;
        }
        c->K.rsrc = drs;
    }
    {
        const mdf_status s = prepare_shape(c);
        if (s != MDF_OK) {
            delete c;
            return s;
        }
    }
    hipError_t e = mdf::launch_init(c->K, u0, v0, p0, c->f[0], c->stream);
    if (e == hipSuccess) e = mdf::launch_wall_fix(c->K, c->f[0], c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        mdf_status s = hip_check(nullptr, e, "initialisation");
        delete c;
        return s;
    }
    *out = c;
    return MDF_OK;
}

mdf_status mdf_set_fields(mdf_ctx* c, const double* u0, const double* v0, const double* p0)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (!u0 || !v0 || !p0) return fail(c, MDF_EINVAL, "u0, v0 and p0 must be non-NULL");
    hipError_t e = mdf::launch_init(c->K, u0, v0, p0, c->f[c->cur], c->stream);
    if (e == hipSuccess) e = mdf::launch_wall_fix(c->K, c->f[c->cur], c->stream);
    return hip_check(c, e, "set fields");
}

mdf_status mdf_step(mdf_ctx* c, int64_t n)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (n < 0) return fail(c, MDF_EINVAL, "n must be >= 0");
    if (n == 0) return MDF_OK;
    for (int64_t i = 0; i < n; ++i) {
        const double* fin = c->f[c->cur];
        double* fout = c->f[1 - c->cur];
        if (c->p.force_harmonic) set_force_time(c->K, c->p, c->steps);
        hipError_t e;
        if (c->variant == 0)
            e = mdf::launch_tiled_step(c->K, fin, c->fmid, fout, c->stream);
        else if (c->variant == 1)
            e = mdf::launch_fused(c->K, c->shape, fin, fout, c->stream);
        else
            e = mdf::launch_fused2(c->K, c->shape, fin, fout, c->stream);
        if (e != hipSuccess) return hip_check(c, e, "step launch");
        c->cur = 1 - c->cur;
        c->steps += 1;
    }
    if (c->variant != 0) {
        hipError_t e = mdf::launch_wall_fix(c->K, c->f[c->cur], c->stream);
        if (e != hipSuccess) return hip_check(c, e, "wall rule launch");
    }
    return MDF_OK;
}

mdf_status mdf_moments(mdf_ctx* c, double* u, double* v, double* p)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (!u && !v && !p) return MDF_OK;
    return hip_check(c, mdf::launch_moments(c->K, c->f[c->cur], u, v, p, c->stream), "moments launch");
}

mdf_status mdf_derived(mdf_ctx* c, double* out, uint32_t mask)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (!out) return fail(c, MDF_EINVAL, "out is NULL");
    if (mask == 0 || mask >= (1u << 14)) return fail(c, MDF_EINVAL, "mask must be in [1, 2^14)");
    return hip_check(c, mdf::launch_derived(c->K, c->f[c->cur], out, mask, c->stream), "derived launch");
}

mdf_status mdf_diagnostics(mdf_ctx* c, double out[8])
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (!out) return fail(c, MDF_EINVAL, "out is NULL");
    hipError_t e = mdf::launch_diagnostics(c->K, c->f[c->cur], c->diag_part, c->diag_out, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, c->diag_out, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "diagnostics");
    if (out[6] != 0.0) return fail(c, MDF_EUNSTABLE, "state holds %.0f non-finite values", out[6]);
    return MDF_OK;
}

mdf_status mdf_save(mdf_ctx* c, double* f)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (!f) return fail(c, MDF_EINVAL, "f is NULL");
    return hip_check(c, mdf::launch_pack(c->K, c->f[c->cur], f, c->stream), "save launch");
}

mdf_status mdf_load(mdf_ctx* c, const double* f)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (!f) return fail(c, MDF_EINVAL, "f is NULL");
    return hip_check(c, mdf::launch_unpack(c->K, f, c->f[c->cur], c->stream), "load launch");
}

mdf_status mdf_set_kernel(mdf_ctx* c, int32_t variant, int32_t tile_w, int32_t seg_h, int32_t prefetch)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (variant < 0 || variant > 2) return fail(c, MDF_EINVAL, "variant must be 0, 1 or 2");
    if (variant == 2 && c->K.ff) return fail(c, MDF_EINVAL, "a force field runs on variant 0 or 1 only");
    if (variant != 0 && c->K.met) return fail(c, MDF_EINVAL, "a general mapping runs on variant 0 only");
    if (variant != 0 && c->K.rsrc) return fail(c, MDF_EINVAL, "a mass source runs on variant 0 only");
    if (seg_h < -4) return fail(c, MDF_EINVAL, "seg_h below 0 selects 1 to 4 rounds of the balanced table");
    mdf::FusedShape sh = c->shape;
    int rounds = c->rounds;
    if (tile_w) sh.tile_w = tile_w;
    if (seg_h > 0) sh.seg_h = seg_h;
    if (seg_h < 0) {
        sh.seg_h = -1;
        rounds = -seg_h;
    }
    if (prefetch) sh.prefetch = prefetch;
    if (variant != 0 && !mdf::fused_shape_ok(c->K, sh))
        return fail(c, MDF_EINVAL,
                    c->K.ff ? "a force field takes tile_w 64 and prefetch 2"
                            : "tile_w must be 64, 128 or 256 and prefetch 2 or 3");
    const int old_variant = c->variant, old_rounds = c->rounds;
    const mdf::FusedShape old_shape = c->shape;
    c->variant = variant;
    c->shape = sh;
    c->rounds = rounds;
    const mdf_status s = prepare_shape(c);
    if (s != MDF_OK) {
        c->variant = old_variant;
        c->shape = old_shape;
        c->rounds = old_rounds;
    }
    return s;
}

int32_t mdf_plan_segments(const mdf_params* p, int32_t variant, int32_t tile_w, int32_t slots, int32_t* out,
                          int32_t cap)
{
    if (validate(p)) return 0;
    if (variant != 1 && variant != 2) return 0;
    if (variant == 2) tile_w = 64;
    if (tile_w != 64 && tile_w != 128 && tile_w != 256) return 0;
    if (slots < 1 || cap < 1 || !out) return 0;
    double cx, cy;
    segment_costs(variant, cx, cy);
    int4* host = new (std::nothrow) int4[cap];
    if (!host) return 0;
    const int n = mdf::balanced_partition(p->nx, p->ny, p->bc_x == MDF_BC_WALL, p->bc_y == MDF_BC_WALL, tile_w, slots,
                                          cx, cy, host, cap);
    for (int i = 0; i < n; ++i) {
        out[3 * i + 0] = host[i].x;
        out[3 * i + 1] = host[i].y;
        out[3 * i + 2] = host[i].z;
    }
    delete[] host;
    return n;
}

mdf_status mdf_set_partition_costs(mdf_ctx* c, double x_wall_scale, double y_wall_scale)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (!(x_wall_scale >= 0.0 && x_wall_scale <= 10.0 && y_wall_scale >= 0.0 && y_wall_scale <= 10.0))
        return fail(c, MDF_EINVAL, "cost scales must lie in [0, 10]");
    const double ox = c->cx_scale, oy = c->cy_scale;
    c->cx_scale = x_wall_scale;
    c->cy_scale = y_wall_scale;
    const mdf_status s = prepare_shape(c);
    if (s != MDF_OK) {
        c->cx_scale = ox;
        c->cy_scale = oy;
        (void)prepare_shape(c);
    }
    return s;
}

mdf_status mdf_autotune(mdf_ctx* c, int32_t steps, double* choice)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (steps < 1) return fail(c, MDF_EINVAL, "steps must be >= 1");
    if (c->K.met || c->K.rsrc) {   // one step kernel (the tiled step): nothing to choose
        if (choice) {
            const double ch[6] = {0.0, (double)c->shape.prefetch, c->cx_scale, c->cy_scale, 0.0, (double)c->shape.tile_w};
            for (int k = 0; k < 6; ++k) choice[k] = ch[k];
        }
        return MDF_OK;
    }
    // state backup in the spare state-sized buffer of the workspace
    const size_t bytes = 10 * (size_t)c->K.pitch * (size_t)c->K.ny * sizeof(double);
    const int cur0 = c->cur;
    const int64_t steps0 = c->steps;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e == hipSuccess) e = hipMemcpyAsync(c->fbp, c->f[cur0], bytes, hipMemcpyDeviceToDevice, c->stream);
    const bool power = c->p.pl_n != 1.0;

    // candidates: kernel (variant, tile_w, deepest prefetch) in (1, 64, 3),
    // (1, 128, 3), (1, 256, 2), (2, 64, 3) -- the per-component kernel exceeds
    // 256 registers for a power law -- times prefetch 2.. times eight scalings
    // of the wall-row cost factors
    struct Cand {
        int var, tw, pf;
        double sx, sy;
        float ms;
    };
    // (below 1 for wide strips, where a wall strip's extra work is spread
    // over more columns)
    const double scales[8][2] = {{0.3, 0.6}, {0.6, 0.8}, {1.0, 1.0}, {1.35, 1.0},
                                 {1.7, 1.3}, {2.2, 1.6}, {2.8, 2.0}, {3.5, 2.4}};
    std::vector<Cand> cands;
    const int kernels[4][3] = {{1, 64, 3}, {1, 128, 3}, {1, 256, 3}, {2, 64, 3}};
    const bool field = c->K.ff != nullptr;
    for (int kv = 0; kv < 4; ++kv) {
        const int var = kernels[kv][0], tw = kernels[kv][1];
        if (var == 2 && (power || field)) continue;
        if (field && tw != 64) continue;
        const bool pf2_only = field;   // the force-field kernels exist for prefetch 2 only
        for (int pf = 2; pf <= (pf2_only ? 2 : kernels[kv][2]); ++pf)
            for (int sc = 0; sc < 8; ++sc) cands.push_back(Cand{var, tw, pf, scales[sc][0], scales[sc][1], 1e30f});
    }
    auto apply = [&](const Cand& k) {
        c->variant = k.var;
        c->shape = mdf::FusedShape{k.tw, -1, k.pf, nullptr, 0};
        c->rounds = 1;
        c->cx_scale = k.sx;
        c->cy_scale = k.sy;
        return prepare_shape(c);
    };
    mdf_status launch = MDF_OK;
    // time one candidate over n steps from the saved state, then restore it
    auto time_cand = [&](Cand& k, int n) {
        if (e != hipSuccess || launch != MDF_OK || apply(k) != MDF_OK) return;
        launch = mdf_step(c, 1);   // first launch of this kernel outside the timing
        if (launch == MDF_OK) e = hipEventRecord(t0, c->stream);
        if (launch == MDF_OK && e == hipSuccess) launch = mdf_step(c, n);
        if (launch == MDF_OK && e == hipSuccess) e = hipEventRecord(t1, c->stream);
        if (launch == MDF_OK && e == hipSuccess) e = hipEventSynchronize(t1);
        float ms = 0.0f;
        if (launch == MDF_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (launch == MDF_OK && e == hipSuccess) k.ms = ms / n;
        c->cur = cur0;
        const hipError_t er = hipMemcpyAsync(c->f[cur0], c->fbp, bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = er;
    };
    // pass 1: every candidate over `steps`; pass 2: the three fastest again
    // over 4 x `steps`, which settles choices within the noise of short runs
    for (Cand& k : cands) time_cand(k, steps);
    std::vector<Cand> top(cands);
    std::stable_sort(top.begin(), top.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
    if (top.size() > 3) top.resize(3);
    for (Cand& k : top) time_cand(k, 4 * steps);
    Cand best{c->variant, c->shape.tile_w, c->shape.prefetch, c->cx_scale, c->cy_scale, 1e30f};
    for (const Cand& k : top)
        if (k.ms < best.ms) best = k;

    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    c->cur = cur0;
    c->steps = steps0;
    const mdf_status s = apply(best);
    if (e != hipSuccess) return hip_check(c, e, "autotune");
    if (launch != MDF_OK) return launch;
    if (s == MDF_OK && choice) {
        choice[0] = best.var;
        choice[1] = best.pf;
        choice[2] = best.sx;
        choice[3] = best.sy;
        choice[4] = best.ms;
        choice[5] = best.tw;
    }
    return s;
}

double mdf_dt(const mdf_ctx* c) { return c ? c->K.dt : 0.0; }

int64_t mdf_steps(const mdf_ctx* c) { return c ? c->steps : 0; }

const char* mdf_last_error(const mdf_ctx* c)
{
    if (c) return c->err.c_str();
    return g_err.c_str();
}

void mdf_destroy(mdf_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

// ---- learned closure ---------------------------------------------------------

int32_t mdf_cnn_param_count(void) { return mdf::cnn_param_count(); }

size_t mdf_cnn_workspace_size(int32_t batch, int32_t h, int32_t w)
{
    if (batch < 1 || h < 3 || w < 32 || (w % 32) != 0 || (int64_t)batch * h * w > (int64_t)1 << 26) return 0;
    return mdf::cnn_workspace_size(batch, h, w);
}

static const char* cnn_check(const void* ws, size_t ws_bytes, int32_t batch, int32_t h, int32_t w)
{
    const size_t need = mdf_cnn_workspace_size(batch, h, w);
    if (need == 0) return "batch >= 1, h >= 3, w a multiple of 32 and batch*h*w <= 2^26 required";
    if (!ws) return "workspace is NULL";
    if (((uintptr_t)ws & 255) != 0) return "workspace must be 256-byte aligned";
    if (ws_bytes < need) return "workspace too small";
    return nullptr;
}

mdf_status mdf_cnn_forward(void* ws, size_t ws_bytes, const float* params, int32_t batch, int32_t h, int32_t w,
                           const double* uv, double in_scale, double out_scale, double* duv, void* hip_stream)
{
    if (const char* e = cnn_check(ws, ws_bytes, batch, h, w)) return fail(nullptr, MDF_EINVAL, "%s", e);
    if (!params || !uv || !duv) return fail(nullptr, MDF_EINVAL, "params, uv and duv must be non-NULL");
    return hip_check(nullptr, mdf::cnn_forward((char*)ws, params, batch, h, w, uv, in_scale, out_scale, duv,
                                               (hipStream_t)hip_stream), "closure forward");
}

mdf_status mdf_cnn_forward_noalloc(const float* params, int32_t batch, int32_t h, int32_t w, const double* uv,
                                   double in_scale, double out_scale, double* duv, void* hip_stream)
{
    if (mdf_cnn_workspace_size(batch, h, w) == 0)
        return fail(nullptr, MDF_EINVAL, "batch >= 1, h >= 3 and w a multiple of 32 required");
    if ((int64_t)batch * h * w > MDF_CNN_NOALLOC_MAX_PIXELS ||
        mdf::cnn_noalloc_bytes(batch, h, w) > mdf::cnn_noalloc_capacity())
        return fail(nullptr, MDF_EINVAL, "batch*h*w = %lld exceeds the fixed scratch of %d pixels",
                    (long long)batch * h * w, MDF_CNN_NOALLOC_MAX_PIXELS);
    if (!params || !uv || !duv) return fail(nullptr, MDF_EINVAL, "params, uv and duv must be non-NULL");
    return hip_check(nullptr, mdf::cnn_forward_noalloc(params, batch, h, w, uv, in_scale, out_scale, duv,
                                                       (hipStream_t)hip_stream), "closure forward (no allocation)");
}

mdf_status mdf_cnn_backward(void* ws, size_t ws_bytes, const float* params, int32_t batch, int32_t h, int32_t w,
                            const double* duv_target, double out_scale, float* grad, double* loss, void* hip_stream)
{
    if (const char* e = cnn_check(ws, ws_bytes, batch, h, w)) return fail(nullptr, MDF_EINVAL, "%s", e);
    if (!params || !duv_target || !grad) return fail(nullptr, MDF_EINVAL, "params, target and grad must be non-NULL");
    return hip_check(nullptr, mdf::cnn_backward((char*)ws, params, batch, h, w, duv_target, out_scale, grad, loss,
                                                (hipStream_t)hip_stream), "closure backward");
}

mdf_status mdf_cnn_layer_io(const void* ws, size_t ws_bytes, int32_t batch, int32_t h, int32_t w, int32_t layer,
                            uint16_t* in_bf16, float* z, uint16_t* g_bf16, float* g, void* hip_stream)
{
    if (const char* e = cnn_check(ws, ws_bytes, batch, h, w)) return fail(nullptr, MDF_EINVAL, "%s", e);
    if (layer < 1 || layer > 4) return fail(nullptr, MDF_EINVAL, "layer must lie in 1..4");
    return hip_check(nullptr, mdf::cnn_layer_io((const char*)ws, batch, h, w, layer, in_bf16, z, g_bf16, g,
                                                (hipStream_t)hip_stream), "closure layer copy");
}

mdf_status mdf_cnn_adam(float* params, const float* grad, float* m, float* v, int32_t n, float lr, float beta1,
                        float beta2, float eps, int32_t step, void* hip_stream)
{
    if (!params || !grad || !m || !v || n < 1 || step < 1) return fail(nullptr, MDF_EINVAL, "bad Adam arguments");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f))
        return fail(nullptr, MDF_EINVAL, "Adam needs 0 <= beta < 1 and eps > 0");
    return hip_check(nullptr, mdf::cnn_adam(params, grad, m, v, n, lr, beta1, beta2, eps, step,
                                            (hipStream_t)hip_stream), "Adam update");
}

mdf_status mdf_closure_apply(mdf_ctx* c, const double* du, const double* dv, double ke_ref, double div_factor,
                             double* ke_out, double* div_out, int32_t* fell_back)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (c->p.bc_x != MDF_BC_PERIODIC || c->p.bc_y != MDF_BC_PERIODIC || !c->K.uniform)
        return fail(c, MDF_EINVAL, "the closure applies to periodic uniform grids");
    if ((du == nullptr) != (dv == nullptr)) return fail(c, MDF_EINVAL, "du and dv must both be given or both NULL");
    const double hx = c->p.lx / c->p.nx, hy = c->p.ly / c->p.ny;
    double* f = c->f[c->cur];
    // r = {KE, max|div| of the current field, KE, max|div| of the corrected one}
    hipError_t e = mdf::launch_closure_guard(c->K, f, du, dv, hx, hy, c->diag_part, c->diag_out, c->stream);
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    if (e == hipSuccess) e = hipMemcpyAsync(r, c->diag_out, sizeof r, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "closure guard");
    const bool ok = du && std::isfinite(r[2]) && std::isfinite(r[3]) && r[2] <= ke_ref && r[3] <= div_factor * r[1];
    if (ke_out) *ke_out = ok ? r[2] : r[0];
    if (div_out) *div_out = ok ? r[3] : r[1];
    if (fell_back) *fell_back = (du && !ok) ? 1 : 0;
    if (!ok) return MDF_OK;
    return hip_check(c, mdf::launch_closure_apply(c->K, f, du, dv, nullptr, c->stream), "closure apply");
}

static mdf_status closure_async_check(mdf_ctx* c)
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (c->p.bc_x != MDF_BC_PERIODIC || c->p.bc_y != MDF_BC_PERIODIC || !c->K.uniform)
        return fail(c, MDF_EINVAL, "the closure applies to periodic uniform grids");
    return MDF_OK;
}

mdf_status mdf_closure_begin(mdf_ctx* c)
{
    if (const mdf_status s = closure_async_check(c)) return s;
    const double hx = c->p.lx / c->p.nx, hy = c->p.ly / c->p.ny;
    double* state = c->diag_out + 8;
    hipError_t e = mdf::launch_closure_guard(c->K, c->f[c->cur], nullptr, nullptr, hx, hy, c->diag_part, c->diag_out,
                                             c->stream);
    if (e == hipSuccess) e = mdf::launch_closure_decide(c->diag_out, state, 0.0, true, c->stream);
    return hip_check(c, e, "closure begin");
}

mdf_status mdf_closure_apply_async(mdf_ctx* c, const double* du, const double* dv, double div_factor)
{
    if (const mdf_status s = closure_async_check(c)) return s;
    if (!du || !dv) return fail(c, MDF_EINVAL, "du and dv must be non-NULL");
    if (!(div_factor >= 0.0)) return fail(c, MDF_EINVAL, "div_factor must be >= 0");
    const double hx = c->p.lx / c->p.nx, hy = c->p.ly / c->p.ny;
    double* f = c->f[c->cur];
    double* state = c->diag_out + 8;
    hipError_t e = mdf::launch_closure_guard(c->K, f, du, dv, hx, hy, c->diag_part, c->diag_out, c->stream);
    if (e == hipSuccess) e = mdf::launch_closure_decide(c->diag_out, state, div_factor, false, c->stream);
    if (e == hipSuccess) e = mdf::launch_closure_apply(c->K, f, du, dv, state + 2, c->stream);
    return hip_check(c, e, "closure apply (asynchronous)");
}

mdf_status mdf_closure_stats(mdf_ctx* c, double out[3])
{
    if (!check_ctx(c)) return fail(nullptr, MDF_EINVAL, "ctx is NULL");
    if (!out) return fail(c, MDF_EINVAL, "out is NULL");
    double st[4] = {0.0, 0.0, 0.0, 0.0};
    hipError_t e = hipMemcpyAsync(st, c->diag_out + 8, sizeof st, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "closure stats");
    out[0] = st[0];
    out[1] = st[1];
    out[2] = st[3];
    return MDF_OK;
}

// ---- batches ---------------------------------------------------------------

size_t mdf_batch_workspace_size(const mdf_params* ps, int32_t count)
{
    if (validate_batch(ps, count)) return 0;
    return batch_layout(ps, count).total;
}

mdf_status mdf_batch_init(const mdf_params* ps, int32_t count, const double* const* u0s, const double* const* v0s,
                          const double* const* p0s, void* workspace, size_t ws_bytes, void* hip_stream,
                          mdf_batch** out)
{
    if (!out) return fail(nullptr, MDF_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char* e = validate_batch(ps, count)) return fail(nullptr, MDF_EINVAL, "%s", e);
    if (!u0s || !v0s || !p0s) return fail(nullptr, MDF_EINVAL, "initial field arrays are NULL");
    for (int i = 0; i < count; ++i)
        if (!u0s[i] || !v0s[i] || !p0s[i]) return fail(nullptr, MDF_EINVAL, "initial fields of instance %d are NULL", i);
    const BatchLayout B = batch_layout(ps, count);
    if (!workspace) return fail(nullptr, MDF_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(nullptr, MDF_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < B.total) return fail(nullptr, MDF_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, B.total);

    mdf_batch* b = new (std::nothrow) mdf_batch;
    if (!b) return fail(nullptr, MDF_EDEVICE, "out of host memory");
    b->count = count;
    b->stream = (hipStream_t)hip_stream;
    b->ws = (char*)workspace;
    b->ws_bytes = ws_bytes;
    b->d_insts = (mdf::BatchInst*)(b->ws + B.off_insts);
    b->d_table = (int4*)(b->ws + B.off_table);
    b->table_cap = B.table_cap;
    b->f[0] = (double*)(b->ws + B.off_f0);
    b->f[1] = (double*)(b->ws + B.off_f1);
    b->backup = (double*)(b->ws + B.off_backup);
    b->diag_part = (double*)(b->ws + B.off_dp);
    b->diag_out = (double*)(b->ws + B.off_do);
    b->state_doubles = B.state_doubles;
    b->powerlaw = ps[0].pl_n != 1.0;
    b->pl = ps[0].pl_n == 1.0 ? mdf::PL_NEWTON : (ps[0].pl_n == 0.5 ? mdf::PL_HALF : mdf::PL_THREE_HALVES);
    b->variant = b->powerlaw ? 1 : 2;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    b->slots = 4 * (cus > 0 ? cus : 256);
    b->insts.resize(count);
    for (int i = 0; i < count; ++i) {
        Layout L{};
        L.pitch = (size_t)B.pitch[i];
        mdf::BatchInst& I = b->insts[i];
        I.K = make_consts(ps[i], L);
        I.K.gx = nullptr;
        I.K.gy = nullptr;
        I.off = B.offs[i];
        I.nstrips = (ps[i].nx + 55) / 56;
        I.pad = 0;
    }
    hipError_t e = hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_insts, b->insts.data(), sizeof(mdf::BatchInst) * count, hipMemcpyHostToDevice,
                           b->stream);
    for (int i = 0; i < count && e == hipSuccess; ++i)
        e = mdf::launch_init(b->insts[i].K, u0s[i], v0s[i], p0s[i], b->f[0] + b->insts[i].off, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        const mdf_status s = bhip(nullptr, e, "batch initialisation");
        mdf_batch_destroy(b);
        return s;
    }
    const mdf_status s = batch_plan(b);
    if (s != MDF_OK) {
        mdf_batch_destroy(b);
        return s;
    }
    *out = b;
    return MDF_OK;
}

mdf_status mdf_batch_step(mdf_batch* b, int64_t n)
{
    if (!b) return fail(nullptr, MDF_EINVAL, "batch is NULL");
    if (n < 0) return bfail(b, MDF_EINVAL, "n must be >= 0");
    for (int64_t i = 0; i < n; ++i) {
        const hipError_t e = batch_launch(b, b->f[b->cur], b->f[1 - b->cur], b->stream);
        if (e != hipSuccess) return bhip(b, e, "batch step launch");
        b->cur = 1 - b->cur;
        b->steps += 1;
    }
    return MDF_OK;
}

mdf_status mdf_batch_step_graph(mdf_batch* b, int64_t n)
{
    if (!b) return fail(nullptr, MDF_EINVAL, "batch is NULL");
    if (n < 1) return bfail(b, MDF_EINVAL, "n must be >= 1");
    const int par = b->cur;
    if (!b->gexec[par] || b->gn[par] != n) {
        if (b->gexec[par]) (void)hipGraphExecDestroy(b->gexec[par]);
        b->gexec[par] = nullptr;
        hipError_t e = hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return bhip(b, e, "graph capture begin");
        int c = par;
        hipError_t el = hipSuccess;
        for (int64_t i = 0; i < n && el == hipSuccess; ++i) {
            el = batch_launch(b, b->f[c], b->f[1 - c], b->gstream);
            c = 1 - c;
        }
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->gstream, &g);
        if (el != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bhip(b, el != hipSuccess ? el : e, "graph capture");
        }
        e = hipGraphInstantiate(&b->gexec[par], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->gexec[par] = nullptr;
            return bhip(b, e, "graph instantiate");
        }
        b->gn[par] = n;
    }
    // order the replay after the caller's stream and the caller's later work after it
    hipError_t e = hipEventRecord(b->ev_in, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->gstream, b->ev_in, 0);
    if (e == hipSuccess) e = hipGraphLaunch(b->gexec[par], b->gstream);
    if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->gstream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_out, 0);
    if (e != hipSuccess) return bhip(b, e, "graph replay");
    b->cur = (int)(par ^ (n & 1));
    b->steps += n;
    return MDF_OK;
}

mdf_status mdf_batch_set_kernel(mdf_batch* b, int32_t variant, int32_t tile_w, int32_t prefetch, int32_t rounds)
{
    if (!b) return fail(nullptr, MDF_EINVAL, "batch is NULL");
    if (variant != 1 && variant != 2) return bfail(b, MDF_EINVAL, "variant must be 1 or 2");
    if (tile_w == 0) tile_w = 64;
    if (tile_w != 64 && (variant == 2 || (tile_w != 128 && tile_w != 256)))
        return bfail(b, MDF_EINVAL, "tile_w must be 64, 128 or 256 (variant 1) or 64 (variant 2)");
    if (prefetch != 2 && prefetch != 3) return bfail(b, MDF_EINVAL, "prefetch must be 2 or 3");
    if (rounds < 1 || rounds > 8) return bfail(b, MDF_EINVAL, "rounds must lie in 1..8");
    const int ov = b->variant, ot = b->tile_w, op = b->prefetch, orr = b->rounds;
    b->variant = variant;
    b->tile_w = tile_w;
    b->prefetch = prefetch;
    b->rounds = rounds;
    const mdf_status s = batch_plan(b);
    if (s != MDF_OK) {
        b->variant = ov;
        b->tile_w = ot;
        b->prefetch = op;
        b->rounds = orr;
        (void)batch_plan(b);
    }
    return s;
}

mdf_status mdf_batch_autotune(mdf_batch* b, int32_t steps, int32_t* choice)
{
    if (!b) return fail(nullptr, MDF_EINVAL, "batch is NULL");
    if (steps < 1) return bfail(b, MDF_EINVAL, "steps must be >= 1");
    const size_t bytes = b->state_doubles * sizeof(double);
    const int cur0 = b->cur;
    const int64_t steps0 = b->steps;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e == hipSuccess) e = hipMemcpyAsync(b->backup, b->f[cur0], bytes, hipMemcpyDeviceToDevice, b->stream);
    // candidates (variant, tile_w, prefetch, rounds); the per-component kernel
    // spills for a power law
    struct Cand {
        int var, tw, pf, rounds;
        float ms;
    };
    std::vector<Cand> cands;
    const int kernels[8][3] = {{2, 64, 2}, {2, 64, 3}, {1, 64, 2}, {1, 64, 3}, {1, 128, 2}, {1, 128, 3}, {1, 256, 2},
                               {1, 256, 3}};
    for (int r = 1; r <= 3; ++r)
        for (const auto& k : kernels)
            if (!(k[0] == 2 && b->powerlaw)) cands.push_back(Cand{k[0], k[1], k[2], r, 1e30f});
    mdf_status launch = MDF_OK;
    auto time_cand = [&](Cand& k, int n) {
        if (e != hipSuccess || launch != MDF_OK) return;
        if (mdf_batch_set_kernel(b, k.var, k.tw, k.pf, k.rounds) != MDF_OK) return;
        launch = mdf_batch_step(b, 1);   // first launch of this kernel outside the timing
        if (launch == MDF_OK) e = hipEventRecord(t0, b->stream);
        if (launch == MDF_OK && e == hipSuccess) launch = mdf_batch_step(b, n);
        if (launch == MDF_OK && e == hipSuccess) e = hipEventRecord(t1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (launch == MDF_OK && e == hipSuccess) k.ms = ms / n;
        // back to the state the tuning started from
        b->cur = cur0;
        const hipError_t er = hipMemcpyAsync(b->f[cur0], b->backup, bytes, hipMemcpyDeviceToDevice, b->stream);
        if (e == hipSuccess) e = er;
    };
    // every candidate over `steps`, then the three fastest over 4 x `steps`
    for (Cand& k : cands) time_cand(k, steps);
    std::vector<Cand> top(cands);
    std::stable_sort(top.begin(), top.end(), [](const Cand& a, const Cand& c) { return a.ms < c.ms; });
    if (top.size() > 3) top.resize(3);
    for (Cand& k : top) time_cand(k, 4 * steps);
    Cand best{b->variant, b->tile_w, b->prefetch, b->rounds, 1e30f};
    for (const Cand& k : top)
        if (k.ms < best.ms) best = k;
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    b->cur = cur0;
    b->steps = steps0;
    const mdf_status s = mdf_batch_set_kernel(b, best.var, best.tw, best.pf, best.rounds);
    if (e != hipSuccess) return bhip(b, e, "autotune");
    if (launch != MDF_OK) return launch;
    if (s == MDF_OK && choice) {
        choice[0] = best.var;
        choice[1] = best.pf;
        choice[2] = best.rounds;
        choice[3] = best.tw;
    }
    return s;
}

mdf_status mdf_batch_moments(mdf_batch* b, int32_t i, double* u, double* v, double* p)
{
    if (!b) return fail(nullptr, MDF_EINVAL, "batch is NULL");
    if (i < 0 || i >= b->count) return bfail(b, MDF_EINVAL, "instance index out of range");
    if (!u && !v && !p) return MDF_OK;
    const mdf::BatchInst& I = b->insts[i];
    return bhip(b, mdf::launch_moments(I.K, b->f[b->cur] + I.off, u, v, p, b->stream), "batch moments launch");
}

mdf_status mdf_batch_save(mdf_batch* b, int32_t i, double* f)
{
    if (!b) return fail(nullptr, MDF_EINVAL, "batch is NULL");
    if (i < 0 || i >= b->count) return bfail(b, MDF_EINVAL, "instance index out of range");
    if (!f) return bfail(b, MDF_EINVAL, "f is NULL");
    const mdf::BatchInst& I = b->insts[i];
    return bhip(b, mdf::launch_pack(I.K, b->f[b->cur] + I.off, f, b->stream), "batch save launch");
}

mdf_status mdf_batch_derived(mdf_batch* b, int32_t i, double* out, uint32_t mask)
{
    if (!b) return fail(nullptr, MDF_EINVAL, "batch is NULL");
    if (i < 0 || i >= b->count) return bfail(b, MDF_EINVAL, "instance index out of range");
    if (!out) return bfail(b, MDF_EINVAL, "out is NULL");
    if (mask == 0 || mask >= (1u << 14)) return bfail(b, MDF_EINVAL, "mask must be in [1, 2^14)");
    const mdf::BatchInst& I = b->insts[i];
    return bhip(b, mdf::launch_derived(I.K, b->f[b->cur] + I.off, out, mask, b->stream), "batch derived launch");
}

mdf_status mdf_batch_diagnostics(mdf_batch* b, int32_t i, double out[8])
{
    if (!b) return fail(nullptr, MDF_EINVAL, "batch is NULL");
    if (i < 0 || i >= b->count) return bfail(b, MDF_EINVAL, "instance index out of range");
    if (!out) return bfail(b, MDF_EINVAL, "out is NULL");
    const mdf::BatchInst& I = b->insts[i];
    hipError_t e = mdf::launch_diagnostics(I.K, b->f[b->cur] + I.off, b->diag_part, b->diag_out, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, b->diag_out, 8 * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "batch diagnostics");
    if (out[6] != 0.0) return bfail(b, MDF_EUNSTABLE, "instance state holds non-finite values");
    return MDF_OK;
}

double mdf_batch_dt(const mdf_batch* b, int32_t i)
{
    if (!b || i < 0 || i >= b->count) return 0.0;
    return b->insts[i].K.dt;
}

int64_t mdf_batch_steps(const mdf_batch* b) { return b ? b->steps : 0; }

int32_t mdf_batch_workgroups(const mdf_batch* b) { return b ? b->nwg : 0; }

const char* mdf_batch_last_error(const mdf_batch* b)
{
    if (b) return b->err.c_str();
    return g_err.c_str();
}

void mdf_batch_destroy(mdf_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->gstream) (void)hipStreamSynchronize(b->gstream);
    batch_drop_graphs(b);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->gstream) (void)hipStreamDestroy(b->gstream);
    delete b;
}

mdf_status mdf_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream)
{
    if (!src || !dst) return fail(nullptr, MDF_EINVAL, "src and dst must be non-NULL");
    if ((bytes & 15) != 0 || ((uintptr_t)src & 15) != 0 || ((uintptr_t)dst & 15) != 0)
        return fail(nullptr, MDF_EINVAL, "bytes and both pointers must be multiples of 16");
    const uintptr_t a = (uintptr_t)src, d = (uintptr_t)dst;
    if (bytes > 0 && a < d + bytes && d < a + bytes) return fail(nullptr, MDF_EINVAL, "regions overlap");
    if (bytes == 0) return MDF_OK;
    return hip_check(nullptr, mdf::launch_stream_copy(src, dst, bytes, (hipStream_t)hip_stream), "stream copy");
}

}  // extern "C"
