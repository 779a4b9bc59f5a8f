// Internal interface between the C ABI and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mdf_device.hpp"

namespace mdf {

hipError_t launch_init(const StepConsts& K, const double* u0, const double* v0, const double* p0, double* f,
                       hipStream_t s);
hipError_t launch_wall_fix(const StepConsts& K, double* f, hipStream_t s);
hipError_t launch_moments(const StepConsts& K, const double* f, double* u, double* v, double* p, hipStream_t s);
hipError_t launch_derived(const StepConsts& K, const double* f, double* out, uint32_t mask, hipStream_t s);
// diagnostics partials: 8 doubles per block of the reduction, at most this many blocks
constexpr int kDiagMaxBlocks = 4096;
int diag_blocks(const StepConsts& K);
hipError_t launch_diagnostics(const StepConsts& K, const double* f, double* partials, double* out8, hipStream_t s);
hipError_t launch_pack(const StepConsts& K, const double* f, double* dense, hipStream_t s);
// streaming copy of bytes (a multiple of 16) with 16-byte loads and stores
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_unpack(const StepConsts& K, const double* dense, double* f, hipStream_t s);
hipError_t launch_tiled_step(const StepConsts& K, const double* fh, double* fmid, double* fnew, hipStream_t s);

// Fused single-pass step: strips of tile_w lanes (one column each, 8 halo
// columns) marching over row segments.  Segments are either seg_h rows each
// (seg_h > 0) or taken from a device table of (strip, ys0, ys1, 0) entries,
// one per workgroup, that balances the cost of wall and interior segments.
struct FusedShape {
    int tile_w;          // lanes per workgroup (multiple of 64, 64..1024)
    int seg_h;           // rows per segment, or <= 0 for the table
    int prefetch;        // rows loaded ahead of the one being collided (2 or 3)
    const int4* table;   // device segment table (used when seg_h <= 0)
    int nwg;             // workgroup entries of the table
    int wall_tasks;      // 1: the table runs the columns next to the x walls as single-wave tasks
};

// Partition of the strips into segments so that the costliest segment is as
// cheap as possible with at most `slots` segments.  A segment of h rows costs
// f * (h + 8) row units (8 halo rows are recomputed), f = cx on strips next
// to an x wall, times cy on segments next to a y wall.  Returns the number of
// entries written to out (capacity cap), or 0 if cap is too small.
int balanced_partition(int nx, int ny, bool wall_x, bool wall_y, int tile_w, int slots, double cx, double cy,
                       int4* out, int cap);

// The same over several independent grids (a batch): entries carry the grid
// index in their fourth field.
struct PlanGrid {
    int nx, ny;
    bool wall_x, wall_y;
};
int balanced_partition_multi(const PlanGrid* grids, int count, int tile_w, int slots, double cx, double cy, int4* out,
                             int cap);

// Columns next to each x wall that run as single-wave tasks (one 64-lane strip).
constexpr int kWallCols = 56;

// Wide strips (tile_w > 64) on a grid with x walls run the kWallCols columns
// next to each x wall as single-wave tasks, tile_w/64 to a workgroup, and cut
// only the columns between them into strips (see fusedk::FusedGrid).
bool wall_tasks_apply(int nx, bool wall_x, int tile_w);
// That plan: returns the number of workgroup entries (0 if it does not fit),
// the whole table (entries and tasks) holding *total int4.
int balanced_partition_wall_tasks(int nx, int ny, bool wall_y, int tile_w, int slots, double cx, double cy, int4* out,
                                  int cap, int* total);

// One instance of a batch, as the batched step kernels read it.
struct BatchInst {
    StepConsts K;
    long long off;   // offset of the instance's state, in doubles, within each state buffer
    int nstrips;     // 56-column strips of the instance (64-lane strips; wider tiles derive their own)
    int pad;
};

// Batched fused step: every segment of every instance in one launch.  The
// instances share the boundary type and fluid model (periodic, uniform grid);
// table entries are (strip, ys0, ys1, instance).
hipError_t launch_fused2_batch(const BatchInst* insts, const int4* table, int nwg, bool powerlaw, int prefetch,
                               const double* fin, double* fout, hipStream_t s);
hipError_t launch_fused_batch(const BatchInst* insts, const int4* table, int nwg, int pl, int tile_w, int prefetch,
                              const double* fin, double* fout, hipStream_t s);
bool fused_shape_ok(const StepConsts& K, FusedShape sh);
hipError_t launch_fused(const StepConsts& K, FusedShape sh, const double* fin, double* fout, hipStream_t s);
// Same step with one wave per velocity component (64-column strips; tile_w unused).
hipError_t launch_fused2(const StepConsts& K, FusedShape sh, const double* fin, double* fout, hipStream_t s);

// Learned closure network (BF16 MFMA) and the correction step.
int32_t cnn_param_count();
size_t cnn_workspace_size(int B, int H, int W);
hipError_t cnn_forward(char* ws, const float* params, int B, int H, int W, const double* uv, double in_scale,
                       double out_scale, double* duv, hipStream_t s);
// The forward pass on the library's fixed device scratch (no allocation);
// cnn_noalloc_bytes(B, H, W) must not exceed cnn_noalloc_capacity().
size_t cnn_noalloc_capacity();
size_t cnn_noalloc_bytes(int B, int H, int W);
hipError_t cnn_forward_noalloc(const float* params, int B, int H, int W, const double* uv, double in_scale,
                               double out_scale, double* duv, hipStream_t s);
hipError_t cnn_backward(char* ws, const float* params, int B, int H, int W, const double* duv_t, double out_scale,
                        float* grad, double* loss_dev, hipStream_t s);
hipError_t cnn_layer_io(const char* ws, int B, int H, int W, int layer, unsigned short* in_bf16, float* z_f32,
                        unsigned short* g_bf16, float* g_f32, hipStream_t s);
hipError_t cnn_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                    int step, hipStream_t s);
int closure_guard_blocks(const StepConsts& K);
hipError_t launch_closure_guard(const StepConsts& K, const double* f, const double* du, const double* dv, double hx,
                                double hy, double* part, double* out4, hipStream_t s);
// f_hat += f^eq(u + du, P) - f^eq(u, P); skipped when flag (device) holds 0
hipError_t launch_closure_apply(const StepConsts& K, double* f, const double* du, const double* dv, const double* flag,
                                hipStream_t s);
// guard decision from the guard's out4 into state {ke_ref, fall-backs, flag, windows}
hipError_t launch_closure_decide(const double* out4, double* state, double div_factor, bool reset, hipStream_t s);

}  // namespace mdf
