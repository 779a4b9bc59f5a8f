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
int diag_blocks(const StepConsts& K);
hipError_t launch_diagnostics(const StepConsts& K, const double* f, double* partials, double* out8, hipStream_t s);
hipError_t launch_pack(const StepConsts& K, const double* f, double* dense, hipStream_t s);
hipError_t launch_unpack(const StepConsts& K, const double* dense, double* f, hipStream_t s);
hipError_t launch_three_pass(const StepConsts& K, const double* fh, double* fbp, double* fmid, double* fnew,
                             hipStream_t s);

// Fused single-pass step: strips of tile_w lanes (one column each, 8 halo
// columns) marching over row segments of seg_h rows.
struct FusedShape {
    int tile_w;    // lanes per workgroup (multiple of 64, 64..1024)
    int seg_h;     // rows per segment
    int prefetch;  // rows loaded ahead of the one being collided (2 or 3)
};
bool fused_shape_ok(const StepConsts& K, FusedShape sh);
hipError_t launch_fused(const StepConsts& K, FusedShape sh, const double* fin, double* fout, hipStream_t s);
// Same step with one wave per velocity component (64-column strips; tile_w unused).
hipError_t launch_fused2(const StepConsts& K, FusedShape sh, const double* fin, double* fout, hipStream_t s);

}  // namespace mdf
