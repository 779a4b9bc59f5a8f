// Fused step kernels: 64-lane strips, Newtonian fluid.
#include "mdf_fused_impl.hpp"

namespace mdf {

template hipError_t launch_fused_family<64, false>(const StepConsts&, const fusedk::FusedGrid&, int, const double*,
                                                  double*, hipStream_t);
template hipError_t launch_batch_family<64, false>(const BatchInst*, const int4*, int, int, int, const double*, double*,
                                                  hipStream_t);

}  // namespace mdf
