// Host-side launch functions of the libshape kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace shape {

hipError_t launch_centroid(const shape_batch& b, const KOpts& o, float* rec, int32_t* iters,
                           uint32_t* status, hipStream_t stream);
hipError_t launch_moments(const shape_batch& b, const KOpts& o, const float* rec_in,
                          float* rec_out, int32_t* iters, uint32_t* status, hipStream_t stream);
hipError_t launch_fit(const shape_batch& b, const KOpts& o, const float* p_init, const float* rec,
                      float* p_out, float* chi2, float* perr, int32_t* iters, uint32_t* status,
                      int32_t* sweeps, hipStream_t stream);

}  // namespace shape
