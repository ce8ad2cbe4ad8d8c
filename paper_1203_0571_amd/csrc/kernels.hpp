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

// Work-queue configuration (see shape_queue_cfg in shape.h).
struct QCfg {
  int team;           // waves per stamp for large stamps: 1, 2 or 4
  int team_min_side;  // stamps with side >= this are taken by a team
  int grid;           // persistent workgroups; 0 = all that fit on the device
  int chunk;          // stamps per cursor pop at most; 0 = the default
};

// Workspace layout of the queue form: a 256-byte header, the cursor lines,
// the (model, side) histogram, the stamp order, two stamp lists and the
// per-stamp state (parameters, trial point, current sums, damping, counters,
// phase, the last sweep's sums and the pending sweep's constants), each an
// array over the stamps.
constexpr int kBuckets = 512;
constexpr int kClasses = 4;        // (Sersic, Moffat) x (team of waves, single wave)
constexpr int kCursors = 8;
constexpr int kCursorStride = 32;  // uint32 per cursor line (128 bytes)
constexpr size_t kCursorBytes = (size_t)kClasses * kCursors * kCursorStride * 4;
constexpr int kConstRow = 32;      // floats of sweep constants per stamp (27 used)
__host__ __device__ constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
__host__ __device__ constexpr size_t queue_workspace_bytes(int64_t n) {
  const size_t m = (size_t)n;
  return 256 + kCursorBytes + align256(kBuckets * 4) + 3 * align256(m * 4) +  // order, lists
         2 * align256(m * 64) + align256(m * 45 * 8) +                        // p, pt, sums
         2 * align256(m * 8) + 4 * align256(m * 4) +                          // lambda, smax, ints
         align256(m * 45 * 8) + align256(m * kConstRow * 4);
}
hipError_t launch_queue_start(const shape_batch& b, const KOpts& o, void* ws, const float* p_init,
                              const float* rec, const QCfg& cfg, hipStream_t stream);
hipError_t launch_queue_step(const shape_batch& b, const KOpts& o, void* ws, const QCfg& cfg,
                             hipStream_t stream);
hipError_t launch_queue_drain(const shape_batch& b, const KOpts& o, void* ws, const QCfg& cfg,
                              hipStream_t stream);
hipError_t launch_queue_finish(const shape_batch& b, const KOpts& o, void* ws, float* p_out,
                               float* chi2, float* perr, int32_t* iters, uint32_t* status,
                               int32_t* sweeps, hipStream_t stream);

// The queue fit on the library's static workspace (at most
// SHAPE_STATIC_MAX_STAMPS stamps); no allocation.
size_t static_queue_scratch_bytes();
hipError_t launch_fit_queue_static(const shape_batch& b, const KOpts& o, const float* p_init,
                                   const float* rec, const QCfg& cfg, float* p_out, float* chi2,
                                   float* perr, int32_t* iters, uint32_t* status,
                                   int32_t* sweeps, hipStream_t stream);

hipError_t launch_stars(const shape_batch& b, int profile, const float* rec, double tol,
                        int max_iter, double beta, float* out, int32_t* iters, uint32_t* status,
                        hipStream_t stream);

int frame_bins(int height, int width);
hipError_t launch_frame_detect(const shape_frames& f, int max_side, float* info, int32_t* peak,
                               int32_t* box, uint32_t* status, hipStream_t stream);
hipError_t launch_frame_offsets(const int32_t* box, int64_t n, int64_t* offset, int64_t* total,
                                hipStream_t stream);
hipError_t launch_frame_cut(const shape_frames& f, const int32_t* box, const int64_t* offset,
                            float* stamps, int64_t capacity, int32_t* sides, hipStream_t stream);

hipError_t launch_chi2(const shape_batch& b, const float* params, const float* grad_chi2,
                       float* chi2, float* grad_p, float* jtj, float* jtr, bool grad,
                       hipStream_t stream);
hipError_t launch_grad_scale(const float* grad_unit, const float* grad_chi2, int64_t n,
                             float* grad_p, hipStream_t stream);

}  // namespace shape
