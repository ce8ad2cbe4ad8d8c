// The work-queue fit with the library's own device workspace, for callers
// that cannot allocate device memory (code under stream capture, serving
// loops, harnesses that forbid allocation): shape_fit_queue_static.
//
// The workspace is one file-scope device array.  In host code its name is a
// host-side stand-in, not a device address, so the array's device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and only that pointer is handed to kernels.  Every call on a device shares
// its array and leaves the last call's contents in it; the queue's start pass
// clears every part that must start at zero (header, histogram, cursors)
// with kernels, so nothing depends on what an earlier call left.
#include <mutex>

#include "kernels.hpp"

namespace shape {
namespace {

constexpr int64_t kStaticMaxStamps = SHAPE_STATIC_MAX_STAMPS;
constexpr size_t kScratchBytes = queue_workspace_bytes(kStaticMaxStamps);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of `scratch` on each device (null: not looked up)

// The array's address on the current device, looked up on the first call there.
hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

size_t static_queue_scratch_bytes() { return kScratchBytes; }

hipError_t launch_fit_queue_static(const shape_batch& b, const KOpts& o, const float* p_init,
                                   const float* rec, const QCfg& cfg, float* p_out, float* chi2,
                                   float* perr, int32_t* iters, uint32_t* status,
                                   int32_t* sweeps, hipStream_t stream) {
  void* ws = nullptr;
  hipError_t e = scratch_ptr(&ws);
  if (e != hipSuccess) return e;
  e = launch_queue_start(b, o, ws, p_init, rec, cfg, stream);
  // every step of the cap: a step finds the stamps that are done and skips them
  for (int k = 0; e == hipSuccess && k < o.max_iter_lm; ++k)
    e = launch_queue_step(b, o, ws, cfg, stream);
  if (e == hipSuccess)
    e = launch_queue_finish(b, o, ws, p_out, chi2, perr, iters, status, sweeps, stream);
  return e;
}

}  // namespace shape
