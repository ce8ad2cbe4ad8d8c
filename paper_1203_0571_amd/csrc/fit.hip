// Profile fit by Levenberg-Marquardt, fused: one wave per stamp runs the whole
// fit (Sec. 4.1) with the stamp's LM state in LDS.  The pieces (start, one
// iteration, finish) live in lm.hpp and are shared with the work-queue form.
#include "kernels.hpp"
#include "lm.hpp"

namespace shape {
namespace {

// Four waves per SIMD: the 8-parameter kernels then get 128 VGPRs; the pixel
// loop still fits without spills (the LM solve between sweeps spills a few
// values), and the kernel runs about 8% faster than at three waves and 26%
// faster than at two.
#ifndef SHAPE_FIT_WAVES_PER_SIMD
#define SHAPE_FIT_WAVES_PER_SIMD 4
#endif
#ifndef SHAPE_FIT_STAGE_F16
#define SHAPE_FIT_STAGE_F16 1
#endif
template <int DT, int MODEL, uint32_t MASK, int LAYOUT, bool PROF>
__device__ __forceinline__ void fit_one(const shape_batch& b, const KOpts& o, const Stamp& st,
                                        const float* p_init, const float* rec, int64_t s,
                                        LmShared& W, float* p_out, float* chi2, float* perr,
                                        int32_t* iters, uint32_t* status, int32_t* sweeps,
                                        int tid) {
  lm_start<DT, MODEL, MASK, 1, LAYOUT>(b, o, st, p_init, rec, s, W, nullptr, tid);
  while (!W.L.done && W.L.it < o.max_iter_lm)
    lm_iterate<DT, MODEL, MASK, 1, LAYOUT, PROF>(b, o, st, W, nullptr, tid);
  lm_finish<MODEL, MASK>(o, st, W.L, W.sums[W.cur], s, p_out, chi2, perr, iters, status, sweeps,
                         tid);
}

template <int DT, int MODEL, uint32_t MASK, int LAYOUT, bool PROF = true>
__global__ __launch_bounds__(kWave, SHAPE_FIT_WAVES_PER_SIMD) void fit_kernel(
    shape_batch b, KOpts o, const float* p_init, const float* rec, float* p_out, float* chi2,
    float* perr, int32_t* iters, uint32_t* status, int32_t* sweeps) {
  __shared__ LmShared W;
  const int tid = threadIdx.x;
  for (int64_t s = blockIdx.x; s < b.n; s += gridDim.x) {
    const Stamp st = stamp_info(b, s);
    if (!st.bad && st.model != MODEL) continue;  // the other model's kernel owns it
    if (st.bad) {
      if (MODEL != SHAPE_SERSIC) continue;       // reported once, by the Sersic kernel
      if (tid < 8) {
        p_out[s * 8 + tid] = qnan();
        if (perr) perr[s * 8 + tid] = qnan();
      }
      if (tid == 0) {
        chi2[s] = qnan();
        iters[s] = 0;
        status[s] = st.bad;
        if (sweeps) sweeps[s] = 0;
      }
      continue;
    }
    if constexpr (SHAPE_FIT_STAGE_F16 && DT == SHAPE_F16_SCALED && LAYOUT == kLayoutRows) {
      // FP16 stamps of a uniform batch (at most 64 x 64, 8 KiB) are staged in
      // LDS once and every LM sweep reads them there: at four waves per SIMD
      // the 16 stamps of a CU (128 KiB) fit beside the LM state, while the
      // waves' stamps together exceed the L2.
      __shared__ __align__(16) _Float16 lds_px[kWave * kWave];
      const uint4* src = reinterpret_cast<const uint4*>(static_cast<const _Float16*>(b.pixels) +
                                                        st.off);
      for (int q = tid; q < st.npix / 8; q += kWave) reinterpret_cast<uint4*>(lds_px)[q] = src[q];
      wave_sync();
      shape_batch bl = b;
      bl.pixels = lds_px;
      Stamp sl = st;
      sl.off = 0;
      fit_one<DT, MODEL, MASK, LAYOUT, PROF>(bl, o, sl, p_init, rec, s, W, p_out, chi2, perr,
                                             iters, status, sweeps, tid);
    } else {
      fit_one<DT, MODEL, MASK, LAYOUT, PROF>(b, o, st, p_init, rec, s, W, p_out, chi2, perr,
                                             iters, status, sweeps, tid);
    }
    __syncthreads();  // W (and the staged stamp) are reused by the next stamp of this wave
  }
}

template <int DT, int MODEL, uint32_t MASK, bool PROF>
void launch_layout(int layout, dim3 g, dim3 t, hipStream_t stream, const shape_batch& b,
                   const KOpts& o, const float* p_init, const float* rec, float* p_out,
                   float* chi2, float* perr, int32_t* iters, uint32_t* status, int32_t* sweeps) {
  if (layout == kLayoutRows) {
    if constexpr (MODEL == SHAPE_SERSIC)
      hipLaunchKernelGGL((fit_kernel<DT, MODEL, MASK, kLayoutRows, PROF>), g, t, 0, stream, b, o,
                         p_init, rec, p_out, chi2, perr, iters, status, sweeps);
  } else if (layout == kLayoutAny) {
    hipLaunchKernelGGL((fit_kernel<DT, MODEL, MASK, kLayoutAny, PROF>), g, t, 0, stream, b, o,
                       p_init, rec, p_out, chi2, perr, iters, status, sweeps);
  } else {
    hipLaunchKernelGGL((fit_kernel<DT, MODEL, MASK, kLayoutSegs, PROF>), g, t, 0, stream, b, o,
                       p_init, rec, p_out, chi2, perr, iters, status, sweeps);
  }
}

template <int DT, int MODEL>
void launch_fit_model(const shape_batch& b, const KOpts& o, const float* p_init,
                      const float* rec, float* p_out, float* chi2, float* perr, int32_t* iters,
                      uint32_t* status, int32_t* sweeps, hipStream_t stream) {
  const int64_t grid = b.n < (1ll << 30) ? b.n : (1ll << 30);
  const dim3 g((unsigned)grid), t(kWave);
  const int layout = single_wave_layout(b, MODEL);
  if (!o.linear_init) {
    // the unprofiled form: Sersic, (Re, n, I0, sky) free (checked by the caller)
    if constexpr (MODEL != SHAPE_SERSIC) return;
    launch_layout<DT, SHAPE_SERSIC, kMaskSize, false>(layout, g, t, stream, b, o, p_init, rec,
                                                      p_out, chi2, perr, iters, status, sweeps);
  } else if (o.free_mask == kMaskAll) {
    launch_layout<DT, MODEL, kMaskAll, true>(layout, g, t, stream, b, o, p_init, rec, p_out, chi2,
                                             perr, iters, status, sweeps);
  } else {
    launch_layout<DT, MODEL, kMaskSize, true>(layout, g, t, stream, b, o, p_init, rec, p_out,
                                              chi2, perr, iters, status, sweeps);
  }
}

template <int DT>
hipError_t launch_fit_dt(const shape_batch& b, const KOpts& o, const float* p_init,
                         const float* rec, float* p_out, float* chi2, float* perr, int32_t* iters,
                         uint32_t* status, int32_t* sweeps, hipStream_t stream) {
  launch_fit_model<DT, SHAPE_SERSIC>(b, o, p_init, rec, p_out, chi2, perr, iters, status, sweeps,
                                     stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !b.model) return e;
  launch_fit_model<DT, SHAPE_MOFFAT>(b, o, p_init, rec, p_out, chi2, perr, iters, status, sweeps,
                                     stream);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fit(const shape_batch& b, const KOpts& o, const float* p_init, const float* rec,
                      float* p_out, float* chi2, float* perr, int32_t* iters, uint32_t* status,
                      int32_t* sweeps, hipStream_t stream) {
  if (b.dtype == SHAPE_F32)
    return launch_fit_dt<SHAPE_F32>(b, o, p_init, rec, p_out, chi2, perr, iters, status, sweeps,
                                    stream);
  return launch_fit_dt<SHAPE_F16_SCALED>(b, o, p_init, rec, p_out, chi2, perr, iters, status,
                                         sweeps, stream);
}

}  // namespace shape
