// chi^2 of given parameters (Sec. 4.1, eq. chi2) and its gradient by the
// adjoint of the render, one wave per stamp.
//
// With r_i = (d_i - m_i) / sigma the adjoint of pixel i is
//   dL/dm_i = -(2 / sigma) r_i dL/dchi2,
// and dL/dp_k = sum_i dL/dm_i dm_i/dp_k.  The backward sweep is the device
// function the fit uses for its J^T r and J^T J, instantiated in FP64 (FP64
// render, Jacobian and sums; log2 / exp2 from series): the FP32 instance's
// rounding of the exponent b t is amplified where the gradient components
// cancel over the stamp, up to ~1e-4 of the largest component.
#include "kernels.hpp"
#include "sweep.hpp"

namespace shape {
namespace {

template <int DT, int MODEL, bool GRAD>
__global__ __launch_bounds__(kWave) void chi2_kernel(shape_batch b, const float* params,
                                                     const float* grad_chi2, float* chi2,
                                                     float* grad_p, float* jtj, float* jtr) {
  constexpr uint32_t EM = GRAD ? 0xFFu : 0u;
  __shared__ double S[45];
  const int lane = threadIdx.x;
  for (int64_t s = blockIdx.x; s < b.n; s += gridDim.x) {
    const Stamp st = stamp_info(b, s);
    if (!st.bad && st.model != MODEL) continue;  // the other model's launch owns it
    if (st.bad && MODEL != SHAPE_SERSIC) continue;
    double p[8];
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      p[k] = params[s * 8 + k];
      finite = finite && __builtin_isfinite(p[k]);
    }
    if (st.bad || !finite) {
      if (lane == 0) {
        if (chi2) chi2[s] = qnan();
        if (GRAD) {
          for (int k = 0; k < 8; ++k) {
            grad_p[s * 8 + k] = qnan();
            if (jtr) jtr[s * 8 + k] = qnan();
          }
          if (jtj)
            for (int k = 0; k < 36; ++k) jtj[s * 36 + k] = qnan();
        }
      }
      continue;
    }
    {
      Acc<EM, double> acc;
      sweep<DT, MODEL, EM, kWave, double>(b, st, make_trial<double>(p, MODEL, p[5]), acc);
      reduce_store<EM, double>(acc, S, lane);
    }
    // lane 0 wrote S and is the only reader
    const double inv2 = 1.0 / (st.sigma * st.sigma);
    if (lane == 0) {
      if (chi2) chi2[s] = (float)(S[0] * inv2);
      if constexpr (GRAD) {
        const double up = grad_chi2 ? (double)grad_chi2[s] : 1.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          grad_p[s * 8 + k] = (float)(-2.0 * up * S[1 + k] * inv2);
          if (jtr) jtr[s * 8 + k] = (float)(S[1 + k] * inv2);
        }
        if (jtj) {
#pragma unroll
          for (int k = 0; k < 36; ++k)
            jtj[s * 36 + k] = (k == tri(7, 7)) ? (float)(st.npix * inv2) : (float)(S[9 + k] * inv2);
        }
      }
    }
    wave_sync();  // S is reused by the next stamp
  }
}

template <int DT, bool GRAD>
hipError_t launch_dt(const shape_batch& b, const float* params, const float* grad_chi2,
                     float* chi2, float* grad_p, float* jtj, float* jtr, hipStream_t stream) {
  const int64_t grid = b.n < (1ll << 30) ? b.n : (1ll << 30);
  hipLaunchKernelGGL((chi2_kernel<DT, SHAPE_SERSIC, GRAD>), dim3((unsigned)grid), dim3(kWave), 0,
                     stream, b, params, grad_chi2, chi2, grad_p, jtj, jtr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !b.model) return e;
  hipLaunchKernelGGL((chi2_kernel<DT, SHAPE_MOFFAT, GRAD>), dim3((unsigned)grid), dim3(kWave), 0,
                     stream, b, params, grad_chi2, chi2, grad_p, jtj, jtr);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_chi2(const shape_batch& b, const float* params, const float* grad_chi2,
                       float* chi2, float* grad_p, float* jtj, float* jtr, bool grad,
                       hipStream_t stream) {
  if (b.dtype == SHAPE_F32)
    return grad ? launch_dt<SHAPE_F32, true>(b, params, grad_chi2, chi2, grad_p, jtj, jtr, stream)
                : launch_dt<SHAPE_F32, false>(b, params, grad_chi2, chi2, grad_p, jtj, jtr, stream);
  return grad ? launch_dt<SHAPE_F16_SCALED, true>(b, params, grad_chi2, chi2, grad_p, jtj, jtr,
                                                  stream)
              : launch_dt<SHAPE_F16_SCALED, false>(b, params, grad_chi2, chi2, grad_p, jtj, jtr,
                                                   stream);
}

}  // namespace shape
