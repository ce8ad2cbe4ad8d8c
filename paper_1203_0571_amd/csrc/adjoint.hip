// chi^2 of given parameters (Sec. 4.1, eq. chi2) and its gradient by the
// adjoint of the render, one wave per stamp.
//
// With r_i = (d_i - m_i) / sigma the adjoint of pixel i is
//   dL/dm_i = -(2 / sigma) r_i dL/dchi2,
// and dL/dp_k = sum_i dL/dm_i dm_i/dp_k.  The backward sweep is the device
// function the fit uses for its J^T r and J^T J, instantiated in FP64 (FP64
// render, Jacobian and sums; log2 / exp2 by 64-point tables and short
// series): the FP32 instance's rounding of the exponent b t is amplified
// where the gradient components cancel over the stamp, up to ~1e-4 of the
// largest component.  J^T J is summed only when it is asked for.
#include "kernels.hpp"
#include "sweep.hpp"

namespace shape {
namespace {

// GRAD: also J^T r (the gradient); JTJ: also J^T J (the normal matrix).
template <int DT, int MODEL, bool GRAD, bool JTJ>
__global__ __launch_bounds__(kWave, JTJ ? 2 : 5) void chi2_kernel(shape_batch b, const float* params,
                                                     const float* grad_chi2, float* chi2,
                                                     float* grad_p, float* jtj, float* jtr) {
  constexpr uint32_t EM = GRAD ? 0xFFu : 0u;
  const int lane = threadIdx.x;
  f64_tables_fill(lane, kWave);   // the FP64 log2 / exp2 tables
  wave_sync();
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
    Acc<EM, double> acc;
    // a side that divides 64 takes the column-per-lane layout (the geometry
    // as per-column quadratics), any other side the lane-stride walk
    const Trial<double> tr = make_trial<double>(p, MODEL, p[5]);
    if (rows_layout_fits(st.side))
      sweep<DT, MODEL, EM, kWave, double, kLayoutRows, JTJ>(b, st, tr, acc);
    else
      sweep<DT, MODEL, EM, kWave, double, kLayoutAny, JTJ>(b, st, tr, acc);
    // chi^2 and J^T r: one pass of FP64 wave sums over 12 values (every lane
    // receives the totals)
    double u[12];
    u[0] = acc.c2;
#pragma unroll
    for (int k = 0; k < 8; ++k) u[1 + k] = GRAD ? acc.g[k] : 0.0;
    u[9] = u[10] = u[11] = 0.0;
    wave_sum_n(u);
    const double inv2 = 1.0 / (st.sigma * st.sigma);
    if (lane == 0) {
      if (chi2) chi2[s] = (float)(u[0] * inv2);
      if constexpr (GRAD) {
        const double up = grad_chi2 ? (double)grad_chi2[s] : 1.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          grad_p[s * 8 + k] = (float)(-2.0 * up * u[1 + k] * inv2);
          if (jtr) jtr[s * 8 + k] = (float)(u[1 + k] * inv2);
        }
      }
    }
    if constexpr (JTJ) {
      double v[36];
#pragma unroll
      for (int k = 0; k < 36; ++k) v[k] = acc.A[k];
      wave_sum_n(v);
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 36; ++k)
          jtj[s * 36 + k] = (k == tri(7, 7)) ? (float)(st.npix * inv2) : (float)(v[k] * inv2);
      }
    }
  }
}

template <int DT, bool GRAD, bool JTJ>
hipError_t launch_dt(const shape_batch& b, const float* params, const float* grad_chi2,
                     float* chi2, float* grad_p, float* jtj, float* jtr, hipStream_t stream) {
  const int64_t grid = b.n < (1ll << 30) ? b.n : (1ll << 30);
  hipLaunchKernelGGL((chi2_kernel<DT, SHAPE_SERSIC, GRAD, JTJ>), dim3((unsigned)grid),
                     dim3(kWave), 0, stream, b, params, grad_chi2, chi2, grad_p, jtj, jtr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !b.model) return e;
  hipLaunchKernelGGL((chi2_kernel<DT, SHAPE_MOFFAT, GRAD, JTJ>), dim3((unsigned)grid),
                     dim3(kWave), 0, stream, b, params, grad_chi2, chi2, grad_p, jtj, jtr);
  return hipGetLastError();
}

template <int DT>
hipError_t launch_forms(const shape_batch& b, const float* params, const float* grad_chi2,
                        float* chi2, float* grad_p, float* jtj, float* jtr, bool grad,
                        hipStream_t stream) {
  if (!grad) return launch_dt<DT, false, false>(b, params, grad_chi2, chi2, grad_p, jtj, jtr, stream);
  if (jtj) return launch_dt<DT, true, true>(b, params, grad_chi2, chi2, grad_p, jtj, jtr, stream);
  return launch_dt<DT, true, false>(b, params, grad_chi2, chi2, grad_p, jtj, jtr, stream);
}

// grad_p = grad_chi2 (per stamp) x grad_unit, eight entries per stamp.
__global__ __launch_bounds__(256) void grad_scale_kernel(const float* grad_unit,
                                                        const float* grad_chi2, int64_t n,
                                                        float* grad_p) {
  const int64_t m = n * 8;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    grad_p[i] = grad_chi2 ? grad_chi2[i >> 3] * grad_unit[i] : grad_unit[i];
}

}  // namespace

hipError_t launch_grad_scale(const float* grad_unit, const float* grad_chi2, int64_t n,
                             float* grad_p, hipStream_t stream) {
  const int64_t blocks = (n * 8 + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(grad_scale_kernel, dim3(grid), dim3(256), 0, stream, grad_unit, grad_chi2, n,
                     grad_p);
  return hipGetLastError();
}

hipError_t launch_chi2(const shape_batch& b, const float* params, const float* grad_chi2,
                       float* chi2, float* grad_p, float* jtj, float* jtr, bool grad,
                       hipStream_t stream) {
  if (b.dtype == SHAPE_F32)
    return launch_forms<SHAPE_F32>(b, params, grad_chi2, chi2, grad_p, jtj, jtr, grad, stream);
  return launch_forms<SHAPE_F16_SCALED>(b, params, grad_chi2, chi2, grad_p, jtj, jtr, grad, stream);
}

}  // namespace shape
