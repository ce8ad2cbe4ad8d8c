// Star sizes from weighted moments (Sec. 4.2), one wave per stamp.
//
// About the centre and ellipticity of the moments stage, with R the model's
// elliptical radius (R^2 = |S(g) theta|^2 / (1 - |g|^2)) and f = I - sky0, each
// step sums r0 = sum f W, r2 = sum f W R^2, r4 = sum f W R^4 (FP64) for the
// current weight width w, then:
//   Gaussian (Sec. 4.2.1, W = exp(-R^2 / 2 w^2)): sigma = sqrt(r2 / r0),
//            I0 = r0 / (pi sigma^2)  (exact when w = sigma);
//   Moffat   (Sec. 4.2.2, W = (1 + R^2 / w^2)^-3): beta = 1 / (r4 r0 / 2 r2^2 - 1),
//            rd = sqrt(r2 / r0 (beta + 1)), I0 = r0 (beta + 2) / (pi rd^2)
//            (exact when w = rd);
// and sets w to the new size until the fractional change is below tol.
#include "kernels.hpp"

namespace shape {
namespace {

constexpr double kPi = 3.14159265358979323846;

template <int DT, int PROFILE>
__global__ __launch_bounds__(kWave) void star_kernel(shape_batch b, const float* rec, double tol,
                                                     int max_iter, float* out, int32_t* iters,
                                                     uint32_t* status) {
  const int lane = threadIdx.x;
  for (int64_t s = blockIdx.x; s < b.n; s += gridDim.x) {
    const Stamp st = stamp_info(b, s);
    float r[SHAPE_REC_LEN];
    bool finite = true;
#pragma unroll
    for (int q = 0; q < SHAPE_REC_LEN; ++q) {
      r[q] = rec[s * SHAPE_REC_LEN + q];
      finite = finite && __builtin_isfinite(r[q]);
    }
    if (st.bad || !finite) {
      if (lane < 4) out[s * 4 + lane] = qnan();
      if (lane == 0) {
        iters[s] = 0;
        status[s] = st.bad ? st.bad : SHAPE_ST_BAD_INPUT;
      }
      continue;
    }
    const float x0 = r[SHAPE_REC_X0], y0 = r[SHAPE_REC_Y0];
    const double g1 = r[SHAPE_REC_E1], g2 = r[SHAPE_REC_E2];
    const float a11 = (float)(1.0 - g1), a12 = (float)(-g2), a22 = (float)(1.0 + g1);
    const float invD = (float)(1.0 / (1.0 - g1 * g1 - g2 * g2));
    const float sky = r[SHAPE_REC_SKY0];
    // starting width: the Gaussian of half-light radius r50, or the beta = 3
    // Moffat of that half-light radius (r50 = rd sqrt(2^(1/2) - 1))
    double w = PROFILE == 0 ? (double)r[SHAPE_REC_SIGW]
                            : (double)r[SHAPE_REC_R50] / sqrt(sqrt(2.0) - 1.0);
    double size = w, beta = 0.0, I0 = 0.0, r0 = 0.0;
    uint32_t stt = 0;
    int it = 0;
    while (it < max_iter) {
      const float c = (float)(PROFILE == 0 ? kLog2e / (2.0 * w * w) : 1.0 / (w * w));
      double s0 = 0.0, s2 = 0.0, s4 = 0.0;
      for_pixels(st.side, [&](int k, int i, int j) {
        const float d = load_px<DT>(b.pixels, st.off, k, st.scale);
        const float t1 = (float)j - x0, t2 = (float)i - y0;
        const float v1 = fmaf(a11, t1, a12 * t2), v2 = fmaf(a12, t1, a22 * t2);
        const float R2 = fmaf(v1, v1, v2 * v2) * invD;
        float W;
        if constexpr (PROFILE == 0) {
          W = fast_exp2(-R2 * c);
        } else {
          const float ib = fast_rcp(fmaf(R2, c, 1.0f));
          W = ib * ib * ib;
        }
        const float fw = (d - sky) * W;
        s0 += (double)fw;
        s2 += (double)(fw * R2);
        s4 += (double)(fw * R2 * R2);
      });
      s0 = wave_sum(s0);
      s2 = wave_sum(s2);
      s4 = wave_sum(s4);
      ++it;
      r0 = s0;
      if (!(s0 > 0.0) || !(s2 > 0.0)) {
        stt |= SHAPE_ST_NONPOSITIVE_FLUX;
        break;
      }
      double ns;
      if constexpr (PROFILE == 0) {
        ns = sqrt(s2 / s0);
        I0 = s0 / (kPi * ns * ns);
      } else {
        const double q = s4 * s0 / (2.0 * s2 * s2) - 1.0;
        if (!(q > 0.0)) {
          stt |= SHAPE_ST_SINGULAR;
          break;
        }
        beta = 1.0 / q;
        ns = sqrt(s2 / s0 * (beta + 1.0));
        I0 = s0 * (beta + 2.0) / (kPi * ns * ns);
      }
      const double change = fabs(ns - w) / ns;
      size = ns;
      w = ns;
      if (change < tol) {
        stt |= SHAPE_ST_CONVERGED;
        break;
      }
    }
    if (!(stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_SINGULAR)))
      stt |= SHAPE_ST_MAX_ITER;
    if (lane == 0) {
      out[s * 4 + 0] = (float)size;
      out[s * 4 + 1] = (float)beta;
      out[s * 4 + 2] = (float)I0;
      out[s * 4 + 3] = (float)r0;
      iters[s] = it;
      status[s] = stt;
    }
  }
}

}  // namespace

hipError_t launch_stars(const shape_batch& b, int profile, const float* rec, double tol,
                        int max_iter, float* out, int32_t* iters, uint32_t* status,
                        hipStream_t stream) {
  const int64_t grid = b.n < (1ll << 30) ? b.n : (1ll << 30);
  const dim3 g((unsigned)grid), t(kWave);
  if (b.dtype == SHAPE_F32) {
    if (profile == 0)
      hipLaunchKernelGGL((star_kernel<SHAPE_F32, 0>), g, t, 0, stream, b, rec, tol, max_iter, out,
                         iters, status);
    else
      hipLaunchKernelGGL((star_kernel<SHAPE_F32, 1>), g, t, 0, stream, b, rec, tol, max_iter, out,
                         iters, status);
  } else {
    if (profile == 0)
      hipLaunchKernelGGL((star_kernel<SHAPE_F16_SCALED, 0>), g, t, 0, stream, b, rec, tol,
                         max_iter, out, iters, status);
    else
      hipLaunchKernelGGL((star_kernel<SHAPE_F16_SCALED, 1>), g, t, 0, stream, b, rec, tol,
                         max_iter, out, iters, status);
  }
  return hipGetLastError();
}

}  // namespace shape
