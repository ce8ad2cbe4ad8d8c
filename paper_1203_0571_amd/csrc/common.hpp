// Device helpers shared by the libshape kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bn_table.h"
#include "shape.h"

namespace shape {

constexpr int kWave = 64;
constexpr int kMinSide = 4;
constexpr int kMaxSide = 128;
constexpr float kR2Min = 1e-8f;          // floor on the elliptical R^2 (px^2)
constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;

// Scalar options as the kernels see them (copied from shape_opts by value).
struct KOpts {
  int max_iter_centroid, max_iter_moments, max_iter_lm;
  uint32_t free_mask;
  double k_gain, tol_x, tol_g, gmax, tol_lm, lambda0, chi2_rtol, n0, moffat_beta;
  int linear_init;
};

// What one wave needs to know about its stamp.
struct Stamp {
  int64_t off;
  int side;
  int npix;
  float scale;
  double sigma;
  int model;
  uint32_t bad;   // SHAPE_ST_BAD_INPUT when the stamp cannot be processed
};

__device__ inline Stamp stamp_info(const shape_batch& b, int64_t s) {
  Stamp st;
  st.side = b.side ? b.side[s] : b.side0;
  st.npix = st.side * st.side;
  st.off = b.offset ? b.offset[s] : s * (int64_t)b.side0 * b.side0;
  st.scale = (b.dtype == SHAPE_F16_SCALED) ? b.scale[s] : 1.0f;
  st.sigma = b.sigma[s];
  st.model = b.model ? b.model[s] : SHAPE_SERSIC;
  bool ok = st.side >= kMinSide && st.side <= kMaxSide && st.sigma > 0.0 &&
            (st.model == SHAPE_SERSIC || st.model == SHAPE_MOFFAT) && st.off >= 0 &&
            st.off + (int64_t)st.npix <= b.n_pixels && st.scale > 0.0f;
  st.bad = ok ? 0u : SHAPE_ST_BAD_INPUT;
  return st;
}

// Pixel k of a stamp as float (FP16 storage is multiplied by its scale).
template <int DT>
__device__ inline float load_px(const void* base, int64_t off, int k, float scale) {
  if constexpr (DT == SHAPE_F32) {
    return static_cast<const float*>(base)[off + k];
  } else {
    return static_cast<float>(static_cast<const _Float16*>(base)[off + k]) * scale;
  }
}

// Butterfly sums over the 64 lanes; every lane ends with the same bits.
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}
__device__ inline bool wave_any(bool p) { return __any(p); }

// Walk the pixels owned by this lane: k = lane, lane + 64, ... with (row, col).
template <class F>
__device__ inline void for_pixels(int side, F&& f) {
  const int npix = side * side;
  const int lane = threadIdx.x & (kWave - 1);
  int i = lane / side;
  int j = lane - i * side;
  const int di = kWave / side;
  const int dj = kWave - di * side;
#pragma unroll 1
  for (int k = lane; k < npix; k += kWave) {
    f(k, i, j);
    i += di;
    j += dj;
    if (j >= side) {
      j -= side;
      ++i;
    }
  }
}

// Sersic b(n) and db/dn from the generated Chebyshev table (FP64).
__device__ inline void sersic_bn(double n, double* b, double* db) {
  double x = log(n);
  double t = (x - kBnLogLo) / (kBnLogHi - kBnLogLo) * kBnIntervals;
  // clamp in floating point first (fmin/fmax drop a NaN), so k is always a
  // valid interval; outside [0.2, 10] the series is extrapolated
  int k = (int)fmin(fmax(t, 0.0), kBnIntervals - 0.5);
  double z = 2.0 * (t - k) - 1.0;
  double b1 = 0.0, b2 = 0.0, d1 = 0.0, d2 = 0.0;
  for (int i = kBnDegree; i >= 1; --i) {
    double nb = kBnValue[k][i] + 2.0 * z * b1 - b2;
    b2 = b1;
    b1 = nb;
    double nd = kBnDeriv[k][i] + 2.0 * z * d1 - d2;
    d2 = d1;
    d1 = nd;
  }
  double h = kBnValue[k][0] + z * b1 - b2;
  double dh = kBnDeriv[k][0] + z * d1 - d2;
  double dzdx = 2.0 * kBnIntervals / (kBnLogHi - kBnLogLo);
  *b = h + 2.0 * n;
  *db = 2.0 + dh * dzdx / n;
}

// Hardware transcendentals (v_exp_f32 = 2^x, v_log_f32 = log2, v_rcp_f32).
__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ inline float qnan() { return __builtin_nanf(""); }

}  // namespace shape
