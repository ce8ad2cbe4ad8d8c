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
  double k_gain, tol_x, tol_g, gmax, tol_lm, lambda0, chi2_rtol, n0, moffat_beta, tol_sigma;
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

// Sums over the 64 lanes with DPP: an inclusive scan inside each row of 16
// lanes (row_shr 1, 2, 4, 8), then row_bcast:15 and row_bcast:31 carry the row
// totals up, so lane 63 holds the total; it is read back as a wave-uniform
// value (every lane gets the same bits, run after run).
namespace dpp {
constexpr int kShr1 = 0x111, kShr2 = 0x112, kShr4 = 0x114, kShr8 = 0x118;
constexpr int kBcast15 = 0x142, kBcast31 = 0x143;
template <int CTRL, int ROWS>
__device__ inline int mov(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ inline float add(float v) {
  return v + __builtin_bit_cast(float, mov<CTRL, ROWS>(__builtin_bit_cast(int, v)));
}
template <int CTRL, int ROWS>
__device__ inline double add(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = mov<CTRL, ROWS>((int)(uint32_t)u);
  const int hi = mov<CTRL, ROWS>((int)(uint32_t)(u >> 32));
  return v + __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int CTRL, int ROWS>
__device__ inline long long add(long long v) {
  const uint64_t u = (uint64_t)v;
  const int lo = mov<CTRL, ROWS>((int)(uint32_t)u);
  const int hi = mov<CTRL, ROWS>((int)(uint32_t)(u >> 32));
  return (long long)(u + (((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
}  // namespace dpp

template <class T>
__device__ inline T wave_total(T v) {
  v = dpp::add<dpp::kShr1, 0xf>(v);
  v = dpp::add<dpp::kShr2, 0xf>(v);
  v = dpp::add<dpp::kShr4, 0xf>(v);
  v = dpp::add<dpp::kShr8, 0xf>(v);
  v = dpp::add<dpp::kBcast15, 0xa>(v);
  v = dpp::add<dpp::kBcast31, 0xc>(v);
  return v;
}
__device__ inline float wave_sum(float v) {
  const float t = wave_total(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, t), 63));
}
__device__ inline double wave_sum(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, wave_total(v));
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ inline long long readlane64(long long v, int lane) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return (long long)(((uint64_t)hi << 32) | lo);
}
__device__ inline double read_lane_f64(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ inline bool wave_any(bool p) { return __any(p); }

// Halving steps of a wave reduction: the values a (kept) and b are summed
// over lane pairs, v_permlane32_swap pairing lane l with l + 32 (afterwards
// lanes 0-31 carry a's sums, lanes 32-63 b's), v_permlane16_swap pairing the
// rows of 16 within each half (rows 0 and 2 carry a's, rows 1 and 3 b's).
// (The swapped pair is taken into scalar locals before the reinterpretation:
// reinterpreting the elements of the returned pair in place compiled to an
// add of the first element to itself.)
__device__ __forceinline__ void swap_add32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  const unsigned x = r[0], y = r[1];
  a = __builtin_bit_cast(float, x) + __builtin_bit_cast(float, y);
}
__device__ __forceinline__ void swap_add16(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  const unsigned x = r[0], y = r[1];
  a = __builtin_bit_cast(float, x) + __builtin_bit_cast(float, y);
}

__device__ __forceinline__ double pair_to_double(unsigned lo, unsigned hi) {
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// The same halving for FP64 values: both 32-bit halves take the same swap.
__device__ __forceinline__ void swap_add32(double& a, double& b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  const unsigned x0 = lo[0], y0 = lo[1], x1 = hi[0], y1 = hi[1];
  a = pair_to_double(x0, x1) + pair_to_double(y0, y1);
}
__device__ __forceinline__ void swap_add16(double& a, double& b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  const unsigned x0 = lo[0], y0 = lo[1], x1 = hi[0], y1 = hi[1];
  a = pair_to_double(x0, x1) + pair_to_double(y0, y1);
}

// Sums of N FP64 values (N a multiple of 4) over the wave, every lane
// receiving all N: two halving steps (row k then carries entries
// kN/4 .. kN/4 + N/4 - 1), a scan within each row of 16, and the row totals
// read back from lanes 15, 31, 47 and 63.
template <int N>
__device__ inline void wave_sum_n(double (&u)[N]) {
  static_assert(N % 4 == 0, "N must be a multiple of 4");
  constexpr int H = N / 2, Q = N / 4;
#pragma unroll
  for (int j = 0; j < H; ++j) swap_add32(u[j], u[j + H]);
#pragma unroll
  for (int j = 0; j < Q; ++j) swap_add16(u[j], u[j + Q]);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    u[j] = dpp::add<dpp::kShr1, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr2, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr4, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr8, 0xf>(u[j]);
  }
  double t[N];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const uint64_t w = __builtin_bit_cast(uint64_t, u[j]);
      const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)w, 16 * k + 15);
      const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(w >> 32), 16 * k + 15);
      t[Q * k + j] = __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = t[i];
}

// The same for N FP32 values.
template <int N>
__device__ inline void wave_sum_n(float (&u)[N]) {
  static_assert(N % 4 == 0, "N must be a multiple of 4");
  constexpr int H = N / 2, Q = N / 4;
#pragma unroll
  for (int j = 0; j < H; ++j) swap_add32(u[j], u[j + H]);
#pragma unroll
  for (int j = 0; j < Q; ++j) swap_add16(u[j], u[j + Q]);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    u[j] = dpp::add<dpp::kShr1, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr2, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr4, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr8, 0xf>(u[j]);
  }
  float t[N];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int j = 0; j < Q; ++j)
      t[Q * k + j] = __builtin_bit_cast(
          float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, u[j]), 16 * k + 15));
  }
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = t[i];
}

// Walk the pixels owned by thread `tid` of a team of STRIDE threads working on
// one stamp: k = tid, tid + STRIDE, ... with (row, col).
template <int STRIDE = kWave, class F>
__device__ inline void for_pixels(int side, F&& f, int tid = -1) {
  const int npix = side * side;
  const int t0 = tid < 0 ? (int)(threadIdx.x & (kWave - 1)) : tid;
  int i = t0 / side;
  int j = t0 - i * side;
  const int di = STRIDE / side;
  const int dj = STRIDE - di * side;
#pragma unroll 1
  for (int k = t0; k < npix; k += STRIDE) {
    f(k, i, j);
    i += di;
    j += dj;
    if (j >= side) {
      j -= side;
      ++i;
    }
  }
}

// Stamp pixel at a 32-bit element index from the stamp's own base.
template <int DT>
__device__ __forceinline__ float load_rel(const void* sp, uint32_t k, float scale) {
  if constexpr (DT == SHAPE_F32) {
    return static_cast<const float*>(sp)[k];
  } else {
    return static_cast<float>(static_cast<const _Float16*>(sp)[k]) * scale;
  }
}

template <int DT>
__device__ __forceinline__ const void* stamp_base(const shape_batch& b, const Stamp& st) {
  if constexpr (DT == SHAPE_F32)
    return static_cast<const float*>(b.pixels) + st.off;
  else
    return static_cast<const _Float16*>(b.pixels) + st.off;
}

// The pixels of one stamp as a wave sweeps them, for kernels that sweep a
// stamp several times: each(f) calls f(value, k, i, j) for every pixel k of
// this lane (row i, column j).  SIDE = 0: any side, read from memory on every
// sweep.  SIDE in {8, 16, 32, 64}: the stamp is read once into registers,
// lane l holding pixel l + 64 m in slot m (row m * 64 / SIDE + l / SIDE,
// column l % SIDE), and every later sweep runs from registers.
template <int DT, int SIDE>
struct StampPixels {
  static_assert(SIDE == 8 || SIDE == 16 || SIDE == 32 || SIDE == 64, "side must divide 64");
  static constexpr int kSlots = SIDE * SIDE / kWave;
  float v[kSlots];
  int lane;
  __device__ __forceinline__ StampPixels(const shape_batch& b, const Stamp& st, int l) : lane(l) {
    const void* sp = stamp_base<DT>(b, st);
#pragma unroll
    for (int m = 0; m < kSlots; ++m) v[m] = load_rel<DT>(sp, (uint32_t)(l + kWave * m), st.scale);
  }
  template <class F>
  __device__ __forceinline__ void each(F&& f) const {
    int il = lane / SIDE, jl = lane & (SIDE - 1);
    // Opaque to the optimiser, so coordinates derived from il, jl are formed
    // anew in each sweep instead of being hoisted out of the caller's
    // iteration loop into one register per pixel.
    asm volatile("" : "+v"(il), "+v"(jl));
#pragma unroll
    for (int m = 0; m < kSlots; ++m) f(v[m], lane + kWave * m, m * (kWave / SIDE) + il, jl);
  }
};

template <int DT>
struct StampPixels<DT, 0> {
  const void* base;
  int64_t off;
  int side;
  float scale;
  __device__ __forceinline__ StampPixels(const shape_batch& b, const Stamp& st, int)
      : base(b.pixels), off(st.off), side(st.side), scale(st.scale) {}
  template <class F>
  __device__ __forceinline__ void each(F&& f) const {
    for_pixels(side, [&](int k, int i, int j) { f(load_px<DT>(base, off, k, scale), k, i, j); });
  }
};

// Whether a batch of one side (no side array) may use StampPixels<_, side0>.
__host__ __device__ inline constexpr bool register_side(int side) {
  return side == 8 || side == 16 || side == 32 || side == 64;
}

// Make LDS writes of one lane visible to the other lanes of its wave (no
// cross-wave barrier: usable where the waves of a workgroup diverge).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Sersic b(n) and db/dn from the generated Chebyshev table in FP64 (the FP64
// sweep of the adjoint).  The interval variable ln n is taken in FP64: from
// the FP32 hardware log2, b(n) was off by up to 5e-8 relative, which moved
// the FP64 gradient by up to 4e-5 of its scale on 32 x 32 Gaussian stamps
// (b t reaches ~10 inside the stamp).
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

// b(n) and db/dn in FP32 (in = 1/n) for the FP32 sweep's constants, from
// the FP32 copy of the series (cut at degree kBnDegreeF; the dropped terms
// are below 2e-11, far under FP32 rounding).
__device__ inline void sersic_bn_f32(float n, float in, float* b, float* db) {
  const float x = __builtin_amdgcn_logf(n) * (float)kLn2;
  const float t = (x - (float)kBnLogLo) * (float)(kBnIntervals / (kBnLogHi - kBnLogLo));
  const int k = (int)fminf(fmaxf(t, 0.0f), kBnIntervals - 0.5f);
  const float z = 2.0f * (t - (float)k) - 1.0f, z2 = 2.0f * z;
  float b1 = 0.0f, b2 = 0.0f, d1 = 0.0f, d2 = 0.0f;
#pragma unroll
  for (int i = kBnDegreeF; i >= 1; --i) {
    const float nb = fmaf(z2, b1, kBnValueF[k][i]) - b2;
    b2 = b1;
    b1 = nb;
    const float nd = fmaf(z2, d1, kBnDerivF[k][i]) - d2;
    d2 = d1;
    d1 = nd;
  }
  const float h = fmaf(z, b1, kBnValueF[k][0]) - b2;
  const float dh = fmaf(z, d1, kBnDerivF[k][0]) - d2;
  *b = fmaf(2.0f, n, h);
  *db = fmaf(dh * (float)(2.0 * kBnIntervals / (kBnLogHi - kBnLogLo)), in, 2.0f);
}

// 1/x for a positive normal double: the hardware estimate and two Newton
// steps (each squares the relative error).
__device__ inline double rcp_f64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// Hardware transcendentals (v_exp_f32 = 2^x, v_log_f32 = log2, v_rcp_f32).
__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ inline float qnan() { return __builtin_nanf(""); }

}  // namespace shape
