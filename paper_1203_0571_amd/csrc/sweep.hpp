// The per-pixel sweep shared by the fit and the chi^2 forward/backward
// kernels: render the model (Sec. 4.1 eq. ser, Sec. 4.2.2 eq. mof) at a set of
// parameters, form r = d - m and the Jacobian columns, and accumulate
// sum r^2, J^T r (FP64) and J^T J (FP32) over the stamp.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace shape {


__host__ __device__ inline constexpr int tri(int k, int l) {
  return k <= l ? k * 8 - k * (k - 1) / 2 + (l - k) : l * 8 - l * (l - 1) / 2 + (k - l);
}
// Parameters with a Jacobian column for a given model and free mask (beta is
// never fitted for Moffat stars).
__host__ __device__ inline constexpr uint32_t eff_mask(uint32_t mask, int model) {
  return model == SHAPE_MOFFAT ? (mask & ~(1u << 5)) : mask;
}
__host__ __device__ inline constexpr bool has(uint32_t m, int k) { return (m >> k) & 1u; }
__host__ __device__ inline constexpr int popcount(uint32_t m) { return m ? (int)(m & 1u) + popcount(m >> 1) : 0; }
// Index of the a-th set bit of m (a counted from 0); 0 when there is none.
__host__ __device__ inline constexpr int nth_bit(uint32_t m, int a) {
  for (int k = 0; k < 32; ++k)
    if ((m >> k) & 1u) {
      if (a == 0) return k;
      --a;
    }
  return 0;
}

// FP64 log2 and exp2 from series alone, accurate to about 1e-17 relative:
//   log2 x: x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh z,
//           z = (m - 1)/(m + 1), |z| <= 3 - 2 sqrt(2); the odd series to z^23
//           leaves a relative error below 1e-19.
//   exp2 x: x = k + f with k = rint(x), |f| <= 1/2; e^(f ln 2) by its Taylor
//           series to degree 13 (remainder below 1e-17), scaled by 2^k.
// They fill the tables of the per-pixel forms below.
__device__ __forceinline__ double log2_series(double x) {
  int e;
  double m = __builtin_frexp(x, &e);  // [0.5, 1)
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  const double z = (m - 1.0) / (m + 1.0);
  const double w = z * z;
  double s = 1.0 / 23.0;
#pragma unroll
  for (int k = 21; k >= 1; k -= 2) s = fma(s, w, 1.0 / (double)k);
  return (double)e + 2.0 * z * s * kLog2e;
}

// 1 / n! for Taylor series of e^y, as compile-time constants.
template <int N>
struct InvFact {
  static constexpr double v = InvFact<N - 1>::v / N;
};
template <>
struct InvFact<0> {
  static constexpr double v = 1.0;
};
// sum_{n = M..D} y^(n-M) / n! by Horner (M = 0: the series of e^y to degree D).
template <int D, int M = 0>
__device__ __forceinline__ double exp_taylor(double y) {
  if constexpr (M == D)
    return InvFact<D>::v;
  else
    return fma(exp_taylor<D, M + 1>(y), y, InvFact<M>::v);
}

__device__ __forceinline__ double exp2_series(double x) {
  if (!(x > -1100.0)) return x != x ? x : 0.0;
  if (x > 1100.0) return __builtin_inf();
  const double k = __builtin_rint(x);
  const double y = (x - k) * kLn2;
  return __builtin_ldexp(exp_taylor<13>(y), (int)k);
}

// Per-pixel FP64 log2 and exp2 of the FP64 instance (Tang's table method):
// the argument is reduced against 64 table points, and a short series covers
// the remainder, cut where its error is below 4e-14 relative -- some 1e5
// times below what the gradient's bar needs (the FP32 instance, at ~1e-7,
// misses it by ~1e3; the largest gradient error against the oracle, about
// 1e-7 of the largest component, is the same as with the series cut at
// 1e-17).
//   log2 x: x = 2^e m2, m2 in [1, 2); j = the top 6 bits of m2's fraction,
//           c_j = 1 + (j + 1/2) / 64, r = m2 / c_j - 1 (|r| < 1/128);
//           log2 x = e + log2 c_j + ln(1 + r) log2 e, ln(1 + r) to r^5
//           (the first dropped term, r^6 / 6, is below 4e-14).
//   exp2 x: x = (64 k + j) / 64 + f, |f| <= 1/128; 2^x = 2^k 2^(j/64) e^(f ln 2),
//           the Taylor series of e^y to degree 4 (remainder below 4e-14).
// The tables (2^(j/64), 1 / c_j, log2 c_j) live in LDS; f64_tables_fill
// forms them with the series above, before the first sweep of a kernel.
constexpr int kF64Tab = 64;
__shared__ double f64_tab[3 * kF64Tab];

__device__ __forceinline__ void f64_tables_fill(int t, int nthreads) {
  for (int j = t; j < kF64Tab; j += nthreads) {
    const double c = 1.0 + (j + 0.5) / kF64Tab;
    f64_tab[j] = exp2_series(j / (double)kF64Tab);
    f64_tab[kF64Tab + j] = 1.0 / c;
    f64_tab[2 * kF64Tab + j] = log2_series(c);
  }
}

__device__ __forceinline__ double log2_f64(double x) {   // x > 0, finite
  int e;
  const double m = __builtin_frexp(x, &e);   // [0.5, 1), the same fraction bits
  const uint32_t hi = (uint32_t)(__builtin_bit_cast(uint64_t, m) >> 32);
  const int j = (int)((hi >> 14) & (kF64Tab - 1));   // top 6 of the 52 fraction bits
  const double r = fma(2.0 * m, f64_tab[kF64Tab + j], -1.0);
  double s = 1.0 / 5.0;   // ln(1 + r) = r (1 - r/2 + r^2/3 - r^3/4 + r^4/5)
#pragma unroll
  for (int k = 4; k >= 1; --k) s = fma(s, r, ((k & 1) ? 1.0 : -1.0) / (double)k);
  return fma(r * s, kLog2e, (double)(e - 1) + f64_tab[2 * kF64Tab + j]);
}

__device__ __forceinline__ double exp2_f64(double x) {
  if (!(x > -1100.0)) return x != x ? x : 0.0;
  if (x > 1100.0) return __builtin_inf();
  const double K = __builtin_rint(x * kF64Tab);
  const int ki = (int)K;
  const int j = ki & (kF64Tab - 1), k = ki >> 6;   // floor division by 64
  const double y = fma(K, -1.0 / kF64Tab, x) * kLn2;   // |y| <= ln 2 / 128
  return __builtin_ldexp(f64_tab[j] * exp_taylor<4>(y), k);
}

// Arithmetic of one sweep instance: FP32 with the hardware transcendentals
// (about 1 ulp; the fit), or FP64 with the series above (the chi^2 gradient).
template <typename T>
struct Arith;
template <>
struct Arith<float> {
  static __device__ __forceinline__ float ex2(float x) { return fast_exp2(x); }
  static __device__ __forceinline__ float lg2(float x) { return fast_log2(x); }
  static __device__ __forceinline__ float rcp(float x) { return fast_rcp(x); }
  static __device__ __forceinline__ float fma(float a, float b, float c) { return fmaf(a, b, c); }
  static __device__ __forceinline__ float uni(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
  }
  static constexpr float kR2Floor = kR2Min;
};
template <>
struct Arith<double> {
  static __device__ __forceinline__ double ex2(double x) { return exp2_f64(x); }
  static __device__ __forceinline__ double lg2(double x) { return log2_f64(x); }
  static __device__ __forceinline__ double rcp(double x) { return rcp_f64(x); }
  static __device__ __forceinline__ double fma(double a, double b, double c) { return ::fma(a, b, c); }
  static __device__ __forceinline__ double uni(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  }
  static constexpr double kR2Floor = 1e-8;
};

// Trial parameters as a sweep instance uses them.  With v = S(e) u,
// R^2 = |v|^2 / D and the amplitude folded into the constants:
//   Sersic: t = 2^(L ha + hc) (L = log2 R^2), m0 = 2^(nb2 t), c = m0 t,
//           dm/dRe = c k4, dm/dn = c (L k5a + k5b), h = c k7 / R^2;
//   Moffat: base = 1 + R^2 irdsq, m0 = base^-beta, c = m0 / base,
//           dm/drd = c R^2 k4, dm/dbeta = m0 log2(base) k5a, h = c k7;
// where h = (2 / D) dm/dR^2, so that dm/dx0 = h (N u)_1, dm/dy0 = h (N u)_2
// with N = -S(e)^2, and dm/de_k = h (w_k + e_k R^2) with w_1 = v2 u2 - v1 u1,
// w_2 = -(v1 u2 + v2 u1).
//
// Along one column of a stamp (u1 fixed) R^2 and the two e-derivative factors
// are quadratics in u2:
//   R^2            = qa u2^2 + qb1 u1 u2 + qc2 u1^2,
//   e1 R^2 + w_1   = p2a u2^2 + e1 qb1 u1 u2 + (e1 qc2 - a11) u1^2,
//   e2 R^2 + w_2   = p3a u2^2 + (e2 qb1 - 2) u1 u2 + (e2 qc2 - a12) u1^2,
// with qa = (a12^2 + a22^2) / D, qb1 = 4 a12 / D, qc2 = (a11^2 + a12^2) / D,
// p2a = e1 qa + a22, p3a = e2 qa - a12 (S(e) = [[a11, a12], [a12, a22]]).
template <typename T>
struct Trial {
  T x0, y0, e1, e2, a11, a12, a22, invD;
  T I0, sky;
  T n11, n12, n22;
  T qa, qb1, qc2, p2a, p3a;
  T ha, hc, nb2;
  T beta, irdsq;
  T k4, k5a, k5b, k7;
};
using TrialF = Trial<float>;

template <uint32_t EM, typename T = float>
struct Acc {
  double c2;
  double g[8];
  T A[36];
};

// The sweep's constants from the FP64 parameters, formed in the instance's
// own arithmetic (FP32: hardware log2 / rcp, about 1 ulp).  UNI: the whole
// wave forms the same constants and keeps them wave-uniform (scalar
// registers); without it one lane forms its own stamp's constants (the
// batched form), with the same arithmetic.
template <typename T = float, bool UNI = true>
__device__ __forceinline__ Trial<T> make_trial(const double* p, int model, double beta) {
  struct A : Arith<T> {
    static __device__ __forceinline__ T uni(T v) { return UNI ? Arith<T>::uni(v) : v; }
  };
  Trial<T> t;
  const T e1 = (T)p[2], e2 = (T)p[3];
  t.x0 = A::uni((T)p[0]);
  t.y0 = A::uni((T)p[1]);
  t.e1 = A::uni(e1);
  t.e2 = A::uni(e2);
  t.a11 = A::uni((T)1 - e1);
  t.a12 = A::uni(-e2);
  t.a22 = A::uni((T)1 + e1);
  t.invD = A::uni(A::rcp((T)(1.0 - p[2] * p[2] - p[3] * p[3])));
  t.I0 = A::uni((T)p[6]);
  t.sky = A::uni((T)p[7]);
  t.n11 = A::uni((T)(-((1.0 - p[2]) * (1.0 - p[2]) + p[3] * p[3])));
  t.n12 = A::uni((T)(2.0 * p[3]));
  t.n22 = A::uni((T)(-((1.0 + p[2]) * (1.0 + p[2]) + p[3] * p[3])));
  // FP32 instance: reciprocals by Newton from the hardware estimate, b(n) from
  // the FP32 series (its constants are rounded to FP32 in the end)
  constexpr bool kF32 = sizeof(T) == 4;
  const double D = 1.0 - p[2] * p[2] - p[3] * p[3];
  const double iD = kF32 ? rcp_f64(D) : 1.0 / D;
  {
    const double a11 = 1.0 - p[2], a12 = -p[3], a22 = 1.0 + p[2];
    const double qa = (a12 * a12 + a22 * a22) * iD;
    t.qa = A::uni((T)qa);
    t.qb1 = A::uni((T)(4.0 * a12 * iD));
    t.qc2 = A::uni((T)((a11 * a11 + a12 * a12) * iD));
    t.p2a = A::uni((T)(p[2] * qa + a22));
    t.p3a = A::uni((T)(p[3] * qa - a12));
  }
  const double I0 = p[6], twoinvD = 2.0 * iD;
  if (model == SHAPE_SERSIC) {
    const T n = (T)p[5], Re = (T)p[4];
    const T invn = A::rcp(n), l2Re = A::lg2(Re);
    const double in = kF32 ? rcp_f64(p[5]) : 1.0 / p[5];
    const double iRe = kF32 ? rcp_f64(p[4]) : 1.0 / p[4];
    double b, db;
    if constexpr (kF32) {
      float bf, dbf;
      sersic_bn_f32((float)p[5], (float)in, &bf, &dbf);
      b = bf;
      db = dbf;
    } else {
      sersic_bn(p[5], &b, &db);
    }
    t.ha = A::uni((T)0.5 * invn);
    t.hc = A::uni(-l2Re * invn);
    t.nb2 = A::uni((T)(-b * kLog2e));
    const double lnRe = kLn2 * (double)l2Re;
    t.k4 = A::uni((T)(I0 * b * in * iRe));
    t.k5a = A::uni((T)(I0 * b * in * in * 0.5 * kLn2));
    t.k5b = A::uni((T)(I0 * (-db - b * in * in * lnRe)));
    t.k7 = A::uni((T)(-I0 * b * 0.5 * in * twoinvD));
  } else {
    const double ird = kF32 ? rcp_f64(p[4]) : 1.0 / p[4];
    t.beta = A::uni((T)beta);
    t.irdsq = A::uni((T)(ird * ird));
    t.k4 = A::uni((T)(I0 * beta * 2.0 * ird * ird * ird));
    t.k5a = A::uni((T)(-I0 * kLn2));
    t.k7 = A::uni((T)(-I0 * beta * ird * ird * twoinvD));
  }
  return t;
}

// One sweep: model, residual, Jacobian columns in EM, and their sums.
// Pixel layouts of a sweep: kLayoutAny walks any side with the lane stride;
// kLayoutRows is for a wave alone on a stamp whose side divides 64 with at
// least 64 pixels (8, 16, 32, 64): every lane then keeps one column, steps
// 64 / side rows at a time, and the trip count is the same for all lanes.
constexpr int kLayoutAny = 0;
constexpr int kLayoutRows = 1;
// kLayoutStaged: any side, the stamp passed through an LDS buffer of
// kStageBytes in blocks (one burst of loads per block, so a sweep of a stamp
// that is not in the caches waits on memory once per block, not once per
// pixel); pixel order per lane and the partial-sum cadence are those of
// kLayoutAny, so the sums are the same bit for bit.
constexpr int kLayoutStaged = 2;
constexpr int kStageBytes = 8192;
// kLayoutSegs: a wave alone on a stamp of any side, the stamp cut into column
// segments of kSegRows rows (segment s: column s mod W, rows kSegRows (s / W)
// on), lane l taking segments l, l + 64, ...: along a segment u1 is fixed, so
// the geometry is the row layout's per-column quadratics, and a segment is
// one FP32 partial of the chi^2 and J^T r sums.  Sides up to 64 take the
// lane-stride walk: their segments fill the wave's last round less evenly
// (measured on the 48 x 48 workload: fit 6.2 ms in segments, 6.05 ms
// walking; on the uneven workload 82.2 ms with segments above side 64,
// 88.9 ms walking every stamp).
constexpr int kLayoutSegs = 3;
constexpr int kSegRows = 8;
constexpr int kSegsMinSide = 65;
// kLayoutSegsStaged: the same, with the smaller stamps' walk through the LDS
// buffer of kLayoutStaged (the same sums).
constexpr int kLayoutSegsStaged = 4;

__host__ __device__ inline constexpr bool rows_layout_fits(int side) {
  return side == 8 || side == 16 || side == 32 || side == 64;
}

// The layout of a wave alone on a stamp of batch b for the given model; the
// fused fit and the work queue's single waves take the same one, so their
// sums agree bit for bit: the row layout for a batch of one side that divides
// 64 (Sersic stamps of a batch without a model array), the lane-stride walk
// for a batch of one other side up to 64, column segments otherwise (a batch
// of mixed sides walks its stamps up to side 64).  A batch of one side up to
// 64 gets a kernel without the segment code: in a kernel that also holds it,
// the walk spills more and ran slower (48 x 48 fit 6.85 ms instead of 6.05).
inline int single_wave_layout(const shape_batch& b, int model) {
  if (!b.side) {
    if (model == SHAPE_SERSIC && !b.model && rows_layout_fits(b.side0)) return kLayoutRows;
    if (b.side0 <= kWave) return kLayoutAny;
  }
  return kLayoutSegs;
}

// Pixels of a lane whose chi^2 and J^T r terms the FP32 instance sums in FP32
// before carrying the partial sum on in FP64 (0: every term in FP64).  A
// partial of 8 terms rounds by about as much as the FP32 terms themselves.
#ifndef SHAPE_ROWS_PEEL
#define SHAPE_ROWS_PEEL 1
#endif
#ifndef SHAPE_SWEEP_FLUSH
#define SHAPE_SWEEP_FLUSH 8
#endif

// JTJ = false leaves the J^T J sums at zero (callers that need only chi^2
// and J^T r).
template <int DT, int MODEL, uint32_t EM, int STRIDE = kWave, typename T = float,
          int LAYOUT = kLayoutAny, bool JTJ = true>
__device__ __forceinline__ void sweep(const shape_batch& b, const Stamp& st, const Trial<T>& t,
                             Acc<EM, T>& acc, int tid = -1, void* stage = nullptr) {
  using A = Arith<T>;
  constexpr int kFlush = sizeof(T) == 4 ? SHAPE_SWEEP_FLUSH : 0;
  acc.c2 = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc.g[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 36; ++k) acc.A[k] = (T)0;
  T c2p = (T)0, gp[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) gp[k] = (T)0;
  // For the FP32 Sersic instance the constant factors k7 (of the x0, y0, e1,
  // e2 columns) and k4 (of the Re column) are applied to the sums once, after
  // the sweep.
  constexpr bool kFold = sizeof(T) == 4 && MODEL == SHAPE_SERSIC;
  // Moment form of the row layout (Sersic with x0, y0, e1, e2 free; the FP32
  // instance of the fit and the FP64 instance of the adjoint):
  // along a lane's column the four shape columns are h times polynomials in
  // u2 of degree 1, 1, 2, 2 with per-column coefficients, J_k = sum_j C_kj
  // h u2^j.  The lane therefore sums H_j = h u2^j (j = 0..2) against the
  // other quantities instead of the four columns: M_s = sum h^2 u2^s
  // (s = 0..4) for the 4 x 4 block, sum H_j v for v = J_Re, J_n, J_I0, 1 and
  // r, and forms the column sums from them once per sweep -- 22 VALU
  // operations per pixel where the columns cost 40.
  constexpr bool kMom = MODEL == SHAPE_SERSIC && LAYOUT == kLayoutRows && (EM & 0xFu) == 0xFu &&
                        (sizeof(T) == 8 || JTJ);
  constexpr int kMomN = kMom ? 3 : 1;
  T mM[2 * kMomN - 1], mX[3][kMomN], mY[kMomN], gq[kMomN];
  double gm[kMomN];
#pragma unroll
  for (int j = 0; j < kMomN; ++j) {
    mY[j] = gq[j] = (T)0;
    gm[j] = 0.0;
#pragma unroll
    for (int v = 0; v < 3; ++v) mX[v][j] = (T)0;
  }
#pragma unroll
  for (int s = 0; s < 2 * kMomN - 1; ++s) mM[s] = (T)0;
  auto flush = [&]() {
    if constexpr (kFlush > 0) {
      acc.c2 += (double)c2p;
      c2p = (T)0;
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        if (!has(EM, a) || (kMom && a < 4)) continue;
        acc.g[a] += (double)gp[a];
        gp[a] = (T)0;
      }
      if constexpr (kMom) {
#pragma unroll
        for (int j = 0; j < kMomN; ++j) {
          gm[j] += (double)gq[j];
          gq[j] = (T)0;
        }
      }
    }
  };
  // Per pixel: d = data, R2 = R^2 (unfloored), (n1, n2) = N u and the
  // e-derivative factors P2 = e1 R^2 + w_1, P3 = e2 R^2 + w_2.
  // first: the pixel opens a run of kFlush pixels, so its terms start the
  // FP32 partials instead of being added to them (the same values as adding
  // them to zeros; a compile-time constant where the runs are unrolled)
  auto pixel = [&](const T d, T R2, const T n1, const T n2, const T P2, const T P3,
                   const bool first = false) {
    const bool floored = R2 < A::kR2Floor;
    R2 = floored ? A::kR2Floor : R2;
    T J[8];
    T m0, h;
    if constexpr (MODEL == SHAPE_SERSIC) {
      const T L = A::lg2(R2);
      const T tt = A::ex2(A::fma(L, t.ha, t.hc));
      m0 = A::ex2(t.nb2 * tt);
      const T c = m0 * tt;
      if constexpr (kFold) {
        h = c * A::rcp(R2);
        if constexpr (has(EM, 4)) J[4] = c;
      } else {
        h = c * A::rcp(R2) * t.k7;
        if constexpr (has(EM, 4)) J[4] = c * t.k4;
      }
      if constexpr (has(EM, 5)) J[5] = c * A::fma(L, t.k5a, t.k5b);
    } else {
      const T base = A::fma(R2, t.irdsq, (T)1);
      const T lb = A::lg2(base);
      m0 = A::ex2(-t.beta * lb);
      const T c = m0 * A::rcp(base);
      h = c * t.k7;
      if constexpr (has(EM, 4)) J[4] = c * R2 * t.k4;
      if constexpr (has(EM, 5)) J[5] = m0 * lb * t.k5a;   // d/dbeta
    }
    h = floored ? (T)0 : h;
    const T r = d - A::fma(t.I0, m0, t.sky);
    if constexpr (has(EM, 0) || has(EM, 1)) {
      J[0] = h * n1;
      J[1] = h * n2;
    }
    if constexpr (has(EM, 2) || has(EM, 3)) {
      J[2] = h * P2;
      J[3] = h * P3;
    }
    J[6] = m0;
    J[7] = (T)1;
    const double rd = (double)r;
    if constexpr (kFlush > 0)
      c2p = first ? r * r : A::fma(r, r, c2p);
    else
      acc.c2 = fma(rd, rd, acc.c2);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (!has(EM, a)) continue;
      if constexpr (kFlush > 0)
        gp[a] = (a == 7) ? (first ? r : gp[a] + r) : (first ? J[a] * r : A::fma(J[a], r, gp[a]));
      else
        acc.g[a] = (a == 7) ? acc.g[a] + rd : fma((double)J[a], rd, acc.g[a]);
      if constexpr (JTJ) {
#pragma unroll
        for (int c = a; c < 8; ++c) {
          if (!has(EM, c)) continue;
          if (c == 7 && a == 7) continue;   // the count of pixels, set by the caller
          if (c == 7)
            acc.A[tri(a, c)] += J[a];
          else
            acc.A[tri(a, c)] = A::fma(J[a], J[c], acc.A[tri(a, c)]);
        }
      }
    }
  };
  // The moment form's pixel (kMom): the Sersic render as in pixel(), then the
  // H_j sums; the Re, n, I0 and sky columns are summed among themselves as
  // there.  The FP32 instance takes R^2 in units of Re^2, s = R^2 S with
  // S = 1 / Re^2 (2^(hc / ha)): then t = 2^(ha log2 s) needs no added
  // constant, and t / R^2 = S 2^((ha - 1) log2 s) gives h without a
  // reciprocal (one transcendental fewer per pixel; S goes into the folded
  // factor of the x0, y0, e1, e2 columns, log2 S into the n column's
  // constant).  The FP64 instance (the adjoint's; its exp2 costs more than
  // its reciprocal) renders as pixel() does, with the factors k7 and k4 in
  // the columns, and sums J^T J only when asked for.
  constexpr bool kF32Mom = kMom && sizeof(T) == 4;
  T mS = (T)1, mFloor = A::kR2Floor, mHam1 = (T)0, mK5b = (T)0;
  if constexpr (kF32Mom) {
    const T lS = A::uni(t.hc * A::rcp(t.ha));
    mS = A::uni(A::ex2(lS));
    mFloor = A::uni(A::kR2Floor * mS);
    mHam1 = A::uni(t.ha - (T)1);
    mK5b = A::uni(A::fma(-lS, t.k5a, t.k5b));
  }
  auto mom_pixel = [&](const T d, const T u2, T s2, const bool first) {
    const bool floored = s2 < mFloor;
    s2 = floored ? mFloor : s2;
    const T L = A::lg2(s2);
    T m0, c, h;
    if constexpr (kF32Mom) {
      const T tr = A::ex2(L * mHam1);   // t / s
      const T tt = tr * s2;
      m0 = A::ex2(t.nb2 * tt);
      c = m0 * tt;
      h = m0 * tr;                      // h / S
    } else {
      const T tt = A::ex2(A::fma(L, t.ha, t.hc));
      m0 = A::ex2(t.nb2 * tt);
      c = m0 * tt;
      h = c * A::rcp(s2) * t.k7;
    }
    h = floored ? (T)0 : h;
    T J[8];
    J[4] = kF32Mom ? c : c * t.k4;
    if constexpr (has(EM, 5)) J[5] = c * A::fma(L, t.k5a, kF32Mom ? mK5b : t.k5b);
    J[6] = m0;
    J[7] = (T)1;
    const T r = d - A::fma(t.I0, m0, t.sky);
    T H[kMomN];
    H[0] = h;
#pragma unroll
    for (int j = 1; j < kMomN; ++j) H[j] = H[j - 1] * u2;
    if constexpr (kFlush > 0) {
      c2p = first ? r * r : A::fma(r, r, c2p);
#pragma unroll
      for (int j = 0; j < kMomN; ++j) gq[j] = first ? H[j] * r : A::fma(H[j], r, gq[j]);
    } else {
      acc.c2 = fma((double)r, (double)r, acc.c2);
#pragma unroll
      for (int j = 0; j < kMomN; ++j) gm[j] = fma((double)H[j], (double)r, gm[j]);
    }
    if constexpr (JTJ) {
#pragma unroll
      for (int s = 0; s < 2 * kMomN - 1; ++s) {
        const int i = s < kMomN ? s : kMomN - 1, j = s - i;   // H_i H_j, i + j = s
        mM[s] = A::fma(H[i], H[j], mM[s]);
      }
    }
#pragma unroll
    for (int a = 4; a < 8; ++a) {
      if (!has(EM, a)) continue;
      if constexpr (kFlush > 0)
        gp[a] = (a == 7) ? (first ? r : gp[a] + r) : (first ? J[a] * r : A::fma(J[a], r, gp[a]));
      else
        acc.g[a] = (a == 7) ? acc.g[a] + (double)r : fma((double)J[a], (double)r, acc.g[a]);
      if constexpr (JTJ) {
#pragma unroll
        for (int j = 0; j < kMomN; ++j)
          if (a == 7)
            mY[j] += H[j];
          else
            mX[a - 4][j] = A::fma(H[j], J[a], mX[a - 4][j]);
#pragma unroll
        for (int c2 = a; c2 < 8; ++c2) {
          if (!has(EM, c2) || (c2 == 7 && a == 7)) continue;
          if (c2 == 7)
            acc.A[tri(a, c2)] += J[a];
          else
            acc.A[tri(a, c2)] = A::fma(J[a], J[c2], acc.A[tri(a, c2)]);
        }
      }
    }
  };
  if constexpr (LAYOUT == kLayoutRows) {
    static_assert(STRIDE == kWave, "the row layout is for a wave alone on its stamp");
    const int lane = tid < 0 ? (int)(threadIdx.x & (kWave - 1)) : tid;
    const int sd = st.side;                      // 8, 16, 32 or 64
    // the lane's column: u1 fixed, the quadratics' per-column coefficients
    const T u1 = (T)(lane & (sd - 1)) - t.x0;
    const T uu = u1 * u1;
    const T qb = t.qb1 * u1, qc = t.qc2 * uu;
    const T p2b = t.e1 * qb, p2c = A::fma(t.e1, qc, -t.a11 * uu);
    const T p3b = A::fma(t.e2, qb, (T)-2 * u1), p3c = A::fma(t.e2, qc, -t.a12 * uu);
    const T c3 = t.n11 * u1, c4 = t.n12 * u1;
    const T di = (T)(kWave / sd);
    T u2 = (T)(lane / sd) - t.y0;
    const int nstep = st.npix / kWave;
    const void* sp = stamp_base<DT>(b, st);
    uint32_t k = (uint32_t)lane;
    // FP32 stamps in memory, whole runs of kRun rows (sides 32 and 64): the
    // run is unrolled, so its loads issue together, and in the FP32 instance
    // its first pixel opens the partials (2 fewer VALU per pixel); measured
    // on 262,144 64 x 64 stamps: fit 23.1 -> 20.8 ms, 32 x 32 4-parameter fit
    // 3.72 -> 2.83 ms; FP64 chi^2 0.74 -> 0.72 ms, with J^T J 1.47 -> 1.33 ms
    // (65,536 stamps).  FP16 stamps staged in LDS ran 5% slower unrolled (4%
    // in the moment form: 18.1 vs 17.5 ms) and keep the loop, as does the
    // FP64 gradient without J^T J, whose five waves per SIMD leave the
    // unrolled run too few registers (136 spilled, 4x slower).
    constexpr int kRun = 8;
    static_assert(kFlush == 0 || kFlush == kRun, "a run is one partial-sum block");
    constexpr bool kUnroll = DT == SHAPE_F32 && (sizeof(T) == 4 || EM == 0u || JTJ);
    const bool blocked = kUnroll && nstep % kRun == 0;   // wave-uniform
    // R^2 S along the column (the moment form's units)
    const T qas = A::uni(t.qa * mS), qbs = qb * mS, qcs = qc * mS;
    auto row_pixel = [&](const T d, const T u2, const bool first) {
      if constexpr (kMom)
        mom_pixel(d, u2, A::fma(A::fma(qas, u2, qbs), u2, qcs), first);
      else
        pixel(d, A::fma(A::fma(t.qa, u2, qb), u2, qc), A::fma(t.n12, u2, c3),
              A::fma(t.n22, u2, c4), A::fma(A::fma(t.p2a, u2, p2b), u2, p2c),
              A::fma(A::fma(t.p3a, u2, p3b), u2, p3c), first);
    };
    if (blocked) {
#pragma unroll 1
      for (int m0 = 0; m0 < nstep; m0 += kRun) {
#pragma unroll
        for (int q = 0; q < kRun; ++q) {
          row_pixel((T)load_rel<DT>(sp, k + (uint32_t)(q * kWave), st.scale), u2, q == 0);
          u2 += di;
        }
        k += (uint32_t)(kRun * kWave);
        flush();
      }
    }
    // The moment form's loop in runs of kRun rows with the run's first pixel
    // peeled: it opens the FP32 partials, so a flush needs no zeroing.
    constexpr bool kPeel = SHAPE_ROWS_PEEL && kMom && kFlush == kRun;
    const bool peeled = kPeel && !blocked && nstep % kRun == 0;   // wave-uniform
    if (peeled) {
#pragma unroll 1
      for (int m0 = 0; m0 < nstep; m0 += kRun) {
        row_pixel((T)load_rel<DT>(sp, k, st.scale), u2, true);
        u2 += di;
        k += kWave;
#pragma unroll 1
        for (int q = 1; q < kRun; ++q) {
          row_pixel((T)load_rel<DT>(sp, k, st.scale), u2, false);
          u2 += di;
          k += kWave;
        }
        flush();
      }
    }
    if (!blocked && !peeled) {
#pragma unroll 1
      for (int m = 0; m < nstep; ++m) {
        row_pixel((T)load_rel<DT>(sp, k, st.scale), u2, false);
        u2 += di;
        k += kWave;
        if constexpr (kFlush > 0)
          if (m % kFlush == kFlush - 1) flush();   // m is wave-uniform
      }
    }
    if constexpr (kMom) {
      // the column sums from the moments, per lane, in FP64: column k is
      // h sum_j C[k][j] u2^j (degree 1 for x0, y0, 2 for e1, e2)
      flush();
      // the FP32 instance folds the factor k7 S of these columns (and k4 of
      // the Re column) in here, not into the sums afterwards
      const double f7 = kF32Mom ? (double)(t.k7 * mS) : 1.0;
      const double f4 = kF32Mom ? (double)t.k4 : 1.0;
      const double C[4][3] = {{c3 * f7, t.n12 * f7, 0.0},
                              {c4 * f7, t.n22 * f7, 0.0},
                              {p2c * f7, p2b * f7, t.p2a * f7},
                              {p3c * f7, p3b * f7, t.p3a * f7}};
      double M[5], X[3][3], Y[3];
#pragma unroll
      for (int s = 0; s < 5; ++s) M[s] = (double)mM[s];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        Y[j] = (double)mY[j];
#pragma unroll
        for (int v = 0; v < 3; ++v) X[v][j] = (double)mX[v][j] * (v == 0 ? f4 : 1.0);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int da = a < 2 ? 2 : 3;   // coefficients of column a
        double g = 0.0, y = 0.0, x[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < da; ++j) {
          g = fma(C[a][j], gm[j], g);
          y = fma(C[a][j], Y[j], y);
#pragma unroll
          for (int v = 0; v < 3; ++v) x[v] = fma(C[a][j], X[v][j], x[v]);
        }
        acc.g[a] = g;
        if constexpr (JTJ) {
          if (has(EM, 7)) acc.A[tri(a, 7)] = (T)y;
#pragma unroll
          for (int v = 0; v < 3; ++v)
            if (has(EM, 4 + v)) acc.A[tri(a, 4 + v)] = (T)x[v];
        }
      }
      // P[c][i] = sum_j C[c][j] M[i + j]; entry (a, c) = sum_i C[a][i] P[c][i]
      if constexpr (JTJ) {
        double P[4][3];
#pragma unroll
        for (int c2 = 0; c2 < 4; ++c2) {
          const int dc = c2 < 2 ? 2 : 3;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            double q = 0.0;
#pragma unroll
            for (int j = 0; j < dc; ++j) q = fma(C[c2][j], M[i + j], q);
            P[c2][i] = q;
          }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int da = a < 2 ? 2 : 3;
#pragma unroll
          for (int c2 = a; c2 < 4; ++c2) {
            double q = 0.0;
#pragma unroll
            for (int i = 0; i < da; ++i) q = fma(C[a][i], P[c2][i], q);
            acc.A[tri(a, c2)] = (T)q;
          }
        }
      }
    }
  } else {
    // the lane-stride walk (any side, any team), directly or through LDS
    auto any_walk = [&]() {
      int cnt = 0;
      // pixel (i, j) with value d, in the lane-stride order of for_pixels
      auto any_pixel = [&](const T d, int i, int j) {
        const T u1 = (T)j - t.x0, u2 = (T)i - t.y0;
        // (v1, v2) = S(e) u
        const T v1 = A::fma(t.a11, u1, t.a12 * u2), v2 = A::fma(t.a12, u1, t.a22 * u2);
        const T R2 = A::fma(v1, v1, v2 * v2) * t.invD;
        pixel(d, R2, A::fma(t.n11, u1, t.n12 * u2), A::fma(t.n12, u1, t.n22 * u2),
              A::fma(t.e1, R2, A::fma(v2, u2, -v1 * u1)), A::fma(t.e2, R2, -A::fma(v1, u2, v2 * u1)));
        if constexpr (kFlush > 0) {
          if (++cnt == kFlush) {
            flush();
            cnt = 0;
          }
        }
      };
      if constexpr (LAYOUT == kLayoutStaged || LAYOUT == kLayoutSegsStaged) {
        using E = typename std::conditional<DT == SHAPE_F32, float, _Float16>::type;
        constexpr int kBlk = kStageBytes / (int)sizeof(E);
        static_assert(kBlk % (STRIDE * (kFlush > 0 ? kFlush : 1)) == 0,
                      "blocks keep the partial-sum cadence");
        auto stage_sync = [] {
          if constexpr (STRIDE == kWave)
            wave_sync();
          else
            __syncthreads();
        };
        E* buf = static_cast<E*>(stage);
        const E* src = static_cast<const E*>(b.pixels) + st.off;
        const int side = st.side, npix = st.npix;
        const int t0 = tid < 0 ? (int)(threadIdx.x & (kWave - 1)) : tid;
        int i = t0 / side, j = t0 - i * side;
        const int di = STRIDE / side, dj = STRIDE - di * side;
        int k = t0;
#pragma unroll 1
        for (int k0 = 0; k0 < npix; k0 += kBlk) {
          const int nb = npix - k0 < kBlk ? npix - k0 : kBlk;
          stage_sync();   // the previous block's reads are done
#pragma unroll 8
          for (int q = t0; q < nb; q += STRIDE) buf[q] = src[k0 + q];
          stage_sync();
#pragma unroll 1
          for (; k < k0 + nb; k += STRIDE) {
            const E e = buf[k - k0];
            const T d = DT == SHAPE_F32 ? (T)(float)e : (T)((float)e * st.scale);
            any_pixel(d, i, j);
            i += di;
            j += dj;
            if (j >= side) {
              j -= side;
              ++i;
            }
          }
        }
      } else {
        for_pixels<STRIDE>(st.side, [&](int k, int i, int j) {
          any_pixel((T)load_px<DT>(b.pixels, st.off, k, st.scale), i, j);
        }, tid);
      }
  
    };
    if constexpr (LAYOUT == kLayoutSegs || LAYOUT == kLayoutSegsStaged) {
      static_assert(STRIDE == kWave, "the segment layout is for a wave alone on its stamp");
      if (st.side >= kSegsMinSide) {
        const int lane = tid < 0 ? (int)(threadIdx.x & (kWave - 1)) : tid;
        const int W = st.side, last = W - 1;
        const int S = W * ((W + kSegRows - 1) / kSegRows);   // segments
        const void* sp = stamp_base<DT>(b, st);
#pragma unroll 1
        for (int s0 = 0; s0 < S; s0 += kWave) {   // wave-uniform
          const int sg = s0 + lane;
          const bool on = sg < S;
          const int g = on ? sg / W : 0, j = on ? sg - g * W : 0, r0 = g * kSegRows;
          const T u1 = (T)j - t.x0;
          const T uu = u1 * u1;
          const T qb = t.qb1 * u1, qc = t.qc2 * uu;
          const T p2b = t.e1 * qb, p2c = A::fma(t.e1, qc, -t.a11 * uu);
          const T p3b = A::fma(t.e2, qb, (T)-2 * u1), p3c = A::fma(t.e2, qc, -t.a12 * uu);
          const T c3 = t.n11 * u1, c4 = t.n12 * u1;
          // the segment's pixels (rows past the stamp read its last row and are
          // skipped below), loaded back to back
          T d[kSegRows];
#pragma unroll
          for (int q = 0; q < kSegRows; ++q) {
            const int i = r0 + q < last ? r0 + q : last;
            d[q] = (T)load_rel<DT>(sp, (uint32_t)(i * W + j), st.scale);
          }
#pragma unroll
          for (int q = 0; q < kSegRows; ++q) {
            if (on && r0 + q < W) {
              const T u2 = (T)(r0 + q) - t.y0;
              pixel(d[q], A::fma(A::fma(t.qa, u2, qb), u2, qc), A::fma(t.n12, u2, c3),
                    A::fma(t.n22, u2, c4), A::fma(A::fma(t.p2a, u2, p2b), u2, p2c),
                    A::fma(A::fma(t.p3a, u2, p3b), u2, p3c));
            }
          }
          flush();   // one partial per segment
        }
      } else {
        any_walk();
      }
    } else {
      any_walk();
    }
  }
  flush();
  if constexpr (kFold) {
    // the folded constant factors: column a of J is s_a times what was summed
    // (the moment form folded them into its recombination, but for the
    // Re column's sums among the Re, n, I0 and sky columns)
    const T sc[8] = {t.k7, t.k7, t.k7, t.k7, t.k4, (T)1, (T)1, (T)1};
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      if (!has(EM, a) || (kMom && a < 4)) continue;
      acc.g[a] *= (double)sc[a];
#pragma unroll
      for (int c = a; c < 8; ++c)
        if (has(EM, c)) acc.A[tri(a, c)] *= sc[a] * sc[c];
    }
  }
}

// Reduce a sweep's per-lane partial sums over the wave and store them (FP64)
// at dst (entry k at dst[k * stride]): [0] = chi^2 sum, [1 + k] = (J^T r)_k,
// [9 + tri] = J^T J.  One
// quantity at a time by wave sums, with scheduling barriers, so the
// reductions do not all hold registers at once, and lane 0 stores.
//
// With six or more free parameters the sums are reduced by halving instead:
// v_permlane32_swap pairs entry j of the lower half-wave with entry j + 18 of
// the upper one (lanes 0-31 then carry entries 0..17 of the 36 J^T J sums,
// lanes 32-63 entries 18..35), v_permlane16_swap does the same between rows
// of 16 (row k then carries entries 9k..9k+8), and a row scan leaves each
// total in the row's last lane, which stores it: about 90 instructions for
// J^T J where one wave sum per entry takes about 360; the 9 FP64 sums go the
// same way (padded to 12, row k ends with entries 3k..3k+2).
template <uint32_t EM, typename T = float>
__device__ __forceinline__ void reduce_store(const Acc<EM, T>& acc, double* dst, int lane,
                                             int64_t stride = 1) {
  if constexpr (sizeof(T) == 4 && popcount(EM) >= 6) {
    // chi^2 and J^T r (FP64), padded to 12: after the two swaps row k holds
    // entries 3k..3k+2 (dst[0] = chi^2, dst[1 + a] = (J^T r)_a)
    double u[12];
    u[0] = acc.c2;
#pragma unroll
    for (int a = 0; a < 8; ++a) u[1 + a] = acc.g[a];   // unused entries are 0
    u[9] = u[10] = u[11] = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) swap_add32(u[j], u[j + 6]);
#pragma unroll
    for (int j = 0; j < 3; ++j) swap_add16(u[j], u[j + 3]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      u[j] = dpp::add<dpp::kShr1, 0xf>(u[j]);
      u[j] = dpp::add<dpp::kShr2, 0xf>(u[j]);
      u[j] = dpp::add<dpp::kShr4, 0xf>(u[j]);
      u[j] = dpp::add<dpp::kShr8, 0xf>(u[j]);
    }
    if ((lane & 15) == 15 && lane < 48) {
      const int base = 3 * (lane >> 4);
#pragma unroll
      for (int j = 0; j < 3; ++j) dst[(base + j) * stride] = u[j];
    }
    __builtin_amdgcn_sched_barrier(0);
    float v[36];
#pragma unroll
    for (int i = 0; i < 36; ++i) v[i] = acc.A[i];   // unused entries are 0
#pragma unroll
    for (int j = 0; j < 18; ++j) swap_add32(v[j], v[j + 18]);
#pragma unroll
    for (int j = 0; j < 9; ++j) swap_add16(v[j], v[j + 9]);
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      v[j] = dpp::add<dpp::kShr1, 0xf>(v[j]);
      v[j] = dpp::add<dpp::kShr2, 0xf>(v[j]);
      v[j] = dpp::add<dpp::kShr4, 0xf>(v[j]);
      v[j] = dpp::add<dpp::kShr8, 0xf>(v[j]);
    }
    if ((lane & 15) == 15) {
      const int base = 9 + 9 * (lane >> 4);
#pragma unroll
      for (int j = 0; j < 9; ++j) dst[(base + j) * stride] = (double)v[j];
    }
    return;
  }
  {
    const double v = wave_sum(acc.c2);
    if (lane == 0) dst[0] = v;
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if (has(EM, a)) {
      const double v = wave_sum(acc.g[a]);
      if (lane == 0) dst[(1 + a) * stride] = v;
    } else if (lane == 0) {
      dst[(1 + a) * stride] = 0.0;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = a; c < 8; ++c) {
      if (has(EM, a) && has(EM, c)) {
        const T v = wave_sum(acc.A[tri(a, c)]);
        if (lane == 0) dst[(9 + tri(a, c)) * stride] = (double)v;
      } else if (lane == 0) {
        dst[(9 + tri(a, c)) * stride] = 0.0;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

}  // namespace shape
