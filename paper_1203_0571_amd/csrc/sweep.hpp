// The per-pixel sweep shared by the fit and the chi^2 forward/backward
// kernels: render the model (Sec. 4.1 eq. ser, Sec. 4.2.2 eq. mof) at a set of
// parameters, form r = d - m and the Jacobian columns, and accumulate
// sum r^2, J^T r (FP64) and J^T J (FP32) over the stamp.
#pragma once

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

// Trial parameters as the FP32 sweep uses them.
struct TrialF {
  float x0, y0, e1, e2, a11, a12, a22, invD;
  float I0, sky;
  // Sersic: t = 2^(L ha + hc), m0 = 2^(nb2 t); Moffat: base = 1 + R^2 irdsq
  float ha, hc, nb2, b, hinvn, invnRe, ndb, invn2, nlnRe;
  float beta, irdsq, twoirdsq_rd;
};

template <uint32_t EM>
struct Acc {
  double c2;
  double g[8];
  float A[36];
};

__device__ __forceinline__ float uniform(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ TrialF make_trial(const double* p, int model, double beta) {
  // The sweep is FP32, so its constants are formed in FP32 from the FP64
  // parameters (hardware log2 / rcp, about 1 ulp).
  TrialF t;
  const float e1 = (float)p[2], e2 = (float)p[3];
  t.x0 = uniform((float)p[0]);
  t.y0 = uniform((float)p[1]);
  t.e1 = uniform(e1);
  t.e2 = uniform(e2);
  t.a11 = uniform(1.0f - e1);
  t.a12 = uniform(-e2);
  t.a22 = uniform(1.0f + e1);
  t.invD = uniform(fast_rcp((float)(1.0 - p[2] * p[2] - p[3] * p[3])));
  t.I0 = uniform((float)p[6]);
  t.sky = uniform((float)p[7]);
  if (model == SHAPE_SERSIC) {
    const float n = (float)p[5], Re = (float)p[4];
    const float invn = fast_rcp(n), l2Re = fast_log2(Re);
    double b, db;
    sersic_bn(p[5], &b, &db);
    t.ha = uniform(0.5f * invn);
    t.hc = uniform(-l2Re * invn);
    t.nb2 = uniform((float)(-b * kLog2e));
    t.b = uniform((float)b);
    t.hinvn = uniform(0.5f * invn);
    t.invnRe = uniform(invn * fast_rcp(Re));
    t.ndb = uniform((float)(-db));
    t.invn2 = uniform(invn * invn);
    t.nlnRe = uniform(-(float)kLn2 * l2Re);
  } else {
    const float rd = (float)p[4];
    const float ird = fast_rcp(rd);
    t.beta = uniform((float)beta);
    t.irdsq = uniform(ird * ird);
    t.twoirdsq_rd = uniform(2.0f * ird * ird * ird);
  }
  return t;
}

// One sweep: model, residual, Jacobian columns in EM, and their sums.
template <int DT, int MODEL, uint32_t EM, int STRIDE = kWave>
__device__ __forceinline__ void sweep(const shape_batch& b, const Stamp& st, const TrialF& t,
                             Acc<EM>& acc, int tid = -1) {
  acc.c2 = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc.g[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 36; ++k) acc.A[k] = 0.0f;
  for_pixels<STRIDE>(st.side, [&](int k, int i, int j) {
    const float d = load_px<DT>(b.pixels, st.off, k, st.scale);
    const float u1 = (float)j - t.x0, u2 = (float)i - t.y0;
    const float v1 = fmaf(t.a11, u1, t.a12 * u2);
    const float v2 = fmaf(t.a12, u1, t.a22 * u2);
    const float q = fmaf(v1, v1, v2 * v2);
    float R2 = q * t.invD;
    const bool floored = R2 < kR2Min;
    R2 = floored ? kR2Min : R2;
    float J[8];
    float m0, dmdR2;
    if constexpr (MODEL == SHAPE_SERSIC) {
      const float L = fast_log2(R2);
      const float tt = fast_exp2(fmaf(L, t.ha, t.hc));
      m0 = fast_exp2(t.nb2 * tt);
      const float w = t.I0 * m0;
      const float ct = w * t.b * tt;
      dmdR2 = -ct * fast_rcp(R2) * t.hinvn;
      if constexpr (has(EM, 4)) J[4] = ct * t.invnRe;
      if constexpr (has(EM, 5)) {
        const float lns = fmaf(L, (float)(0.5 * kLn2), t.nlnRe);
        J[5] = fmaf(w * tt, t.ndb, ct * lns * t.invn2);
      }
    } else {
      const float base = fmaf(R2, t.irdsq, 1.0f);
      const float lb = fast_log2(base);
      m0 = fast_exp2(-t.beta * lb);
      const float w = t.I0 * m0;
      const float gb = w * t.beta * fast_rcp(base);
      dmdR2 = -gb * t.irdsq;
      if constexpr (has(EM, 4)) J[4] = gb * R2 * t.twoirdsq_rd;
      if constexpr (has(EM, 5)) J[5] = -w * lb * (float)kLn2;   // d/dbeta
    }
    dmdR2 = floored ? 0.0f : dmdR2;
    const float r = d - fmaf(t.I0, m0, t.sky);
    if constexpr (has(EM, 0) || has(EM, 1)) {
      const float g2 = dmdR2 * (-2.0f * t.invD);
      J[0] = g2 * fmaf(t.a11, v1, t.a12 * v2);
      J[1] = g2 * fmaf(t.a12, v1, t.a22 * v2);
    }
    if constexpr (has(EM, 2) || has(EM, 3)) {
      const float ti = 2.0f * t.invD;
      const float qq = q * ti * t.invD;
      J[2] = dmdR2 * fmaf(ti, fmaf(v2, u2, -v1 * u1), t.e1 * qq);
      J[3] = dmdR2 * fmaf(ti, -fmaf(v1, u2, v2 * u1), t.e2 * qq);
    }
    J[6] = m0;
    J[7] = 1.0f;
    const double rd = (double)r;
    acc.c2 = fma(rd, rd, acc.c2);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (!has(EM, a)) continue;
      acc.g[a] = (a == 7) ? acc.g[a] + rd : fma((double)J[a], rd, acc.g[a]);
#pragma unroll
      for (int c = a; c < 8; ++c) {
        if (!has(EM, c)) continue;
        if (c == 7)
          acc.A[tri(a, c)] += J[a];
        else
          acc.A[tri(a, c)] = fmaf(J[a], J[c], acc.A[tri(a, c)]);
      }
    }
  }, tid);
}

// Reduce a sweep's per-lane partial sums over the wave and let lane 0 store
// them (FP64) at dst: [0] = chi^2 sum, [1 + k] = (J^T r)_k, [9 + tri] = J^T J.
// One quantity at a time, with scheduling barriers, so the reductions do not
// all hold registers at once.
template <uint32_t EM>
__device__ __forceinline__ void reduce_store(const Acc<EM>& acc, double* dst, int lane) {
  {
    const double v = wave_sum(acc.c2);
    if (lane == 0) dst[0] = v;
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if (has(EM, a)) {
      const double v = wave_sum(acc.g[a]);
      if (lane == 0) dst[1 + a] = v;
    } else if (lane == 0) {
      dst[1 + a] = 0.0;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = a; c < 8; ++c) {
      if (has(EM, a) && has(EM, c)) {
        const float v = wave_sum(acc.A[tri(a, c)]);
        if (lane == 0) dst[9 + tri(a, c)] = (double)v;
      } else if (lane == 0) {
        dst[9 + tri(a, c)] = 0.0;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

}  // namespace shape
