// Profile fit by Levenberg-Marquardt, one wave per stamp (Sec. 4.1: chi^2
// of eq. chi2 over the model of eq. ser, amplitudes from dchi2/dI0 = 0).
//
// Each LM trial is one sweep over the stamp that renders the model and its
// Jacobian at the trial shape with the current amplitudes (I0, sky) and
// accumulates sum r^2, J^T r (FP64) and J^T J (FP32), r = d - m.  Because the
// model is linear in (I0, sky) and every shape derivative is proportional to
// I0, the sums at the amplitude optimum of the trial shape follow exactly
// from the same sweep:
//   dl = A_LL^-1 g_L,  chi2* = chi2 - g_L . dl,  s = I0* / I0,
//   A*_NN = s^2 A_NN,  A*_NL = s A_NL,  g*_N = s (g_N - A_NL dl),  g*_L = 0.
// The step in the free shape parameters solves (M + lambda diag M) d = g*_N
// with M = A*_NN - A*_NL (A*_LL)^-1 A*_LN, in FP64, by Cholesky.  All lanes
// run the FP64 part redundantly on identical reduced sums.
#include "kernels.hpp"

namespace shape {
namespace {

constexpr uint32_t kMaskAll = 0xFFu;
constexpr uint32_t kMaskSize = 0xF0u;

__host__ __device__ constexpr int tri(int k, int l) {
  return k <= l ? k * 8 - k * (k - 1) / 2 + (l - k) : l * 8 - l * (l - 1) / 2 + (k - l);
}
// Parameters with a Jacobian column for a given model and free mask (beta is
// never fitted for Moffat stars).
__host__ __device__ constexpr uint32_t eff_mask(uint32_t mask, int model) {
  return model == SHAPE_MOFFAT ? (mask & ~(1u << 5)) : mask;
}
__host__ __device__ constexpr bool has(uint32_t m, int k) { return (m >> k) & 1u; }
__host__ __device__ constexpr int popcount(uint32_t m) { return m ? (int)(m & 1u) + popcount(m >> 1) : 0; }
// Index of the a-th set bit of m (a counted from 0); 0 when there is none.
__host__ __device__ constexpr int nth_bit(uint32_t m, int a) {
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

__device__ inline float uniform(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ inline TrialF make_trial(const double* p, int model, double beta) {
  TrialF t;
  const double e1 = p[2], e2 = p[3];
  const double D = 1.0 - e1 * e1 - e2 * e2;
  t.x0 = uniform((float)p[0]);
  t.y0 = uniform((float)p[1]);
  t.e1 = uniform((float)e1);
  t.e2 = uniform((float)e2);
  t.a11 = uniform((float)(1.0 - e1));
  t.a12 = uniform((float)(-e2));
  t.a22 = uniform((float)(1.0 + e1));
  t.invD = uniform((float)(1.0 / D));
  t.I0 = uniform((float)p[6]);
  t.sky = uniform((float)p[7]);
  if (model == SHAPE_SERSIC) {
    const double n = p[5], Re = p[4];
    double b, db;
    sersic_bn(n, &b, &db);
    t.ha = uniform((float)(0.5 / n));
    t.hc = uniform((float)(-log2(Re) / n));
    t.nb2 = uniform((float)(-b * kLog2e));
    t.b = uniform((float)b);
    t.hinvn = uniform((float)(0.5 / n));
    t.invnRe = uniform((float)(1.0 / (n * Re)));
    t.ndb = uniform((float)(-db));
    t.invn2 = uniform((float)(1.0 / (n * n)));
    t.nlnRe = uniform((float)(-log(Re)));
  } else {
    const double rd = p[4];
    t.beta = uniform((float)beta);
    t.irdsq = uniform((float)(1.0 / (rd * rd)));
    t.twoirdsq_rd = uniform((float)(2.0 / (rd * rd * rd)));
  }
  return t;
}

// One sweep: model, residual, Jacobian columns in EM, and their sums.
template <int DT, int MODEL, uint32_t EM>
__device__ inline void sweep(const shape_batch& b, const Stamp& st, const TrialF& t,
                             Acc<EM>& acc) {
  acc.c2 = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc.g[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 36; ++k) acc.A[k] = 0.0f;
  for_pixels(st.side, [&](int k, int i, int j) {
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
      m0 = fast_exp2(-t.beta * fast_log2(base));
      const float w = t.I0 * m0;
      const float gb = w * t.beta * fast_rcp(base);
      dmdR2 = -gb * t.irdsq;
      if constexpr (has(EM, 4)) J[4] = gb * R2 * t.twoirdsq_rd;
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
  });
  acc.c2 = wave_sum(acc.c2);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if (!has(EM, a)) continue;
    acc.g[a] = wave_sum(acc.g[a]);
#pragma unroll
    for (int c = a; c < 8; ++c)
      if (has(EM, c)) acc.A[tri(a, c)] = wave_sum(acc.A[tri(a, c)]);
  }
}

// Cholesky solve of the n x n SPD system (row-major M, in place); false if not SPD.
template <int NMAX>
__device__ inline bool chol_solve(int n, double (&M)[NMAX][NMAX], double (&x)[NMAX]) {
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    if (j >= n) break;
    double s = M[j][j];
#pragma unroll
    for (int l = 0; l < NMAX; ++l)
      if (l < j) s -= M[j][l] * M[j][l];
    if (!(s > 0.0)) return false;
    const double d = sqrt(s), id = 1.0 / d;
    M[j][j] = d;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i <= j || i >= n) continue;
      double v = M[i][j];
#pragma unroll
      for (int l = 0; l < NMAX; ++l)
        if (l < j) v -= M[i][l] * M[j][l];
      M[i][j] = v * id;
    }
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i >= n) break;
    double v = x[i];
#pragma unroll
    for (int l = 0; l < NMAX; ++l)
      if (l < i) v -= M[i][l] * x[l];
    x[i] = v / M[i][i];
  }
#pragma unroll
  for (int i = NMAX - 1; i >= 0; --i) {
    if (i >= n) continue;
    double v = x[i];
#pragma unroll
    for (int l = 0; l < NMAX; ++l)
      if (l > i && l < n) v -= M[l][i] * x[l];
    x[i] = v / M[i][i];
  }
  return true;
}

// Reduced sums of one sweep, FP64, in the wave's LDS:
//   [0] = sum r^2, [1 + k] = (J^T r)_k, [9 + tri(k, l)] = (J^T J)_kl.
constexpr int kSums = 45;
__host__ __device__ constexpr int sg(int k) { return 1 + k; }
__host__ __device__ constexpr int sa(int k, int l) { return 9 + tri(k, l); }

// Per-wave LM state in LDS (the workgroup is one wave).
struct LmShared {
  double sums[2][kSums];  // current point and last trial (swapped on accept)
};

// Lane 0 stores the (wave-uniform) reduced sums of a sweep.
template <uint32_t EM>
__device__ inline void store_sums(const Acc<EM>& acc, double* S, int npix) {
  if (threadIdx.x == 0) {
    S[0] = acc.c2;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      S[sg(a)] = has(EM, a) ? acc.g[a] : 0.0;
#pragma unroll
      for (int c = a; c < 8; ++c)
        S[sa(a, c)] = (has(EM, a) && has(EM, c)) ? (double)acc.A[tri(a, c)] : 0.0;
    }
    S[sa(7, 7)] = (double)npix;
  }
  __syncthreads();
}

// Move the sums of a sweep at amplitudes (I0, sky) to the amplitude optimum
// of the same shape (LIN = free amplitudes).  Returns false when the 1x1/2x2
// amplitude block is singular.  On return p[6], p[7] hold the new amplitudes.
// Every lane computes the same values; lane 0 writes them back.
template <uint32_t EM, uint32_t LIN>
__device__ inline bool profile_amplitudes(double* S, double* p) {
  double d6 = 0.0, d7 = 0.0;
  const double g6 = S[sg(6)], g7 = S[sg(7)];
  if constexpr (has(LIN, 6) && has(LIN, 7)) {
    const double a = S[sa(6, 6)], bq = S[sa(6, 7)], c = S[sa(7, 7)];
    const double det = a * c - bq * bq;
    if (!(det > 0.0)) return false;
    d6 = (c * g6 - bq * g7) / det;
    d7 = (a * g7 - bq * g6) / det;
  } else if constexpr (has(LIN, 6)) {
    if (!(S[sa(6, 6)] > 0.0)) return false;
    d6 = g6 / S[sa(6, 6)];
  } else if constexpr (has(LIN, 7)) {
    d7 = g7 / S[sa(7, 7)];
  }
  const double I0n = p[6] + d6;
  const double sc = I0n / p[6];
  if (threadIdx.x == 0) {  // in place, one lane: A_NL, g_N still hold the old values here
    S[0] -= g6 * d6 + g7 * d7;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      if (!has(EM, a)) continue;
      const double a6 = S[sa(a, 6)], a7 = S[sa(a, 7)];
      S[sg(a)] = sc * (S[sg(a)] - a6 * d6 - a7 * d7);
#pragma unroll
      for (int c = a; c < 6; ++c)
        if (has(EM, c)) S[sa(a, c)] *= sc * sc;
      S[sa(a, 6)] = a6 * sc;
      S[sa(a, 7)] = a7 * sc;
    }
    if constexpr (has(LIN, 6)) S[sg(6)] = 0.0;
    if constexpr (has(LIN, 7)) S[sg(7)] = 0.0;
  }
  __syncthreads();
  p[6] = I0n;
  p[7] += d7;
  return true;
}

template <int DT, int MODEL, uint32_t MASK>
__device__ void fit_stamp(const shape_batch& b, const KOpts& o, const Stamp& st, const float* p_init,
                          const float* rec, int64_t s, float* p_out, float* chi2_out,
                          float* perr, int32_t* iters, uint32_t* status, int32_t* sweeps,
                          LmShared& sh) {
  constexpr uint32_t EM = eff_mask(MASK, MODEL);
  constexpr uint32_t LIN = EM & 0xC0u;
  constexpr uint32_t NL = EM & 0x3Fu;      // free shape parameters
  constexpr int NN = popcount(NL);
  const int lane = threadIdx.x;
  const int W = st.side;

  // Starting point.
  double p[8];
  bool bad = false;
  if (p_init) {
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = p_init[s * 8 + k];
  } else {
    const float* r = rec + s * SHAPE_REC_LEN;
    p[0] = r[SHAPE_REC_X0];
    p[1] = r[SHAPE_REC_Y0];
    p[2] = r[SHAPE_REC_E1];
    p[3] = r[SHAPE_REC_E2];
    const double r50 = r[SHAPE_REC_R50];
    if (MODEL == SHAPE_SERSIC) {
      p[4] = r50;
      p[5] = o.n0;
    } else {
      p[4] = r50 / sqrt(exp2(1.0 / o.moffat_beta) - 1.0);
      p[5] = o.moffat_beta;
    }
    p[4] = fmin(fmax(p[4], 0.1), (double)W);
    p[6] = 1.0;
    p[7] = r[SHAPE_REC_SKY0];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) bad |= !__builtin_isfinite(p[k]);
  if (MODEL == SHAPE_MOFFAT) p[5] = o.moffat_beta;
  uint32_t stt = 0;
  if (bad) stt = SHAPE_ST_BAD_INPUT;

  // Linear start: the amplitude optimum at the starting shape (Sec. 4.1).
  bool nonfinite = false;
  if (!bad && LIN != 0u) {
    double q[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] = p[k];
    q[6] = 1.0;
    q[7] = 0.0;
    const TrialF t = make_trial(q, MODEL, o.moffat_beta);
    double sff = 0.0, sf = 0.0, sfd = 0.0, sd = 0.0;
    for_pixels(W, [&](int k, int i, int j) {
      const float d = load_px<DT>(b.pixels, st.off, k, st.scale);
      nonfinite |= !__builtin_isfinite(d);
      const float u1 = (float)j - t.x0, u2 = (float)i - t.y0;
      const float v1 = fmaf(t.a11, u1, t.a12 * u2);
      const float v2 = fmaf(t.a12, u1, t.a22 * u2);
      float R2 = fmaf(v1, v1, v2 * v2) * t.invD;
      R2 = R2 < kR2Min ? kR2Min : R2;
      float m0;
      if constexpr (MODEL == SHAPE_SERSIC) {
        const float tt = fast_exp2(fmaf(fast_log2(R2), t.ha, t.hc));
        m0 = fast_exp2(t.nb2 * tt);
      } else {
        m0 = fast_exp2(-t.beta * fast_log2(fmaf(R2, t.irdsq, 1.0f)));
      }
      const double f = m0, dd = d;
      sff = fma(f, f, sff);
      sf += f;
      sfd = fma(f, dd, sfd);
      sd += dd;
    });
    nonfinite = wave_any(nonfinite);
    sff = wave_sum(sff);
    sf = wave_sum(sf);
    sfd = wave_sum(sfd);
    sd = wave_sum(sd);
    const double np = st.npix;
    if constexpr (has(LIN, 6) && has(LIN, 7)) {
      const double det = sff * np - sf * sf;
      p[6] = (sfd * np - sf * sd) / det;
      p[7] = (sff * sd - sf * sfd) / det;
    } else if constexpr (has(LIN, 6)) {
      p[6] = (sfd - p[7] * sf) / sff;
    } else {
      p[7] = (sd - p[6] * sf) / np;
    }
  }
  if (nonfinite) stt = SHAPE_ST_NONFINITE_INPUT;
  if (!bad && !nonfinite && !(p[6] > 0.0)) stt |= SHAPE_ST_NONPOSITIVE_FLUX;

  int ci = 0;  // which LDS buffer holds the current point
  int it = 0, nsweep = 0;
  if (!bad && !nonfinite) {
    ++nsweep;
    {
      Acc<EM> acc;
      sweep<DT, MODEL, EM>(b, st, make_trial(p, MODEL, o.moffat_beta), acc);
      store_sums<EM>(acc, sh.sums[0], st.npix);
    }
    double lambda = o.lambda0;
    const double gmax2 = o.gmax * o.gmax;
    while (it < o.max_iter_lm) {
      const double* C = sh.sums[ci];
      // Schur complement of the amplitude block, damped.
      double M[NN][NN], x[NN];
      bool ok = true;
      {
        double L00 = 1.0, L01 = 0.0, L11 = 1.0, det = 1.0;
        if constexpr (has(LIN, 6) && has(LIN, 7)) {
          L00 = C[sa(6, 6)];
          L01 = C[sa(6, 7)];
          L11 = C[sa(7, 7)];
          det = L00 * L11 - L01 * L01;
          ok = det > 0.0;
        } else if constexpr (has(LIN, 6)) {
          L00 = C[sa(6, 6)];
          ok = L00 > 0.0;
        } else if constexpr (has(LIN, 7)) {
          L11 = C[sa(7, 7)];
          ok = L11 > 0.0;
        }
#pragma unroll
        for (int a = 0; a < NN; ++a) {
#pragma unroll
          for (int c = 0; c <= a; ++c) {
            const int ka = nth_bit(NL, a), kc = nth_bit(NL, c);
            double v = C[sa(ka, kc)];
            const double a6 = C[sa(ka, 6)], a7 = C[sa(ka, 7)];
            const double c6 = C[sa(kc, 6)], c7 = C[sa(kc, 7)];
            if constexpr (has(LIN, 6) && has(LIN, 7)) {
              v -= (a6 * (L11 * c6 - L01 * c7) + a7 * (L00 * c7 - L01 * c6)) / det;
            } else if constexpr (has(LIN, 6)) {
              v -= a6 * c6 / L00;
            } else if constexpr (has(LIN, 7)) {
              v -= a7 * c7 / L11;
            }
            M[a][c] = v;
          }
        }
#pragma unroll
        for (int a = 0; a < NN; ++a) {
          M[a][a] *= 1.0 + lambda;
          x[a] = C[sg(nth_bit(NL, a))];
        }
      }
      ++it;
      if (!ok || !chol_solve<NN>(NN, M, x)) {
        stt |= SHAPE_ST_SINGULAR;
        lambda *= 10.0;
        if (lambda > 1e10) {
          stt |= SHAPE_ST_STALLED;
          break;
        }
        continue;
      }
      double pt[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) pt[k] = p[k];
      const double scl[6] = {1.0, 1.0, 1.0, 1.0, p[4], p[5]};
      double smax = 0.0;
#pragma unroll
      for (int a = 0; a < NN; ++a) {
        pt[nth_bit(NL, a)] += x[a];
        smax = fmax(smax, fabs(x[a]) / scl[nth_bit(NL, a)]);
      }
      bool inside = pt[2] * pt[2] + pt[3] * pt[3] < gmax2 && pt[4] >= 0.1 && pt[4] <= (double)W &&
                    pt[6] > 0.0 && __builtin_isfinite(pt[0]) && __builtin_isfinite(pt[1]) &&
                    __builtin_isfinite(pt[7]);
      if (MODEL == SHAPE_SERSIC) inside = inside && pt[5] >= 0.2 && pt[5] <= 10.0;
      double* T = sh.sums[ci ^ 1];
      if (inside) {
        ++nsweep;
        {
          Acc<EM> acc;
          sweep<DT, MODEL, EM>(b, st, make_trial(pt, MODEL, o.moffat_beta), acc);
          store_sums<EM>(acc, T, st.npix);
        }
        if (LIN != 0u) {
          if (!profile_amplitudes<EM, LIN>(T, pt)) inside = false;
          inside = inside && pt[6] > 0.0 && __builtin_isfinite(pt[7]);
        }
      }
      if (!inside) {
        stt |= SHAPE_ST_AT_BOUND;
        lambda *= 10.0;
        if (lambda > 1e10) {
          stt |= SHAPE_ST_STALLED;
          break;
        }
        continue;
      }
      const double c2t = T[0];
      if (__builtin_isfinite(c2t) && c2t <= sh.sums[ci][0] * (1.0 + o.chi2_rtol)) {
#pragma unroll
        for (int k = 0; k < 8; ++k) p[k] = pt[k];
        ci ^= 1;
        lambda = fmax(lambda * 0.1, 1e-9);
        if (smax < o.tol_lm) {
          stt |= SHAPE_ST_CONVERGED;
          break;
        }
      } else {
        lambda *= 10.0;
        if (lambda > 1e10) {
          stt |= SHAPE_ST_STALLED;
          break;
        }
      }
    }
    if (!(stt & (SHAPE_ST_CONVERGED | SHAPE_ST_STALLED))) stt |= SHAPE_ST_MAX_ITER;
  }

  const bool valid = !(stt & (SHAPE_ST_BAD_INPUT | SHAPE_ST_NONFINITE_INPUT));
  const double* C = sh.sums[ci];
  if (perr) {
    // sqrt(diag((J^T J / sigma^2)^-1)) over the fitted parameters: one
    // Cholesky factorisation, then lane c < NF solves for unit vector c.
    constexpr uint32_t FM = NL | LIN;
    constexpr int NF = popcount(FM);
    double e = valid ? 0.0 : (double)qnan();
    if (valid) {
      double Lf[NF][NF];
      bool okf = true;
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        double sjj = C[sa(nth_bit(FM, j), nth_bit(FM, j))];
#pragma unroll
        for (int l = 0; l < j; ++l) sjj -= Lf[j][l] * Lf[j][l];
        okf = okf && sjj > 0.0;
        const double d = sqrt(fmax(sjj, 1e-300));
        Lf[j][j] = d;
#pragma unroll
        for (int i = j + 1; i < NF; ++i) {
          double v = C[sa(nth_bit(FM, i), nth_bit(FM, j))];
#pragma unroll
          for (int l = 0; l < j; ++l) v -= Lf[i][l] * Lf[j][l];
          Lf[i][j] = v / d;
        }
      }
      double xf[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        double v = (i == lane) ? 1.0 : 0.0;
#pragma unroll
        for (int l = 0; l < i; ++l) v -= Lf[i][l] * xf[l];
        xf[i] = v / Lf[i][i];
      }
#pragma unroll
      for (int i = NF - 1; i >= 0; --i) {
        double v = xf[i];
#pragma unroll
        for (int l = i + 1; l < NF; ++l) v -= Lf[l][i] * xf[l];
        xf[i] = v / Lf[i][i];
      }
      double diag = 0.0;
#pragma unroll
      for (int i = 0; i < NF; ++i)
        if (i == lane) diag = xf[i];
      e = okf ? st.sigma * sqrt(diag) : (double)qnan();
    }
    // lane c holds the error of the c-th fitted parameter; scatter to slots
    if (lane < 8) {
      double v = valid ? 0.0 : (double)qnan();
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        const double ec = __shfl(e, c, kWave);
        if (lane == nth_bit(FM, c)) v = ec;
      }
      perr[s * 8 + lane] = (float)v;
    } else {
#pragma unroll
      for (int c = 0; c < NF; ++c) (void)__shfl(e, c, kWave);
    }
  }
  if (lane < 8) {
    double v = p[0];
#pragma unroll
    for (int k = 1; k < 8; ++k)
      if (lane == k) v = p[k];
    p_out[s * 8 + lane] = valid ? (float)v : qnan();
  }
  if (lane == 0) {
    chi2_out[s] = valid ? (float)(C[0] / (st.sigma * st.sigma)) : qnan();
    iters[s] = it;
    status[s] = stt;
    if (sweeps) sweeps[s] = nsweep;
  }
  __syncthreads();  // the LDS state is reused by the next stamp of this wave
}

template <int DT, int MODEL, uint32_t MASK>
__global__ __launch_bounds__(kWave) void fit_kernel(shape_batch b, KOpts o, const float* p_init,
                                                    const float* rec, float* p_out, float* chi2,
                                                    float* perr, int32_t* iters, uint32_t* status,
                                                    int32_t* sweeps) {
  __shared__ LmShared sh;
  for (int64_t s = blockIdx.x; s < b.n; s += gridDim.x) {
    const Stamp st = stamp_info(b, s);
    if (!st.bad && st.model != MODEL) continue;  // the other model's kernel owns it
    if (st.bad) {
      if (MODEL != SHAPE_SERSIC) continue;       // reported once, by the Sersic kernel
      const int lane = threadIdx.x;
      if (lane < 8) {
        p_out[s * 8 + lane] = qnan();
        if (perr) perr[s * 8 + lane] = qnan();
      }
      if (lane == 0) {
        chi2[s] = qnan();
        iters[s] = 0;
        status[s] = st.bad;
        if (sweeps) sweeps[s] = 0;
      }
      continue;
    }
    fit_stamp<DT, MODEL, MASK>(b, o, st, p_init, rec, s, p_out, chi2, perr, iters, status, sweeps,
                               sh);
  }
}

template <int DT, int MODEL>
void launch_fit_model(const shape_batch& b, const KOpts& o, const float* p_init,
                      const float* rec, float* p_out, float* chi2, float* perr, int32_t* iters,
                      uint32_t* status, int32_t* sweeps, hipStream_t stream) {
  const int64_t grid = b.n < (1ll << 30) ? b.n : (1ll << 30);
  if (o.free_mask == kMaskAll)
    hipLaunchKernelGGL((fit_kernel<DT, MODEL, kMaskAll>), dim3((unsigned)grid), dim3(kWave), 0,
                       stream, b, o, p_init, rec, p_out, chi2, perr, iters, status, sweeps);
  else
    hipLaunchKernelGGL((fit_kernel<DT, MODEL, kMaskSize>), dim3((unsigned)grid), dim3(kWave), 0,
                       stream, b, o, p_init, rec, p_out, chi2, perr, iters, status, sweeps);
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
