// Levenberg-Marquardt profile fit of one stamp, in pieces shared by the fused
// fit kernel (start, iterate until done, finish) and the persistent work-queue
// kernels (start; one iteration per launch with the state in HBM; finish).
//
// Sec. 4.1: chi^2 (eq. chi2) of the model (eq. ser; eq. mof for stars) over
// the free parameters, the amplitudes following from dchi2/dI0 = 0.
//
// Each trial is one sweep that renders the model and its Jacobian at the
// trial shape with the current amplitudes (I0, sky) and accumulates sum r^2,
// J^T r (FP64) and J^T J (FP32), r = d - m.  The model is linear in (I0, sky)
// and every shape derivative is proportional to I0, so the sums at the
// amplitude optimum of the trial shape follow from the same sweep:
//   dl = A_LL^-1 g_L,  chi2* = chi2 - g_L . dl,  s = I0* / I0,
//   A*_NN = s^2 A_NN,  A*_NL = s A_NL,  g*_N = s (g_N - A_NL dl),  g*_L = 0.
// The step in the free shape parameters solves (M + lambda diag M) d = g*_N,
// M = A*_NN - A*_NL (A*_LL)^-1 A*_LN, in FP64 by an L D L^T factorisation
// (the entries of M formed one per thread into LDS, the factorisation and
// solve in one thread), from the reduced sums kept in LDS.
#pragma once

#include "sweep.hpp"

namespace shape {

constexpr uint32_t kMaskAll = 0xFFu;
constexpr uint32_t kMaskSize = 0xF0u;

// Reduced sums of one sweep, FP64:
//   [0] = sum r^2, [1 + k] = (J^T r)_k, [9 + tri(k, l)] = (J^T J)_kl.
constexpr int kSums = 45;
__host__ __device__ inline constexpr int sg(int k) { return 1 + k; }
__host__ __device__ inline constexpr int sa(int k, int l) { return 9 + tri(k, l); }

// Uniform LM state of one stamp.
struct LmState {
  double p[8];
  double lambda;
  int it;
  int nsweep;
  uint32_t stt;
  int done;
};

// The LDS block one team works in: the current point's and the last trial's
// sums, the LM state and the trial point.  Keeping the state here (not in
// registers) while a sweep runs leaves the sweep all of the register file.
struct LmShared {
  double sums[2][kSums];
  LmState L;
  double pt[8];
  double smax;   // the trial step's max_k |d_k| / s_k (-1: no sweep for it)
  double M[21];  // damped Schur complement, lower triangle row by row
  int cur;       // which of sums[] holds the current point
};

template <int TEAM>
__device__ __forceinline__ void team_sync();

// State updates: every thread computes the same values; thread 0 stores them.
template <int TEAM>
__device__ __forceinline__ void store_L(LmShared& W, const LmState& L, int tid) {
  team_sync<TEAM>();
  if (tid == 0) W.L = L;
  team_sync<TEAM>();
}
__device__ __forceinline__ LmState load_L(const LmShared& W) { return W.L; }

// Solves the SPD system m x = b in one thread, m given as its lower triangle
// row by row (m[i (i + 1) / 2 + j], j <= i), by the factorisation
// m = L D L^T (L unit lower triangular, D diagonal): no square roots, one
// reciprocal per pivot, about 120 FP64 operations for six unknowns.  x holds
// b on entry and the solution on exit.  Returns false if a pivot is not
// positive (x is then meaningless).  The fused fit and the batched form call
// it on the same damped system, so both take the same step bit for bit.
template <int N>
__device__ __forceinline__ bool ldl_solve(const double (&m)[N * (N + 1) / 2], double (&x)[N]) {
  double L[N][N];   // the strictly lower part is used
  double id[N];     // 1 / D
  bool ok = true;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double u[N];    // u_k = L_jk D_k
#pragma unroll
    for (int k = 0; k < j; ++k) {
      double w = m[j * (j + 1) / 2 + k];
#pragma unroll
      for (int l = 0; l < k; ++l) w = fma(-u[l], L[k][l], w);
      u[k] = w;
      L[j][k] = w * id[k];
    }
    double d = m[j * (j + 1) / 2 + j];
#pragma unroll
    for (int k = 0; k < j; ++k) d = fma(-u[k], L[j][k], d);
    ok = ok && d > 0.0;
    id[j] = rcp_f64(d);
  }
  // L y = b, z = D^-1 y, L^T x = z
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < i; ++k) x[i] = fma(-L[i][k], x[k], x[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] *= id[i];
#pragma unroll
  for (int i = N - 1; i >= 0; --i)
#pragma unroll
    for (int k = i + 1; k < N; ++k) x[i] = fma(-L[k][i], x[k], x[i]);
  return ok;
}

// Synchronise a team of TEAM waves (a lone wave needs no barrier).
template <int TEAM>
__device__ __forceinline__ void team_sync() {
  if constexpr (TEAM == 1)
    wave_sync();
  else
    __syncthreads();
}

// One sweep at trial t; the team's reduced sums are left in S (kSums doubles,
// entry k at S[k * stride]: LDS for the fused fit, the stamp's column of the
// workspace for the batched form).  xs is LDS scratch of TEAM * kSums doubles
// for the cross-wave combination (unused for TEAM == 1).  tid = thread index
// within the team; stage: the LDS buffer of kLayoutStaged (kStageBytes).
template <int DT, int MODEL, uint32_t EM, int TEAM, int LAYOUT = kLayoutAny>
__device__ __forceinline__ void sweep_sums(const shape_batch& b, const Stamp& st, const TrialF& t,
                                           double* S, double* xs, int tid, int64_t stride = 1,
                                           void* stage = nullptr) {
  Acc<EM> acc;
  sweep<DT, MODEL, EM, kWave * TEAM, float, LAYOUT>(b, st, t, acc, tid, stage);
  const int lane = tid & (kWave - 1);
  team_sync<TEAM>();  // previous readers of S / xs are done
  if constexpr (TEAM == 1) {
    reduce_store<EM>(acc, S, lane, stride);
  } else {
    reduce_store<EM>(acc, xs + (tid / kWave) * kSums, lane);
  }
  team_sync<TEAM>();
  if constexpr (TEAM > 1) {
    if (tid < kSums) {
      double v = xs[tid];
#pragma unroll
      for (int w = 1; w < TEAM; ++w) v += xs[w * kSums + tid];
      S[tid * stride] = v;
    }
    team_sync<TEAM>();
  }
  if (tid == 0) S[sa(7, 7) * stride] = (double)st.npix;
  team_sync<TEAM>();
}

// Per-stamp arithmetic of one LM trial, lane-local: the fused kernel runs it
// on one thread of the team (on the sums in LDS), the batched form on one lane
// per stamp; both call these same routines, so both forms compute the same
// values.

// The free amplitudes (LIN: bit 6 = I0, bit 7 = sky) from sums S taken at
// amplitudes (I0, sky): ok = false when the amplitude block is singular,
// otherwise (d6, d7) are the amplitude changes.
struct AmpStep {
  bool ok;
  double d6, d7;
};
template <uint32_t LIN>
__device__ __forceinline__ AmpStep amp_solve(const double* S) {
  AmpStep r{true, 0.0, 0.0};
  const double g6 = S[sg(6)], g7 = S[sg(7)];
  if constexpr (has(LIN, 6) && has(LIN, 7)) {
    const double a = S[sa(6, 6)], bq = S[sa(6, 7)], c = S[sa(7, 7)];
    const double det = a * c - bq * bq;
    if (!(det > 0.0)) return AmpStep{false, 0.0, 0.0};
    const double idet = rcp_f64(det);
    r.d6 = (c * g6 - bq * g7) * idet;
    r.d7 = (a * g7 - bq * g6) * idet;
  } else if constexpr (has(LIN, 6)) {
    if (!(S[sa(6, 6)] > 0.0)) return AmpStep{false, 0.0, 0.0};
    r.d6 = g6 / S[sa(6, 6)];
  } else if constexpr (has(LIN, 7)) {
    r.d7 = g7 / S[sa(7, 7)];
  }
  return r;
}

// Move the sums S (taken at amplitude I0 > 0) to the amplitude optimum r, in
// place (A_NL and g_N still hold the old values while they are read).
template <uint32_t EM, uint32_t LIN>
__device__ __forceinline__ void amp_apply(double* S, const AmpStep& r, double I0) {
  const double g6 = S[sg(6)], g7 = S[sg(7)];
  const double d6 = r.d6, d7 = r.d7;
  const double sc = (I0 + d6) * rcp_f64(I0);
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

// The team form: every thread solves, thread 0 rewrites S (in LDS).
template <uint32_t EM, uint32_t LIN, int TEAM>
__device__ __forceinline__ AmpStep profile_amplitudes(double* S, double I0, int tid) {
  const AmpStep r = amp_solve<LIN>(S);
  if (!r.ok) return r;
  team_sync<TEAM>();
  if (tid == 0) amp_apply<EM, LIN>(S, r, I0);
  team_sync<TEAM>();
  return r;
}

// Entry (ka, kc) of the Schur complement of the amplitude block (undamped):
//   M_ac = A_ac - A_aL (A_LL)^-1 A_Lc = A_ac - u_a A_c6 - w_a A_c7.
template <uint32_t LIN>
__device__ __forceinline__ double schur_entry(const double* C, int ka, int kc) {
  double v = C[sa(ka, kc)];
  if constexpr (has(LIN, 6) && has(LIN, 7)) {
    const double L00 = C[sa(6, 6)], L01 = C[sa(6, 7)], L11 = C[sa(7, 7)];
    const double idet = rcp_f64(L00 * L11 - L01 * L01);   // (not positive: the solve fails)
    const double a6 = C[sa(ka, 6)], a7 = C[sa(ka, 7)];
    const double u = (L11 * a6 - L01 * a7) * idet, w = (L00 * a7 - L01 * a6) * idet;
    v -= u * C[sa(kc, 6)] + w * C[sa(kc, 7)];
  } else if constexpr (has(LIN, 6)) {
    v -= C[sa(ka, 6)] * C[sa(kc, 6)] / C[sa(6, 6)];
  } else if constexpr (has(LIN, 7)) {
    v -= C[sa(ka, 7)] * C[sa(kc, 7)] / C[sa(7, 7)];
  }
  return v;
}

// The starting point: p from p_init or the moments record (x0, y0, e1, e2 of
// the moments; Re = the record's size, or r50 where it is undefined; Moffat
// rd from r50 and beta; n = n0; I0 = 1, sky = sky0), and the fresh state.
template <int MODEL>
__device__ __forceinline__ LmState start_point(const KOpts& o, const Stamp& st, const float* p_init,
                                               const float* rec, int64_t s) {
  LmState L;
  double* p = L.p;
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
      const double size = r[SHAPE_REC_SIZE];
      p[4] = __builtin_isfinite(size) ? size : r50;
      p[5] = o.n0;
    } else {
      // the Moffat of half-light radius r50 (beta > 1: the enclosed flux is
      // 1 - (1 + R^2 / rd^2)^(1 - beta) of the total)
      p[4] = r50 / sqrt(exp2(1.0 / (o.moffat_beta - 1.0)) - 1.0);
      p[5] = o.moffat_beta;
    }
    p[4] = fmin(fmax(p[4], 0.1), (double)st.side);
    p[6] = 1.0;
    p[7] = r[SHAPE_REC_SKY0];
  }
  if (MODEL == SHAPE_MOFFAT) p[5] = o.moffat_beta;
  L.lambda = o.lambda0;
  L.it = 0;
  L.nsweep = 0;
  L.stt = 0;
  L.done = 0;
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) finite = finite && __builtin_isfinite(p[k]);
  if (!finite) {
    L.stt = SHAPE_ST_BAD_INPUT;
    L.done = 1;
  }
  return L;
}

// What a trial's decision needs of the current point's sums C besides the
// damped system: the right-hand side g_N of the step and the amplitude block.
template <int NN>
struct StepRhs {
  double g[NN];
  double l66, l67, l77;
};
template <uint32_t NL, int NN>
__device__ __forceinline__ StepRhs<NN> step_rhs(const double* C) {
  StepRhs<NN> r;
#pragma unroll
  for (int a = 0; a < NN; ++a) r.g[a] = C[sg(nth_bit(NL, a))];
  r.l66 = C[sa(6, 6)];
  r.l67 = C[sa(6, 7)];
  r.l77 = C[sa(7, 7)];
  return r;
}

// After the solve of the damped step x (solved: the elimination succeeded):
// counts the trial, forms the trial point pt and decides.  Returns the step's
// max_k |x_k| / s_k when the trial needs a sweep, -1 when it does not (the
// fit converged on a small Gauss-Newton step, or the trial left the box and is
// rejected).  R holds the current point's right-hand side and amplitude block.
template <int MODEL, uint32_t NL, uint32_t LIN, int NN>
__device__ __forceinline__ double lm_propose(LmState& L, const StepRhs<NN>& R,
                                             const double (&x)[NN], bool solved, const KOpts& o,
                                             const Stamp& st, double* ptout) {
  bool ok = solved;
  if constexpr (has(LIN, 6) && has(LIN, 7))
    ok = ok && R.l66 * R.l77 - R.l67 * R.l67 > 0.0;
  else if constexpr (has(LIN, 6))
    ok = ok && R.l66 > 0.0;
  else if constexpr (has(LIN, 7))
    ok = ok && R.l77 > 0.0;
  ++L.it;
  bool inside = false;
  double smax = 0.0, q = 0.0;   // q = d^T A_lambda d = d^T g
#pragma unroll
  for (int k = 0; k < 8; ++k) ptout[k] = L.p[k];
  if (!ok) {
    L.stt |= SHAPE_ST_SINGULAR;
  } else {
    double pt[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) pt[k] = L.p[k];
    // (the scales only feed the stopping test: FP32 reciprocals)
    const double iscl[8] = {1.0, 1.0, 1.0, 1.0, (double)fast_rcp((float)L.p[4]),
                            (double)fast_rcp((float)L.p[5]), (double)fast_rcp(fabsf((float)L.p[6])),
                            (double)fast_rcp((float)st.sigma)};
#pragma unroll
    for (int a = 0; a < NN; ++a) {
      pt[nth_bit(NL, a)] += x[a];
      smax = fmax(smax, fabs(x[a]) * iscl[nth_bit(NL, a)]);
      q += x[a] * R.g[a];
    }
    const double gmax2 = o.gmax * o.gmax;
    inside = pt[2] * pt[2] + pt[3] * pt[3] < gmax2 && pt[4] >= 0.1 &&
             pt[4] <= (double)st.side && pt[6] > 0.0 && __builtin_isfinite(pt[0]) &&
             __builtin_isfinite(pt[1]) && __builtin_isfinite(pt[7]);
    if (MODEL == SHAPE_SERSIC) inside = inside && pt[5] >= 0.2 && pt[5] <= 10.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) ptout[k] = pt[k];
  }
  // At small damping the step is the Gauss-Newton step from the current
  // point; when it is already below the tolerances (max_k |d_k| / s_k <
  // tol_lm, or d^T A_lambda d = d^T g below tol_sigma^2 sigma^2: d^T A d /
  // sigma^2 bounds (d_k / sigma_k)^2 for every k and A_lambda >= A, so every
  // parameter would move by less than tol_sigma standard errors) the current
  // point is the result and the trial needs no sweep.
  const double sig2 = st.sigma * st.sigma;
  const bool small_step = inside && L.lambda <= 1e-3 &&
                          (smax < o.tol_lm || q < o.tol_sigma * o.tol_sigma * sig2);
  if (small_step) {
    L.stt |= SHAPE_ST_CONVERGED;
    L.done = 1;
    return -1.0;  // no sweep for this trial
  }
  if (!inside) {  // rejected before any sweep
    L.lambda *= 10.0;
    if (L.lambda > 1e10) {
      L.stt |= SHAPE_ST_STALLED;
      L.done = 1;
    }
    return -1.0;  // no sweep for this trial
  }
  ++L.nsweep;
  return smax;
}

// The verdict on a swept trial: pt is the trial point with the amplitudes of
// its sweep (a: their optimum at the trial shape, when LIN != 0), c2t the
// trial's profiled chi^2 sum and c2c the current point's.  Accepts (L.p = pt,
// less damping, converged on a step below tol_lm) or rejects (more damping,
// stalled above 1e10).  Returns whether the trial was accepted.
template <uint32_t LIN>
__device__ __forceinline__ bool lm_judge(LmState& L, double* pt, const AmpStep& a, double smax,
                                         double c2t, double c2c, const KOpts& o) {
  bool inside = true;
  if (LIN != 0u) {
    pt[6] += a.d6;
    pt[7] += a.d7;
    inside = a.ok && pt[6] > 0.0 && __builtin_isfinite(pt[7]);
  }
  bool accepted = false;
  if (!inside) {
    L.lambda *= 10.0;
    if (L.lambda > 1e10) {
      L.stt |= SHAPE_ST_STALLED;
      L.done = 1;
    }
  } else if (__builtin_isfinite(c2t) && c2t <= c2c * (1.0 + o.chi2_rtol)) {
#pragma unroll
    for (int k = 0; k < 8; ++k) L.p[k] = pt[k];
    accepted = true;
    L.lambda = fmax(L.lambda * 0.1, 1e-9);
    if (smax < o.tol_lm) {   // a short step taken at larger damping
      L.stt |= SHAPE_ST_CONVERGED;
      L.done = 1;
    }
  } else {
    L.lambda *= 10.0;
    if (L.lambda > 1e10) {
      L.stt |= SHAPE_ST_STALLED;
      L.done = 1;
    }
  }
  return accepted;
}

// Starting point: p from p_init or the moments record, the amplitude optimum
// at that shape (Sec. 4.1) and the first sweep, whose profiled sums become the
// current point (W.sums[W.cur]).  The state ends in W.L.
template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT = kLayoutAny>
__device__ __forceinline__ void lm_start(const shape_batch& b, const KOpts& o, const Stamp& st,
                                         const float* p_init, const float* rec, int64_t s,
                                         LmShared& W, double* xs, int tid) {
  constexpr uint32_t EM = eff_mask(MASK, MODEL);
  constexpr uint32_t LIN = EM & 0xC0u;
  LmState L = start_point<MODEL>(o, st, p_init, rec, s);
  double* p = L.p;
  if (tid == 0) W.cur = 0;
  double* C = W.sums[0];
  // Linear start: the free amplitudes' optimum at the starting shape, from one
  // sweep at unit amplitude / zero sky (exact: the model is linear in them).
  if constexpr (LIN != 0u) {
    if (!L.done) {
      if (has(LIN, 6)) p[6] = 1.0;
      if (has(LIN, 7)) p[7] = 0.0;
      store_L<TEAM>(W, L, tid);
      sweep_sums<DT, MODEL, LIN, TEAM, LAYOUT>(b, st, make_trial(W.L.p, MODEL, o.moffat_beta), C, xs,
                                               tid);
      L = load_L(W);
      if (!__builtin_isfinite(C[0])) {
        L.stt = SHAPE_ST_NONFINITE_INPUT;
        L.done = 1;
      } else {
        const AmpStep a = profile_amplitudes<LIN, LIN, TEAM>(C, p[6], tid);
        if (!a.ok) L.stt |= SHAPE_ST_SINGULAR;
        p[6] += a.d6;
        p[7] += a.d7;
      }
    }
  }
  if (!L.done) {
    if (!(p[6] > 0.0)) L.stt |= SHAPE_ST_NONPOSITIVE_FLUX;
    L.nsweep = 1;
    store_L<TEAM>(W, L, tid);
    sweep_sums<DT, MODEL, EM, TEAM, LAYOUT>(b, st, make_trial(W.L.p, MODEL, o.moffat_beta), C, xs,
                                            tid);
    L = load_L(W);
    if (!__builtin_isfinite(C[0])) {
      L.stt = SHAPE_ST_NONFINITE_INPUT;
      L.done = 1;
    }
  }
  store_L<TEAM>(W, L, tid);
}

// The second half of a trial (W.smax >= 0): the sweep at the trial point W.pt
// into the other sums buffer, the amplitudes at the trial shape, and the
// verdict; an accepted trial's sums become current.
template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT = kLayoutAny, bool PROF = true>
__device__ __forceinline__ void lm_sweep_judge(const shape_batch& b, const KOpts& o,
                                               const Stamp& st, LmShared& W, double* xs,
                                               int tid) {
  constexpr uint32_t EM = eff_mask(MASK, MODEL);
  constexpr uint32_t LIN = PROF ? (EM & 0xC0u) : 0u;  // profiled amplitudes
  const int cur = W.cur;
  // the sweep at the trial point (nothing else is live here)
  double* T = W.sums[cur ^ 1];
  sweep_sums<DT, MODEL, EM, TEAM, LAYOUT>(b, st, make_trial(W.pt, MODEL, o.moffat_beta), T, xs, tid);
  // amplitudes at the trial shape, then accept or reject
  LmState L = load_L(W);
  double pt[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) pt[k] = W.pt[k];
  AmpStep a{true, 0.0, 0.0};
  if (LIN != 0u) a = profile_amplitudes<EM, LIN, TEAM>(T, pt[6], tid);
  const bool accepted = lm_judge<LIN>(L, pt, a, W.smax, T[0], W.sums[cur][0], o);
  team_sync<TEAM>();
  if (tid == 0) {
    W.L = L;
    W.cur = accepted ? cur ^ 1 : cur;
  }
  team_sync<TEAM>();
}

// One LM trial from the current sums; the trial's sums go to the other buffer
// and become current when the trial is accepted.  Sets W.L.done when the fit
// has converged or stalled; the caller enforces max_iter_lm.
// PROF = false: the unprofiled form, the free amplitudes are searched by the
// same damped step as the shape parameters (no Schur complement, no
// amplitude update at the trial), with s_6 = |I0| and s_7 = sigma in the
// stopping rule.
template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT = kLayoutAny, bool PROF = true>
__device__ __forceinline__ void lm_iterate(const shape_batch& b, const KOpts& o, const Stamp& st,
                                           LmShared& W, double* xs, int tid) {
  constexpr uint32_t EM = eff_mask(MASK, MODEL);
  constexpr uint32_t LIN = PROF ? (EM & 0xC0u) : 0u;  // profiled amplitudes
  constexpr uint32_t NL = PROF ? (EM & 0x3Fu) : EM;   // parameters of the damped step
  constexpr int NN = popcount(NL);
  const int cur = W.cur;
  // Phase 1a: the damped Schur complement of the amplitude block, one lower-
  // triangle entry per thread:
  //   M_ac = A_ac - A_aL (A_LL)^-1 A_Lc = A_ac - u_a A_c6 - w_a A_c7.
  constexpr int NT = NN * (NN + 1) / 2;
  if (tid < NT) {
    const double* C = W.sums[cur];
    int a = 0, c = tid;
    while (c > a) {
      c -= a + 1;
      ++a;
    }
    double v = schur_entry<LIN>(C, nth_bit(NL, a), nth_bit(NL, c));
    if (a == c) v *= 1.0 + W.L.lambda;
    W.M[tid] = v;
  }
  team_sync<TEAM>();
  // Phase 1b: one thread solves the damped system and forms the trial point.
  if (tid == 0) {
    double m[NT], x[NN];
#pragma unroll
    for (int e = 0; e < NT; ++e) m[e] = W.M[e];
#pragma unroll
    for (int a = 0; a < NN; ++a) x[a] = W.sums[cur][sg(nth_bit(NL, a))];
    const bool solved = ldl_solve<NN>(m, x);
    LmState L = W.L;
    W.smax = lm_propose<MODEL, NL, LIN, NN>(L, step_rhs<NL, NN>(W.sums[cur]), x, solved, o, st,
                                            W.pt);
    W.L = L;
  }
  team_sync<TEAM>();
  if (W.smax < 0.0) return;
  lm_sweep_judge<DT, MODEL, MASK, TEAM, LAYOUT, PROF>(b, o, st, W, xs, tid);
}

// Whether the end point lies on the edge of the parameter box: a fitted
// parameter within a relative 1e-3 of a bound (|e| >= gmax - 1e-3; Re <=
// 0.1 (1 + 1e-3) or >= side (1 - 1e-3); Sersic n <= 0.2 (1 + 1e-3) or >=
// 10 (1 - 1e-3)).  Such a minimum lies on the box, not at a stationary point
// of chi^2; the fit is flagged AT_BOUND.
template <int MODEL, uint32_t EM>
__device__ __forceinline__ bool at_box_edge(const double* p, double gmax, int side) {
  constexpr double m = 1e-3;
  bool edge = false;
  if constexpr (has(EM, 2) || has(EM, 3)) edge = edge || p[2] * p[2] + p[3] * p[3] >= (gmax - m) * (gmax - m);
  if constexpr (has(EM, 4)) edge = edge || p[4] <= 0.1 * (1.0 + m) || p[4] >= side * (1.0 - m);
  if constexpr (MODEL == SHAPE_SERSIC && has(EM, 5))
    edge = edge || p[5] <= 0.2 * (1.0 + m) || p[5] >= 10.0 * (1.0 - m);
  return edge;
}

// Outputs of a finished (or capped) fit from its state and current sums C:
// parameters, chi^2, optional sqrt(diag((J^T J / sigma^2)^-1)) over the fitted
// parameters, iterations, status, sweeps.
template <int MODEL, uint32_t MASK>
__device__ __forceinline__ void lm_finish(const KOpts& o, const Stamp& st, LmState L,
                                          const double* C, int64_t s, float* p_out,
                                          float* chi2_out, float* perr, int32_t* iters,
                                          uint32_t* status, int32_t* sweeps, int tid) {
  constexpr uint32_t EM = eff_mask(MASK, MODEL);
  constexpr uint32_t LIN = EM & 0xC0u;
  constexpr uint32_t NL = EM & 0x3Fu;
  const bool valid = !(L.stt & (SHAPE_ST_BAD_INPUT | SHAPE_ST_NONFINITE_INPUT));
  if (valid && !(L.stt & (SHAPE_ST_CONVERGED | SHAPE_ST_STALLED))) L.stt |= SHAPE_ST_MAX_ITER;
  if (valid && at_box_edge<MODEL, EM>(L.p, o.gmax, st.side)) L.stt |= SHAPE_ST_AT_BOUND;
  if (tid == 0) {
    if (perr) {
      // sigma_p = sigma sqrt(diag(A^-1)) over the fitted parameters, A = J^T J:
      // A = L L^T by Cholesky, then diag(A^-1)_c = sum_i (L^-1)_ic^2.
      constexpr uint32_t FM = NL | LIN;
      constexpr int NF = popcount(FM);
      double Lf[NF][NF], Li[NF][NF];
      bool okf = valid;
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        double sjj = C[sa(nth_bit(FM, j), nth_bit(FM, j))];
#pragma unroll
        for (int l = 0; l < j; ++l) sjj -= Lf[j][l] * Lf[j][l];
        okf = okf && sjj > 0.0;
        const double d = sqrt(fmax(sjj, 1e-300));
        Lf[j][j] = d;
        Li[j][j] = 1.0 / d;
#pragma unroll
        for (int i = j + 1; i < NF; ++i) {
          double v = C[sa(nth_bit(FM, i), nth_bit(FM, j))];
#pragma unroll
          for (int l = 0; l < j; ++l) v -= Lf[i][l] * Lf[j][l];
          Lf[i][j] = v * Li[j][j];
        }
      }
#pragma unroll
      for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int i = j + 1; i < NF; ++i) {
          double v = 0.0;
#pragma unroll
          for (int k = j; k < i; ++k) v += Lf[i][k] * Li[k][j];
          Li[i][j] = -v * Li[i][i];
        }
      double e[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) e[k] = valid ? 0.0 : (double)qnan();
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        double d2 = 0.0;
#pragma unroll
        for (int i = c; i < NF; ++i) d2 += Li[i][c] * Li[i][c];
        e[nth_bit(FM, c)] = okf ? st.sigma * sqrt(d2) : (double)qnan();
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) perr[s * 8 + k] = (float)e[k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) p_out[s * 8 + k] = valid ? (float)L.p[k] : qnan();
    chi2_out[s] = valid ? (float)(C[0] / (st.sigma * st.sigma)) : qnan();
    iters[s] = L.it;
    status[s] = L.stt;
    if (sweeps) sweeps[s] = L.nsweep;
  }
}

}  // namespace shape
