// Joint centroid + ellipticity with an elliptical Gaussian weight: Sec. 3
// (eqs. psh, newg), App. A (eqs. xshew, eshew), App. B (eqs. dxsh, desh,
// P1..P6).
//
// Every integrand of App. A and App. B is a polynomial of degree <= 4 in the
// offsets theta times f W (W' = -W / 2 sigma_w^2), so one sweep per step
// accumulates the eleven weighted moments
//   M_pq = sum f W theta1^p theta2^q,  (p, q) in {00, 10, 01, 20, 11, 02,
//                                                 40, 31, 22, 13, 04}
// and the 2x2 algebra is done from them in FP64.  A lane owns whole pixel
// columns (theta1 fixed), so the eleven moments come from five column sums
// of f W theta2^q, each summed in FP32 over at most 8 rows at a time and in
// FP64 beyond that.  The stamp is read from memory once into registers:
// moments_kernel for a batch of one side that divides 64 (one wave per
// stamp), moments_any_kernel for any side (a SlotMap column layout; one wave
// up to side 64, a team of three or four waves above).
#include "slots.hpp"
#include "kernels.hpp"

namespace shape {
namespace {

struct Mom {
  double m00, m10, m01, m20, m11, m02;
  float m40, m31, m22, m13, m04;
};

// A column's contribution to the moments: M_pq = theta1^p S_q.
__device__ __forceinline__ void add_column(Mom& M, double t1, const double (&S)[5]) {
  const double p2 = t1 * t1;
  M.m00 += S[0];
  M.m10 += t1 * S[0];
  M.m01 += S[1];
  M.m20 += p2 * S[0];
  M.m11 += t1 * S[1];
  M.m02 += S[2];
  M.m40 += (float)(p2 * p2 * S[0]);
  M.m31 += (float)(p2 * t1 * S[1]);
  M.m22 += (float)(p2 * S[2]);
  M.m13 += (float)(t1 * S[3]);
  M.m04 += (float)S[4];
}

// KSB quantities from the moments (weight ellipticity g, W' = c W).
struct Ksb {
  double T, e1, e2, P11, P12, P21, P22;
};

__device__ inline Ksb ksb_from_moments(const Mom& M, double g1, double g2, double c) {
  const double gg = g1 * g1 + g2 * g2;
  const double A = 1.0 + gg - 2.0 * g1, B = 1.0 + gg + 2.0 * g1;
  const double m40 = M.m40, m31 = M.m31, m22 = M.m22, m13 = M.m13, m04 = M.m04;
  const double tr = M.m20 + M.m02;
  Ksb k;
  k.T = tr;
  const double iT = rcp_f64(tr);   // tr > 0 (checked by the caller)
  k.e1 = (M.m20 - M.m02) * iT;
  k.e2 = 2.0 * M.m11 * iT;
  // App. A: X^SH and the integral part of e^SH.
  const double X11 = (2.0 * tr + 2.0 * c * (A * m40 - (A + B) * m22 + B * m04)) * iT;
  const double X12 = 2.0 * c * ((A + B) * (m31 - m13) - 2.0 * g2 * (m40 - m04)) * iT;
  const double X21 = 4.0 * c * (A * m31 - B * m13) * iT;
  const double X22 = (2.0 * tr + 4.0 * c * ((A + B) * m22 - 2.0 * g2 * (m31 + m13))) * iT;
  const double E1 = 2.0 * k.e1 + 2.0 * c * (A * (m40 + m22) - B * (m22 + m04)) * iT;
  const double E2 = 2.0 * k.e2 +
                    2.0 * c * ((A + B) * (m31 + m13) - 2.0 * g2 * (m40 + 2.0 * m22 + m04)) * iT;
  // App. B: sums of f P1 .. f P6.
  const double d20 = M.m20 - M.m02;
  const double P1 = 4.0 * d20 + 2.0 * c * (A * m40 + (B - A) * m22 - B * m04 - 4.0 * g2 * (m31 - m13));
  const double P2 = 4.0 * M.m11 + 2.0 * c * ((A - B) * (m31 - m13) + 2.0 * g2 * (m40 - 2.0 * m22 + m04));
  const double P3 = 8.0 * M.m11 + 4.0 * c * (A * m31 + B * m13 - 4.0 * g2 * m22);
  const double P4 = -2.0 * d20 + 4.0 * c * ((A - B) * m22 + 2.0 * g2 * (m31 - m13));
  const double P5 = 4.0 * tr + 2.0 * c * (A * (m40 + m22) + B * (m22 + m04) - 4.0 * g2 * (m31 + m13));
  const double P6 = 2.0 * c * ((A - B) * (m31 + m13) + 2.0 * g2 * (m40 - m04));
  const double dX11 = (-g1 * P1 - g2 * P2) * iT, dX12 = (g1 * P2 - g2 * P1) * iT;
  const double dX21 = (-g1 * P3 - g2 * P4) * iT, dX22 = (g1 * P4 - g2 * P3) * iT;
  const double dE1 = (-g1 * P5 - g2 * P6) * iT, dE2 = (g1 * P6 - g2 * P5) * iT;
  // eq. psh with the App. B terms: P_ab = X_ab + dX_ab - e_a (e^SH_b + de^SH_b)
  k.P11 = X11 + dX11 - k.e1 * (E1 + dE1);
  k.P12 = X12 + dX12 - k.e1 * (E2 + dE2);
  k.P21 = X21 + dX21 - k.e2 * (E1 + dE1);
  k.P22 = X22 + dX22 - k.e2 * (E2 + dE2);
  return k;
}

// Shared by both forms: the moments of one step (summed over the stamp)
// turned into the step of Sec. 3.  The FP32 fourth moments are widened here.
struct StepState {
  double x, y, g1, g2;
  double sq_num, sq_den, sq_gg;   // the last step's sum f W R^2, sum f W, |g_w|^2
  uint32_t stt;
};

// Returns true when the iteration stops (status bits in st.stt).
__device__ inline bool moments_step(const double (&u)[12], double c, int W, const KOpts& o,
                                    StepState& z) {
  Mom M;
  M.m00 = u[0];
  M.m10 = u[1];
  M.m01 = u[2];
  M.m20 = u[3];
  M.m11 = u[4];
  M.m02 = u[5];
  M.m40 = (float)u[6];
  M.m31 = (float)u[7];
  M.m22 = (float)u[8];
  M.m13 = (float)u[9];
  M.m04 = (float)u[10];
  const double g1 = z.g1, g2 = z.g2;
  // sum f W R^2 (R^2 of this step's weight), sum f W and |g_w|^2: the fit's
  // starting size comes from the last step's (after the loop)
  z.sq_num = ((1.0 - g1) * (1.0 - g1) + g2 * g2) * M.m20 +
             ((1.0 + g1) * (1.0 + g1) + g2 * g2) * M.m02 - 4.0 * g2 * M.m11;
  z.sq_den = M.m00;
  z.sq_gg = g1 * g1 + g2 * g2;
  if (!(M.m00 > 0.0) || !(M.m20 + M.m02 > 0.0)) {
    z.stt |= SHAPE_ST_NONPOSITIVE_FLUX;
    return true;
  }
  const Ksb K = ksb_from_moments(M, g1, g2, c);
  const double det = K.P11 * K.P22 - K.P12 * K.P21;
  if (!(fabs(det) > 1e-300) || !__builtin_isfinite(det)) {
    z.stt |= SHAPE_ST_SINGULAR;
    return true;
  }
  // eq. newg: dg = (1 - |g_w|^2) P^-1 (e_obs - e_w), e_w = 2 g_w / (1 + |g_w|^2)
  const double gg = g1 * g1 + g2 * g2;
  const double ew = 2.0 * rcp_f64(1.0 + gg), sd = (1.0 - gg) / det;   // det of either sign
  const double r1 = K.e1 - g1 * ew, r2 = K.e2 - g2 * ew;
  double dg1 = sd * (K.P22 * r1 - K.P12 * r2);
  double dg2 = sd * (-K.P21 * r1 + K.P11 * r2);
  double h = 1.0;
  bool halved = false;
  for (int q = 0; q < 60; ++q) {
    const double a = g1 + h * dg1, bb = g2 + h * dg2;
    if (a * a + bb * bb <= o.gmax * o.gmax) break;
    h *= 0.5;
    halved = true;
    z.stt |= SHAPE_ST_G_CLAMPED;
  }
  dg1 *= h;
  dg2 *= h;
  const double iN = rcp_f64(o.k_gain * M.m00);   // M00 > 0 here
  const double dx = M.m10 * iN, dy = M.m01 * iN;
  z.g1 += dg1;
  z.g2 += dg2;
  z.x += dx;
  z.y += dy;
  if (z.x < 0.0 || z.y < 0.0 || z.x > W - 1 || z.y > W - 1) {
    z.stt |= SHAPE_ST_LOST;
    return true;
  }
  // a step cut at the |g_w| bound is small for that reason alone: never a stop
  if (!halved && fabs(dx) < o.tol_x && fabs(dy) < o.tol_x && fabs(dg1) < o.tol_g &&
      fabs(dg2) < o.tol_g) {
    z.stt |= SHAPE_ST_CONVERGED;
    return true;
  }
  return false;
}

// The fit's starting size: a source exp(-R^2 / 2 s^2) gives the weighted
// second moment q = 2 s^2 sigma_w^2 / (s^2 + sigma_w^2); its half-light
// radius along the model's radius R / sqrt(1 - |g|^2) is s sqrt(2 ln 2).
__device__ inline double start_size(const StepState& z, double sigw) {
  const double q = z.sq_num / z.sq_den, s2w = sigw * sigw;
  if (z.sq_den > 0.0 && q > 0.0 && q < 1.96 * s2w)
    return sqrt(2.0 * kLn2 * (q * s2w / (2.0 * s2w - q)) / (1.0 - z.sq_gg));
  return qnan();
}

__device__ inline void write_out(float* out, const float (&r_in)[SHAPE_REC_LEN], const StepState& z,
                                 double size, int it, int32_t* iters, uint32_t* status, int64_t s) {
  out[SHAPE_REC_X0] = (float)z.x;
  out[SHAPE_REC_Y0] = (float)z.y;
  out[SHAPE_REC_E1] = (float)z.g1;
  out[SHAPE_REC_E2] = (float)z.g2;
  out[SHAPE_REC_SIGW] = r_in[SHAPE_REC_SIGW];
  out[SHAPE_REC_R50] = r_in[SHAPE_REC_R50];
  out[SHAPE_REC_SKY0] = r_in[SHAPE_REC_SKY0];
  out[SHAPE_REC_FLUX] = r_in[SHAPE_REC_FLUX];
  out[SHAPE_REC_SIZE] = (float)size;
  iters[s] = it;
  status[s] = z.stt;
}

// Read the whole input record (before anything is written: in == out is
// allowed); false when the record or the stamp cannot be used.
__device__ inline bool read_record(const float* in, float (&r_in)[SHAPE_REC_LEN]) {
#pragma unroll
  for (int q = 0; q < SHAPE_REC_LEN; ++q) r_in[q] = in[q];
  bool bad_rec = false;
#pragma unroll
  for (int q = 0; q < SHAPE_REC_SIZE; ++q) bad_rec |= !__builtin_isfinite(r_in[q]);  // size may be NaN
  return !bad_rec;
}

// The five column sums S_q = sum f W theta2^q from the slot sums
// T_j = sum f W k^j, theta2 = dl + r k.
__device__ __forceinline__ void column_sums(const double (&T)[5], double dl, double r,
                                            double (&S)[5]) {
  const double d2 = dl * dl, r2 = r * r;
  S[0] = T[0];
  S[1] = dl * T[0] + r * T[1];
  S[2] = d2 * T[0] + 2.0 * dl * r * T[1] + r2 * T[2];
  S[3] = d2 * dl * T[0] + 3.0 * d2 * r * T[1] + 3.0 * dl * r2 * T[2] + r2 * r * T[3];
  S[4] = d2 * d2 * T[0] + 4.0 * d2 * dl * r * T[1] + 6.0 * d2 * r2 * T[2] +
         4.0 * dl * r2 * r * T[3] + r2 * r2 * T[4];
}

// R^2 of App. A: [(1-g1)^2+g2^2] t1^2 + [(1+g1)^2+g2^2] t2^2 - 4 g2 t1 t2.
// Along a column the exponent -cw R^2 is a quadratic in theta2:
// theta2 (A theta2 + B) + C; with theta2 = tc + r k it is a quadratic in k,
// (Ak k + Bk) k + Ck.
struct ColumnExp {
  float Ak, Bk, Ck;
  __device__ __forceinline__ ColumnExp(const StepState& z, float cw, float t1, float tc, float r) {
    const float a11 = (float)((1.0 - z.g1) * (1.0 - z.g1) + z.g2 * z.g2);
    const float a22 = (float)((1.0 + z.g1) * (1.0 + z.g1) + z.g2 * z.g2);
    const float a12 = (float)(-4.0 * z.g2);
    const float A = -cw * a22;
    const float B = -cw * (a12 * t1), C = -cw * (a11 * (t1 * t1));
    Ak = A * (r * r);
    Bk = r * fmaf(2.0f * A, tc, B);
    Ck = fmaf(fmaf(A, tc, B), tc, C);
  }
};

// Slot sums of one block of kColumnBlock slots (k = m - kC constants once
// unrolled), added to T in FP64.
template <int K, int M0>
__device__ __forceinline__ void block_sums(const float (&v)[K], const ColumnExp& e, double (&T)[5]) {
  constexpr int kC = K / 2;
  float bs[5] = {};
#pragma unroll
  for (int m = M0; m < M0 + kColumnBlock && m < K; ++m) {
    const float k1 = (float)(m - kC), k2 = k1 * k1;
    const float fw = v[m] * fast_exp2(fmaf(fmaf(e.Ak, k1, e.Bk), k1, e.Ck));
    bs[0] += fw;
    bs[1] = fmaf(fw, k1, bs[1]);
    bs[2] = fmaf(fw, k2, bs[2]);
    bs[3] = fmaf(fw, k2 * k1, bs[3]);
    bs[4] = fmaf(fw, k2 * k2, bs[4]);
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) T[q] += (double)bs[q];
}

// block_sums over the blocks below `rows` (a wave-uniform bound).
template <int K, int M0 = 0>
__device__ __forceinline__ void all_blocks(const float (&v)[K], const ColumnExp& e, double (&T)[5],
                                           int rows) {
  if constexpr (M0 < K) {
    if (M0 < rows) block_sums<K, M0>(v, e, T);
    all_blocks<K, M0 + kColumnBlock>(v, e, T, rows);
  }
}

__device__ __forceinline__ void moments_pack(const Mom& M, double (&u)[12]) {
  u[0] = M.m00;
  u[1] = M.m10;
  u[2] = M.m01;
  u[3] = M.m20;
  u[4] = M.m11;
  u[5] = M.m02;
  u[6] = (double)M.m40;
  u[7] = (double)M.m31;
  u[8] = (double)M.m22;
  u[9] = (double)M.m13;
  u[10] = (double)M.m04;
  u[11] = 0.0;
}

// Waves per SIMD the register budget is sized for: at four, a 64 x 64 stamp
// in registers leaves the FP64 step algebra a few spills, and the kernel runs
// about 4% slower than at three.
#ifndef SHAPE_MOMENTS_WAVES_PER_SIMD
#define SHAPE_MOMENTS_WAVES_PER_SIMD 3
#endif
template <int DT, int SIDE>
__global__ __launch_bounds__(kWave, SHAPE_MOMENTS_WAVES_PER_SIMD) void moments_kernel(
    shape_batch b, KOpts o, const float* rec_in, float* rec_out, int32_t* iters,
    uint32_t* status) {
  static_assert(SIDE == 8 || SIDE == 16 || SIDE == 32 || SIDE == 64, "side must divide 64");
  const int lane = threadIdx.x;
  for (int64_t s = blockIdx.x; s < b.n; s += gridDim.x) {
    const Stamp st = stamp_info(b, s);
    float* out = rec_out + s * SHAPE_REC_LEN;
    float r_in[SHAPE_REC_LEN];
    const bool rec_ok = read_record(rec_in + s * SHAPE_REC_LEN, r_in);
    if (st.bad || !rec_ok) {
      __syncthreads();
      if (lane < SHAPE_REC_LEN) out[lane] = qnan();
      if (lane == 0) {
        iters[s] = 0;
        status[s] = st.bad ? st.bad : SHAPE_ST_BAD_INPUT;
      }
      continue;
    }
    constexpr int W = SIDE;
    constexpr int kR = kWave / SIDE, kSlots = StampPixels<DT, SIDE>::kSlots;
    StampPixels<DT, SIDE> px(b, st, lane);
    const double sigw = r_in[SHAPE_REC_SIGW];
    const float skyf = r_in[SHAPE_REC_SKY0];
    const double c = -1.0 / (2.0 * sigw * sigw);           // W' = c W
    const float cw = (float)(kLog2e / (2.0 * sigw * sigw));
    StepState z = {r_in[SHAPE_REC_X0], r_in[SHAPE_REC_Y0], 0.0, 0.0, 0.0, 0.0, 0.0, 0u};
    // the register stamp becomes f = I - sky0 once, for every step
#pragma unroll
    for (int m = 0; m < kSlots; ++m) px.v[m] -= skyf;
    int it = 0;
    while (it < o.max_iter_moments) {
      // Every moment is theta1^p times a column sum S_q = sum f W theta2^q
      // (q = 0..4) down the lane's column jl at rows il + kR m.  Down the
      // column theta2 = delta + kR k with k = m - kC, so the lane sums
      // T_j = sum f W k^j (k^j a constant of the unrolled slot) in FP32
      // over blocks of up to kColumnBlock rows and in FP64 across blocks, and
      // turns them into S_q once per column.
      constexpr int kC = kSlots / 2;
      float il = (float)(lane / SIDE), jl = (float)(lane & (SIDE - 1));
      asm volatile("" : "+v"(il), "+v"(jl));
      const float xf = (float)z.x, yf = (float)z.y;
      const float t1 = jl - xf, tb = il - yf;
      const ColumnExp e(z, cw, t1, tb + (float)(kR * kC), (float)kR);
      double T[5] = {};
      all_blocks<kSlots>(px.v, e, T, kSlots);
      double S[5];
      column_sums(T, (double)il + (double)(kR * kC) - z.y, (double)kR, S);
      Mom M = {};
      add_column(M, (double)jl - z.x, S);
      double u[12];
      moments_pack(M, u);
      wave_sum_n(u);
      ++it;
      if (moments_step(u, c, W, o, z)) break;
    }
    if (!(z.stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_SINGULAR | SHAPE_ST_LOST)))
      z.stt |= SHAPE_ST_MAX_ITER;
    const double size = start_size(z, sigw);
    __syncthreads();  // all lanes have read the input record
    if (lane == 0) write_out(out, r_in, z, size, it, iters, status, s);
  }
}

// Two 32 x 32 stamps per wave (lanes 32 g + j: column j of stamp g, slot m =
// row m), as centroid_pair_kernel: the moments and the step of
// moments_kernel with the sums taken per half-wave, iterating until both
// stamps stop.
template <int DT>
__global__ __launch_bounds__(kWave, SHAPE_MOMENTS_WAVES_PER_SIMD) void moments_pair_kernel(
    shape_batch b, KOpts o, const float* rec_in, float* rec_out, int32_t* iters,
    uint32_t* status) {
  constexpr int W = kPairSide, kSlots = kPairSide;
  const int lane = threadIdx.x, g = lane >> 5, j = lane & (W - 1);
  for (int64_t s0 = 2 * (int64_t)blockIdx.x; s0 < b.n; s0 += 2 * (int64_t)gridDim.x) {
    const int64_t s = s0 + g < b.n ? s0 + g : s0;   // a missing second stamp repeats the first
    const bool own = s0 + g < b.n;                  // and writes nothing
    const Stamp st = stamp_info(b, s);
    float* out = rec_out + s * SHAPE_REC_LEN;
    float r_in[SHAPE_REC_LEN];
    const bool rec_ok = read_record(rec_in + s * SHAPE_REC_LEN, r_in);
    const bool live = !st.bad && rec_ok;
    float v[kSlots];
    {
      const void* sp = stamp_base<DT>(b, st);
#pragma unroll
      for (int m = 0; m < kSlots; ++m)
        v[m] = live ? load_rel<DT>(sp, (uint32_t)(m * W + j), st.scale) : 0.0f;
    }
    const double sigw = live ? (double)r_in[SHAPE_REC_SIGW] : 1.0;
    const float skyf = live ? r_in[SHAPE_REC_SKY0] : 0.0f;
    const double c = -1.0 / (2.0 * sigw * sigw);           // W' = c W
    const float cw = (float)(kLog2e / (2.0 * sigw * sigw));
    StepState z = {live ? (double)r_in[SHAPE_REC_X0] : 0.0, live ? (double)r_in[SHAPE_REC_Y0] : 0.0,
                   0.0, 0.0, 0.0, 0.0, 0.0, 0u};
#pragma unroll
    for (int m = 0; m < kSlots; ++m) v[m] -= skyf;
    bool done = !live || !own;
    int it = 0;
    for (int step = 0; step < o.max_iter_moments; ++step) {
      if (!__any(!done)) break;
      constexpr int kC = kSlots / 2;
      float jl = (float)j;
      asm volatile("" : "+v"(jl));
      const float xf = (float)z.x, yf = (float)z.y;
      const float t1 = jl - xf;
      const ColumnExp e(z, cw, t1, (float)kC - yf, 1.0f);
      double T[5] = {};
      all_blocks<kSlots>(v, e, T, kSlots);
      double S[5];
      column_sums(T, (double)kC - z.y, 1.0, S);
      Mom M = {};
      add_column(M, (double)jl - z.x, S);
      double u[12];
      moments_pack(M, u);
      half_sum_n(u);
      if (!done) {
        ++it;
        done = moments_step(u, c, W, o, z);
      }
    }
    if (live && !(z.stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_SINGULAR |
                           SHAPE_ST_LOST)))
      z.stt |= SHAPE_ST_MAX_ITER;
    const double size = start_size(z, sigw);
    __syncthreads();  // all lanes have read the input records
    if (own) {
      if (live) {
        if (j == 0) write_out(out, r_in, z, size, it, iters, status, s);
      } else {
        if (j < SHAPE_REC_LEN) out[j] = qnan();
        if (j == 0) {
          iters[s] = 0;
          status[s] = st.bad ? st.bad : SHAPE_ST_BAD_INPUT;
        }
      }
    }
  }
}

// A team's step state as its leader wave hands it to the others.
struct StepShare {
  StepState z;
  int stop;
};

// One stamp of the any-side form, its slots unrolled K wide.
template <int DT, int TEAM, int K>
__device__ __forceinline__ void moments_any(const shape_batch& b, const KOpts& o, const Stamp& st,
                                            int64_t s, const float (&r_in)[SHAPE_REC_LEN],
                                            float* out, int32_t* iters, uint32_t* status,
                                            double* part, StepShare* share, int& parity) {
  const int t = threadIdx.x;
  const SlotMap<TEAM> mp(st.side, t);
  constexpr int RC = fixed_rows_groups<TEAM, K>();
  const int W = mp.W, R = RC ? RC : mp.R, rows = mp.rows;
  float v[K];
  load_slots<DT, TEAM, K>(v, stamp_base<DT>(b, st), mp, st.scale);
  const double sigw = r_in[SHAPE_REC_SIGW];
  const float skyf = r_in[SHAPE_REC_SKY0];
  const double c = -1.0 / (2.0 * sigw * sigw);           // W' = c W
  const float cw = (float)(kLog2e / (2.0 * sigw * sigw));
  StepState z = {r_in[SHAPE_REC_X0], r_in[SHAPE_REC_Y0], 0.0, 0.0, 0.0, 0.0, 0.0, 0u};
#pragma unroll
  for (int m = 0; m < K; ++m) v[m] = mp.valid(m) ? v[m] - skyf : 0.0f;
  constexpr int kC = K / 2;
  int it = 0;
  while (it < o.max_iter_moments) {
    // the register form's column sums, with a runtime row stride R and the
    // blocks past the stamp's rows skipped
    float il = (float)mp.il, jl = (float)mp.jl;
    asm volatile("" : "+v"(il), "+v"(jl));
    const float xf = (float)z.x, yf = (float)z.y, r = (float)R;
    const float t1 = jl - xf, tb = il - yf;
    const ColumnExp e(z, cw, t1, fmaf(r, (float)kC, tb), r);
    double T[5] = {};
    all_blocks<K>(v, e, T, rows);
    double S[5];
    column_sums(T, (double)il + (double)R * kC - z.y, (double)R, S);
    Mom M = {};
    add_column(M, (double)jl - z.x, S);
    double u[12];
    moments_pack(M, u);
    ++it;
    if constexpr (TEAM == 1) {
      wave_sum_n(u);
      if (moments_step(u, c, W, o, z)) break;
    } else {
      // The step's FP64 algebra runs on one wave of the team (the leader,
      // chosen by the stamp index so the leaders of different workgroups
      // fall on different SIMDs); the others wait for its new state.
      wave_sum_n(u);
      const int w = t / kWave, lane = t & (kWave - 1);
      double* b = part + parity * TEAM * 12;
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 12; ++j) b[w * 12 + j] = u[j];
      }
      __syncthreads();
      if (w == (int)(s % TEAM)) {
#pragma unroll
        for (int j = 0; j < 12; ++j) {
          double a = b[j];
#pragma unroll
          for (int q = 1; q < TEAM; ++q) a += b[q * 12 + j];
          u[j] = a;
        }
        const bool stop = moments_step(u, c, W, o, z);
        if (lane == 0) {
          share[parity].z = z;
          share[parity].stop = stop;
        }
      }
      __syncthreads();
      z = share[parity].z;
      const bool stop = share[parity].stop;
      parity ^= 1;
      if (stop) break;
    }
  }
  if (!(z.stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_SINGULAR | SHAPE_ST_LOST)))
    z.stt |= SHAPE_ST_MAX_ITER;
  const double size = start_size(z, sigw);
  __syncthreads();  // every thread has read the input record
  if (t == 0) write_out(out, r_in, z, size, it, iters, status, s);
}

// One form per team size (team_takes: one wave up to side 64, three waves
// for 65..96, four for 97..128); each skips the others' stamps.  Stamps that
// cannot be processed are reported by the one-wave form, or by a team form
// launched without it (take_bad).
#ifndef SHAPE_MOMENTS_ANY_WAVES_PER_SIMD
#define SHAPE_MOMENTS_ANY_WAVES_PER_SIMD 3
#endif
template <int DT, int TEAM>
__global__ __launch_bounds__(kWave * TEAM, SHAPE_MOMENTS_ANY_WAVES_PER_SIMD) void
moments_any_kernel(shape_batch b, KOpts o, const float* rec_in, float* rec_out, int32_t* iters,
                   uint32_t* status, int take_bad, int chunk) {
  __shared__ double part[2 * TEAM * 12];
  __shared__ StepShare share[2];
  int parity = 0;
  const int t = threadIdx.x;
  for (int64_t s0 = (int64_t)blockIdx.x * chunk; s0 < b.n; s0 += (int64_t)gridDim.x * chunk)
  for (uint64_t mine = chunk_mask<TEAM>(b, s0, chunk, take_bad); mine; mine &= mine - 1) {
    const int64_t s = s0 + __builtin_ctzll(mine);
    const Stamp st = stamp_info(b, s);
    float* out = rec_out + s * SHAPE_REC_LEN;
    float r_in[SHAPE_REC_LEN];
    const bool rec_ok = read_record(rec_in + s * SHAPE_REC_LEN, r_in);
    if (st.bad || !rec_ok) {
      __syncthreads();
      if (t < SHAPE_REC_LEN) out[t] = qnan();
      if (t == 0) {
        iters[s] = 0;
        status[s] = st.bad ? st.bad : SHAPE_ST_BAD_INPUT;
      }
      continue;
    }
    if constexpr (TEAM > 1) {
      moments_any<DT, TEAM, 64>(b, o, st, s, r_in, out, iters, status, part, share, parity);
    } else {
      switch (slot_class(SlotMap<TEAM>(st.side, 0).rows)) {
        case 8: moments_any<DT, TEAM, 8>(b, o, st, s, r_in, out, iters, status, part, share, parity); break;
        case 16: moments_any<DT, TEAM, 16>(b, o, st, s, r_in, out, iters, status, part, share, parity); break;
        case 32: moments_any<DT, TEAM, 32>(b, o, st, s, r_in, out, iters, status, part, share, parity); break;
        default: moments_any<DT, TEAM, 64>(b, o, st, s, r_in, out, iters, status, part, share, parity);
      }
    }
  }
}

template <int DT>
void launch_dtype(const shape_batch& b, const KOpts& o, const float* rec_in, float* rec_out,
                  int32_t* iters, uint32_t* status, hipStream_t stream) {
  const int64_t cap = 1ll << 30;
  const dim3 one(kWave);
  if (!b.side && register_side(b.side0)) {
    const dim3 g((unsigned)(b.n < cap ? b.n : cap));
    switch (b.side0) {
      case 8: hipLaunchKernelGGL((moments_kernel<DT, 8>), g, one, 0, stream, b, o, rec_in, rec_out, iters, status); break;
      case 16: hipLaunchKernelGGL((moments_kernel<DT, 16>), g, one, 0, stream, b, o, rec_in, rec_out, iters, status); break;
      case 32: {
        const int64_t n2 = (b.n + 1) / 2;
        hipLaunchKernelGGL((moments_pair_kernel<DT>), dim3((unsigned)(n2 < cap ? n2 : cap)), one, 0,
                           stream, b, o, rec_in, rec_out, iters, status);
        break;
      }
      default: hipLaunchKernelGGL((moments_kernel<DT, 64>), g, one, 0, stream, b, o, rec_in, rec_out, iters, status);
    }
    return;
  }
  // One side for the whole batch: only the form that takes it, a stamp per
  // workgroup.  Mixed sides: every form, each workgroup looking at a chunk of
  // stamps and taking those of its form.
  const bool mixed = b.side != nullptr;
  const bool f1 = mixed || team_takes<1>(b.side0) ||
                  (!team_takes<3>(b.side0) && !team_takes<4>(b.side0));
  const bool f3 = mixed || team_takes<3>(b.side0), f4 = mixed || team_takes<4>(b.side0);
  auto grid = [&](int chunk) {
    const int64_t g = (b.n + chunk - 1) / chunk;
    return dim3((unsigned)(g < cap ? g : cap));
  };
  if (f1) {
    const int c = mixed ? chunk_of<1>() : 1;
    hipLaunchKernelGGL((moments_any_kernel<DT, 1>), grid(c), dim3(kWave), 0, stream, b, o, rec_in, rec_out, iters, status, 1, c);
  }
  if (f3) {
    const int c = mixed ? chunk_of<3>() : 1;
    hipLaunchKernelGGL((moments_any_kernel<DT, 3>), grid(c), dim3(3 * kWave), 0, stream, b, o, rec_in, rec_out, iters, status, f1 ? 0 : 1, c);
  }
  if (f4) {
    const int c = mixed ? chunk_of<4>() : 1;
    hipLaunchKernelGGL((moments_any_kernel<DT, 4>), grid(c), dim3(4 * kWave), 0, stream, b, o, rec_in, rec_out, iters, status, f1 ? 0 : 1, c);
  }
}

}  // namespace

hipError_t launch_moments(const shape_batch& b, const KOpts& o, const float* rec_in,
                          float* rec_out, int32_t* iters, uint32_t* status, hipStream_t stream) {
  if (b.dtype == SHAPE_F32)
    launch_dtype<SHAPE_F32>(b, o, rec_in, rec_out, iters, status, stream);
  else
    launch_dtype<SHAPE_F16_SCALED>(b, o, rec_in, rec_out, iters, status, stream);
  return hipGetLastError();
}

}  // namespace shape
