// Joint centroid + ellipticity with an elliptical Gaussian weight (one wave
// per stamp): Sec. 3 (eqs. psh, newg), App. A (eqs. xshew, eshew), App. B
// (eqs. dxsh, desh, P1..P6).
//
// Every integrand of App. A and App. B is a polynomial of degree <= 4 in the
// offsets theta times f W (W' = -W / 2 sigma_w^2), so one sweep per step
// accumulates the eleven weighted moments
//   M_pq = sum f W theta1^p theta2^q,  (p, q) in {00, 10, 01, 20, 11, 02,
//                                                 40, 31, 22, 13, 04}
// and the 2x2 algebra is done from them in FP64.  A lane owns whole pixel
// columns (theta1 fixed), so the eleven moments come from five column sums
// of f W theta2^q, each summed in FP32 over at most 8 rows at a time and in
// FP64 beyond that; the stamp is held in registers when its side divides 64
// and read by columns from memory otherwise.
#include "columns.hpp"
#include "kernels.hpp"

namespace shape {
namespace {

struct Mom {
  double m00, m10, m01, m20, m11, m02;
  float m40, m31, m22, m13, m04;
};

// One pixel's terms of the column sums S_q = sum f W theta2^q, q = 0..4.
__device__ __forceinline__ void add_pixel(float (&b)[5], float fw, float t2) {
  b[0] += fw;
  float g = fw * t2;
  b[1] += g;
  g *= t2;
  b[2] += g;
  g *= t2;
  b[3] += g;
  b[4] = fmaf(g, t2, b[4]);
}

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
  const int lane = threadIdx.x;
  for (int64_t s = blockIdx.x; s < b.n; s += gridDim.x) {
    const Stamp st = stamp_info(b, s);
    const float* in = rec_in + s * SHAPE_REC_LEN;
    float* out = rec_out + s * SHAPE_REC_LEN;
    // Read the whole input record before anything is written (in == out allowed).
    float r_in[SHAPE_REC_LEN];
#pragma unroll
    for (int q = 0; q < SHAPE_REC_LEN; ++q) r_in[q] = in[q];
    bool bad_rec = false;
#pragma unroll
    for (int q = 0; q < SHAPE_REC_SIZE; ++q) bad_rec |= !__builtin_isfinite(r_in[q]);  // size may be NaN
    if (st.bad || bad_rec) {
      __syncthreads();
      if (lane < SHAPE_REC_LEN) out[lane] = qnan();
      if (lane == 0) {
        iters[s] = 0;
        status[s] = st.bad ? st.bad : SHAPE_ST_BAD_INPUT;
      }
      continue;
    }
    const int W = SIDE ? SIDE : st.side;
    // the stamp in registers (side dividing 64) or read by columns
    StampPixels<DT, SIDE> px(b, st, lane);
    const StampColumns<DT> cols(b, st, lane);
    const double sigw = r_in[SHAPE_REC_SIGW];
    const float skyf = r_in[SHAPE_REC_SKY0];
    const double c = -1.0 / (2.0 * sigw * sigw);           // W' = c W
    const float cw = (float)(kLog2e / (2.0 * sigw * sigw));
    double x = r_in[SHAPE_REC_X0], y = r_in[SHAPE_REC_Y0];
    double g1 = 0.0, g2 = 0.0;
    // the register stamp becomes f = I - sky0 once, for every step
    if constexpr (SIDE > 0) {
#pragma unroll
      for (int m = 0; m < StampPixels<DT, SIDE>::kSlots; ++m) px.v[m] -= skyf;
    }
    double sq_num = 0.0, sq_den = 0.0, sq_gg = 0.0;
    uint32_t stt = 0;
    int it = 0;
    while (it < o.max_iter_moments) {
      // R^2 of App. A: [(1-g1)^2+g2^2] t1^2 + [(1+g1)^2+g2^2] t2^2 - 4 g2 t1 t2
      const float a11 = (float)((1.0 - g1) * (1.0 - g1) + g2 * g2);
      const float a22 = (float)((1.0 + g1) * (1.0 + g1) + g2 * g2);
      const float a12 = (float)(-4.0 * g2);
      const float xf = (float)x, yf = (float)y;
      Mom M = {};
      // Every moment is theta1^p times a column sum S_q = sum f W theta2^q
      // (q = 0..4) down a column the lane owns, taken in FP32 over blocks of
      // up to kColumnBlock rows and in FP64 across blocks.  Along a column the
      // exponent is a quadratic in theta2: -cw R^2 = theta2 (A theta2 + B) + C.
      const float A = -cw * a22;
      if constexpr (SIDE > 0) {
        // registers: lane column jl at rows il + kR m
        constexpr int kR = kWave / SIDE, kSlots = StampPixels<DT, SIDE>::kSlots;
        constexpr int kBlk = kSlots < kColumnBlock ? kSlots : kColumnBlock;
        // Down the column theta2 = delta + kR k with k = m - kC, so the lane
        // sums T_j = sum f W k^j (k^j a constant of the unrolled slot) and
        // turns them into S_q = sum f W theta2^q once per column.
        constexpr int kC = kSlots / 2;
        float il = (float)(lane / SIDE), jl = (float)(lane & (SIDE - 1));
        asm volatile("" : "+v"(il), "+v"(jl));
        const float t1 = jl - xf, tb = il - yf;
        const float B = -cw * (a12 * t1), C = -cw * (a11 * (t1 * t1));
        // the exponent as a quadratic in k: A t2^2 + B t2 + C with
        // t2 = tc + kR k, tc = theta2 at the middle slot
        const float tc = tb + (float)(kR * kC);
        const float Ak = A * (float)(kR * kR), Bk = (float)kR * fmaf(2.0f * A, tc, B);
        const float Ck = fmaf(fmaf(A, tc, B), tc, C);
        double T[5] = {};
#pragma unroll
        for (int m0 = 0; m0 < kSlots; m0 += kBlk) {
          float bs[5] = {};
#pragma unroll
          for (int m = m0; m < m0 + kBlk; ++m) {
            const float k1 = (float)(m - kC), k2 = k1 * k1;   // constants once unrolled
            const float fw = px.v[m] * fast_exp2(fmaf(fmaf(Ak, k1, Bk), k1, Ck));
            bs[0] += fw;
            bs[1] = fmaf(fw, k1, bs[1]);
            bs[2] = fmaf(fw, k2, bs[2]);
            bs[3] = fmaf(fw, k2 * k1, bs[3]);
            bs[4] = fmaf(fw, k2 * k2, bs[4]);
          }
#pragma unroll
          for (int q = 0; q < 5; ++q) T[q] += (double)bs[q];
        }
        const double dl = (double)il + (double)(kR * kC) - y, r = kR;
        const double d2 = dl * dl, r2 = r * r;
        const double S[5] = {
            T[0], dl * T[0] + r * T[1], d2 * T[0] + 2.0 * dl * r * T[1] + r2 * T[2],
            d2 * dl * T[0] + 3.0 * d2 * r * T[1] + 3.0 * dl * r2 * T[2] + r2 * r * T[3],
            d2 * d2 * T[0] + 4.0 * d2 * dl * r * T[1] + 6.0 * d2 * r2 * T[2] +
                4.0 * dl * r2 * r * T[3] + r2 * r2 * T[4]};
        add_column(M, (double)jl - x, S);
      } else {
        // memory: the lane's column(s) of a stamp of any side
        for (int cc = 0; cc < cols.ncol; ++cc) {
          const float t1 = (float)cols.col(cc) - xf;
          const float B = -cw * (a12 * t1), C = -cw * (a11 * (t1 * t1));
          double S[5] = {};
          for (int m0 = 0; m0 < cols.rows; m0 += kColumnBlock) {
            float bs[5] = {};
#pragma unroll
            for (int q = 0; q < kColumnBlock; ++q) {
              bool in;
              const float v = cols.at_clamped(cc, m0 + q, in);
              const float t2 = (float)cols.row(m0 + q) - yf;
              const float w = fast_exp2(fmaf(fmaf(A, t2, B), t2, C));
              const float fw = (v - skyf) * (in ? w : 0.0f);
              add_pixel(bs, fw, t2);
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) S[q] += (double)bs[q];
          }
          add_column(M, (double)cols.col(cc) - x, S);
        }
      }
      {
        double u[12] = {M.m00, M.m10, M.m01, M.m20, M.m11, M.m02, (double)M.m40,
                        (double)M.m31, (double)M.m22, (double)M.m13, (double)M.m04, 0.0};
        wave_sum_n(u);
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
      }
      ++it;
      // sum f W R^2 (R^2 of this step's weight), sum f W and |g_w|^2: the
      // fit's starting size comes from the last step's (after the loop)
      sq_num = ((1.0 - g1) * (1.0 - g1) + g2 * g2) * M.m20 +
               ((1.0 + g1) * (1.0 + g1) + g2 * g2) * M.m02 - 4.0 * g2 * M.m11;
      sq_den = M.m00;
      sq_gg = g1 * g1 + g2 * g2;
      if (!(M.m00 > 0.0) || !(M.m20 + M.m02 > 0.0)) {
        stt |= SHAPE_ST_NONPOSITIVE_FLUX;
        break;
      }
      const Ksb K = ksb_from_moments(M, g1, g2, c);
      const double det = K.P11 * K.P22 - K.P12 * K.P21;
      if (!(fabs(det) > 1e-300) || !__builtin_isfinite(det)) {
        stt |= SHAPE_ST_SINGULAR;
        break;
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
        stt |= SHAPE_ST_G_CLAMPED;
      }
      dg1 *= h;
      dg2 *= h;
      const double iN = rcp_f64(o.k_gain * M.m00);   // M00 > 0 here
      const double dx = M.m10 * iN, dy = M.m01 * iN;
      g1 += dg1;
      g2 += dg2;
      x += dx;
      y += dy;
      if (x < 0.0 || y < 0.0 || x > W - 1 || y > W - 1) {
        stt |= SHAPE_ST_LOST;
        break;
      }
      // a step cut at the |g_w| bound is small for that reason alone: never a stop
      if (!halved && fabs(dx) < o.tol_x && fabs(dy) < o.tol_x && fabs(dg1) < o.tol_g &&
          fabs(dg2) < o.tol_g) {
        stt |= SHAPE_ST_CONVERGED;
        break;
      }
    }
    if (!(stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_SINGULAR | SHAPE_ST_LOST)))
      stt |= SHAPE_ST_MAX_ITER;
    // The fit's starting size: a source exp(-R^2 / 2 s^2) gives the weighted
    // second moment q = 2 s^2 sigma_w^2 / (s^2 + sigma_w^2); its half-light
    // radius along the model's radius R / sqrt(1 - |g|^2) is s sqrt(2 ln 2).
    double size = qnan();
    {
      const double q = sq_num / sq_den, s2w = sigw * sigw;
      if (sq_den > 0.0 && q > 0.0 && q < 1.96 * s2w)
        size = sqrt(2.0 * kLn2 * (q * s2w / (2.0 * s2w - q)) / (1.0 - sq_gg));
    }
    __syncthreads();  // all lanes have read the input record
    if (lane == 0) {
      out[SHAPE_REC_X0] = (float)x;
      out[SHAPE_REC_Y0] = (float)y;
      out[SHAPE_REC_E1] = (float)g1;
      out[SHAPE_REC_E2] = (float)g2;
      out[SHAPE_REC_SIGW] = r_in[SHAPE_REC_SIGW];
      out[SHAPE_REC_R50] = r_in[SHAPE_REC_R50];
      out[SHAPE_REC_SKY0] = r_in[SHAPE_REC_SKY0];
      out[SHAPE_REC_FLUX] = r_in[SHAPE_REC_FLUX];
      out[SHAPE_REC_SIZE] = (float)size;
      iters[s] = it;
      status[s] = stt;
    }
  }
}

template <int DT>
void launch_side(int side, int64_t grid, const shape_batch& b, const KOpts& o, const float* rec_in,
                 float* rec_out, int32_t* iters, uint32_t* status, hipStream_t stream) {
  const dim3 g((unsigned)grid), t(kWave);
  switch (side) {
    case 8: hipLaunchKernelGGL((moments_kernel<DT, 8>), g, t, 0, stream, b, o, rec_in, rec_out, iters, status); break;
    case 16: hipLaunchKernelGGL((moments_kernel<DT, 16>), g, t, 0, stream, b, o, rec_in, rec_out, iters, status); break;
    case 32: hipLaunchKernelGGL((moments_kernel<DT, 32>), g, t, 0, stream, b, o, rec_in, rec_out, iters, status); break;
    case 64: hipLaunchKernelGGL((moments_kernel<DT, 64>), g, t, 0, stream, b, o, rec_in, rec_out, iters, status); break;
    default: hipLaunchKernelGGL((moments_kernel<DT, 0>), g, t, 0, stream, b, o, rec_in, rec_out, iters, status);
  }
}

}  // namespace

hipError_t launch_moments(const shape_batch& b, const KOpts& o, const float* rec_in,
                          float* rec_out, int32_t* iters, uint32_t* status, hipStream_t stream) {
  const int64_t grid = b.n < (1ll << 30) ? b.n : (1ll << 30);
  // A batch of one side that divides 64 keeps each stamp in registers.
  const int side = (!b.side && register_side(b.side0)) ? b.side0 : 0;
  if (b.dtype == SHAPE_F32)
    launch_side<SHAPE_F32>(side, grid, b, o, rec_in, rec_out, iters, status, stream);
  else
    launch_side<SHAPE_F16_SCALED>(side, grid, b, o, rec_in, rec_out, iters, status, stream);
  return hipGetLastError();
}

}  // namespace shape
