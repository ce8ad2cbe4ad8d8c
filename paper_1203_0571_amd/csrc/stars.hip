// Star sizes from weighted moments (Sec. 4.2), one wave per stamp.
//
// About the centre and ellipticity of the moments stage, with R the model's
// elliptical radius (R^2 = |S(g) theta|^2 / (1 - |g|^2)) and f = I - sky0, each
// step sums r0 = sum f W, r2 = sum f W R^2, r4 = sum f W R^4 (FP32 over 8
// pixels of a lane, then FP64) for the current weight width w, then:
//   Gaussian (Sec. 4.2.1, W = exp(-R^2 / 2 w^2)): sigma = sqrt(r2 / r0),
//            I0 = r0 / (pi sigma^2)  (exact when w = sigma);
//   Moffat   (Sec. 4.2.2, W = (1 + R^2 / w^2)^-3): beta = 1 / (r4 r0 / 2 r2^2 - 1),
//            rd = sqrt(r2 / r0 (beta + 1)), I0 = r0 (beta + 2) / (pi rd^2)
//            (exact when w = rd);
//   Moffat with beta fixed (the paper's way out of the rd-beta degeneracy:
//            beta from bright stars, fixed for fainter ones): the same weight,
//            rd and I0 from r0 and r2 with the given beta (r4 unused);
// and sets w to the new size until the fractional change is below tol.
//
// Only w changes from step to step, so f and R^2 of every pixel are formed
// once.  One wave per stamp: stamps of up to 64 x kCache pixels keep f and
// R^2 in registers (pixel lane + 64 q in slot q) and read HBM once; larger
// stamps recompute them from the stamp on every step.  A batch of 32 x 32
// stars in the FP32 instance takes two stars per wave (star_pair_kernel):
// with FP64 reductions that was slower, since a wave iterates as long as the
// slower of its two stars; with FP32 ones it gains a little (3-4%).
//
// Precision (type T of the sums and of the step's closed forms): with 16
// pixels per lane the step's reductions and closed forms cost as much as the
// pixels, and in FP64 they took about 40% of the step.  For tolerances of
// kStarExactTol and above T is FP32: a lane's at most 16 register pixels are
// summed in FP32 (larger stamps' lanes in FP32 runs of 8 pixels carried in
// FP64), and the wave sum and the closed forms run in FP32; the sums' rounding
// (~1e-7 relative, reaching beta amplified by about beta) stays far below such
// a tolerance and the 1e-3 agreement with the FP64 oracle.  Tighter
// tolerances would stop on that rounding, so they take T = FP64: FP32 runs of
// 8 pixels carried in FP64, FP64 wave sums and closed forms.
#include "slots.hpp"
#include "kernels.hpp"

namespace shape {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kCache = 16;   // side <= 32
constexpr double kStarExactTol = 1e-5;

__device__ __forceinline__ float star_rcp(float x) { return fast_rcp(x); }
__device__ __forceinline__ double star_rcp(double x) { return rcp_f64(x); }   // Newton
__device__ __forceinline__ float star_sqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double star_sqrt(double x) { return sqrt(x); }

struct StarGeom {
  float x0, y0, a11, a12, a22, invD, sky;
};

__device__ inline float star_r2(const StarGeom& G, int i, int j) {
  const float t1 = (float)j - G.x0, t2 = (float)i - G.y0;
  const float v1 = fmaf(G.a11, t1, G.a12 * t2), v2 = fmaf(G.a12, t1, G.a22 * t2);
  return fmaf(v1, v1, v2 * v2) * G.invD;
}

// One pixel's terms of r0, r2, r4, added to FP32 partials s[0..2].
template <int PROFILE, int N>
__device__ __forceinline__ void star_accumulate(float f, float R2, float c, float (&s)[N]) {
  static_assert(N >= 3, "three partial sums");
  float W;
  if constexpr (PROFILE == 0) {
    W = fast_exp2(-R2 * c);
  } else {
    const float ib = fast_rcp(fmaf(R2, c, 1.0f));
    W = ib * ib * ib;
  }
  const float fw = f * W;
  const float fw2 = fw * R2;
  s[0] += fw;
  s[1] += fw2;
  s[2] = fmaf(fw2, R2, s[2]);
}

// Pixels a lane sums in FP32 before carrying the partial sums on in FP64.
constexpr int kStarBlock = 8;

// Profiles: 0 Gaussian, 1 Moffat, 2 Moffat with beta fixed.
__host__ __device__ constexpr bool moffat_weight(int profile) { return profile != 0; }

// The weight's constant for width w (w > 0).
template <int PROFILE, typename T>
__device__ __forceinline__ float weight_const(T w) {
  const T iw2 = star_rcp(w * w);
  return (float)(moffat_weight(PROFILE) ? iw2 : (T)(0.5 * kLog2e) * iw2);
}

// The starting width: the Gaussian's sigma_w, or the Moffat (beta = 3, or
// the fixed beta) whose half-light radius is r50: its enclosed flux is
// 1 - (1 + R^2 / rd^2)^(1 - beta) of the total.
template <int PROFILE>
__device__ __forceinline__ double start_width(const float (&r)[SHAPE_REC_LEN], double beta_fixed) {
  if constexpr (PROFILE == 0) return (double)r[SHAPE_REC_SIGW];
  const double bw = PROFILE == 2 ? beta_fixed : 3.0;
  return (double)r[SHAPE_REC_R50] / sqrt(exp2(1.0 / (bw - 1.0)) - 1.0);
}

// One step from the sums (s0, s2, s4) = (r0, r2, r4): the new size, and beta
// for the free Moffat; false when the step cannot be taken (status in stt).
template <int PROFILE, typename T>
__device__ __forceinline__ bool star_step(T s0, T s2, T s4, T& beta, T& ns, uint32_t& stt) {
  if (!(s0 > (T)0) || !(s2 > (T)0)) {
    stt |= SHAPE_ST_NONPOSITIVE_FLUX;
    return false;
  }
  const T is0 = star_rcp(s0);   // s0, s2 > 0 here
  if constexpr (PROFILE == 0) {
    ns = star_sqrt(s2 * is0);
  } else {
    if constexpr (PROFILE == 1) {
      const T is2 = star_rcp(s2);
      const T q = (T)0.5 * (s4 * is2) * (s0 * is2) - (T)1;
      if (!(q > (T)0)) {
        stt |= SHAPE_ST_SINGULAR;
        return false;
      }
      beta = star_rcp(q);
    }
    ns = star_sqrt(s2 * is0 * (beta + (T)1));
  }
  return true;
}

template <int DT, int PROFILE, typename T>
__global__ __launch_bounds__(kWave) void star_kernel(shape_batch b, const float* rec, double tol,
                                                     int max_iter, double beta_fixed, float* out,
                                                     int32_t* iters, uint32_t* status) {
  const int lane = threadIdx.x;
  for (int64_t s = blockIdx.x; s < b.n; s += gridDim.x) {
    const Stamp st = stamp_info(b, s);
    float r[SHAPE_REC_LEN];
    bool finite = true;
#pragma unroll
    for (int q = 0; q < SHAPE_REC_LEN; ++q) {
      r[q] = rec[s * SHAPE_REC_LEN + q];
      finite = finite && (q == SHAPE_REC_SIZE || __builtin_isfinite(r[q]));  // size may be NaN
    }
    if (st.bad || !finite) {
      if (lane < 4) out[s * 4 + lane] = qnan();
      if (lane == 0) {
        iters[s] = 0;
        status[s] = st.bad ? st.bad : SHAPE_ST_BAD_INPUT;
      }
      continue;
    }
    const double g1 = r[SHAPE_REC_E1], g2 = r[SHAPE_REC_E2];
    StarGeom G;
    G.x0 = r[SHAPE_REC_X0];
    G.y0 = r[SHAPE_REC_Y0];
    G.a11 = (float)(1.0 - g1);
    G.a12 = (float)(-g2);
    G.a22 = (float)(1.0 + g1);
    G.invD = (float)(1.0 / (1.0 - g1 * g1 - g2 * g2));
    G.sky = r[SHAPE_REC_SKY0];
    const bool cached = st.npix <= kWave * kCache;
    float cf[kCache], cr[kCache];
    if (cached) {
#pragma unroll
      for (int q = 0; q < kCache; ++q) {
        const int k = lane + kWave * q;
        cf[q] = 0.0f;
        cr[q] = 0.0f;
        if (k < st.npix) {
          const int i = k / st.side;
          cf[q] = load_px<DT>(b.pixels, st.off, k, st.scale) - G.sky;
          cr[q] = star_r2(G, i, k - i * st.side);
        }
      }
    }
    T w = (T)start_width<PROFILE>(r, beta_fixed);
    T size = w, beta = PROFILE == 2 ? (T)beta_fixed : (T)0, r0 = 0, s0_ok = 0;
    const T tolt = (T)tol;
    uint32_t stt = 0;
    int it = 0;
    while (it < max_iter) {
      const float c = weight_const<PROFILE>(w);   // w > 0: the start and every new size
      T u[4] = {0, 0, 0, 0};   // r0, r2, r4 (and a pad)
      if (cached) {
        if constexpr (sizeof(T) == 4) {
#pragma unroll
          for (int q = 0; q < kCache; ++q) star_accumulate<PROFILE>(cf[q], cr[q], c, u);
        } else {
          float sp[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int q = 0; q < kCache; ++q) {
            star_accumulate<PROFILE>(cf[q], cr[q], c, sp);
            if (q % kStarBlock == kStarBlock - 1) {
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                u[k] += (T)sp[k];
                sp[k] = 0.0f;
              }
            }
          }
        }
      } else {
        double ud[3] = {0.0, 0.0, 0.0};
        float sp[3] = {0.0f, 0.0f, 0.0f};
        auto carry = [&]() {
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            ud[q] += (double)sp[q];
            sp[q] = 0.0f;
          }
        };
        int cnt = 0;
        for_pixels(st.side, [&](int k, int i, int j) {
          const float f = load_px<DT>(b.pixels, st.off, k, st.scale) - G.sky;
          star_accumulate<PROFILE>(f, star_r2(G, i, j), c, sp);
          if (++cnt == kStarBlock) {
            carry();
            cnt = 0;
          }
        });
        carry();
#pragma unroll
        for (int q = 0; q < 3; ++q) u[q] = (T)ud[q];
      }
      wave_sum_n(u);
      const T s0 = u[0], s2 = u[1], s4 = u[2];
      ++it;
      r0 = s0;
      T ns;
      if (!star_step<PROFILE>(s0, s2, s4, beta, ns, stt)) break;
      const bool small = fabs(ns - w) < tolt * ns;   // fractional change below tol
      size = ns;
      w = ns;
      s0_ok = s0;
      if (small) {
        stt |= SHAPE_ST_CONVERGED;
        break;
      }
    }
    // I0 of the last completed step (0 if none)
    double I0 = 0.0;
    if (s0_ok > (T)0)
      I0 = (PROFILE == 0 ? (double)s0_ok : (double)s0_ok * ((double)beta + 2.0)) /
           (kPi * (double)size * (double)size);
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

// Two 32 x 32 stars per wave for the FP32 instance (lanes 32 g + j hold
// column j of star g, slot m = row m): each lane sums 32 pixels per step,
// and the step's reduction and closed forms are shared by the two stars;
// the wave iterates until both stop.
template <int DT, int PROFILE>
__global__ __launch_bounds__(kWave) void star_pair_kernel(shape_batch b, const float* rec,
                                                          double tol, int max_iter,
                                                          double beta_fixed, float* out,
                                                          int32_t* iters, uint32_t* status) {
  constexpr int W = kPairSide;
  const int lane = threadIdx.x, g = lane >> 5, j = lane & (W - 1);
  for (int64_t s0 = 2 * (int64_t)blockIdx.x; s0 < b.n; s0 += 2 * (int64_t)gridDim.x) {
    const int64_t s = s0 + g < b.n ? s0 + g : s0;   // a missing second star repeats the first
    const bool own = s0 + g < b.n;                  // and writes nothing
    const Stamp st = stamp_info(b, s);
    float r[SHAPE_REC_LEN];
    bool finite = true;
#pragma unroll
    for (int q = 0; q < SHAPE_REC_LEN; ++q) {
      r[q] = rec[s * SHAPE_REC_LEN + q];
      finite = finite && (q == SHAPE_REC_SIZE || __builtin_isfinite(r[q]));  // size may be NaN
    }
    const bool live = !st.bad && finite;
    const double g1 = live ? r[SHAPE_REC_E1] : 0.0, g2 = live ? r[SHAPE_REC_E2] : 0.0;
    StarGeom G;
    G.x0 = live ? r[SHAPE_REC_X0] : 0.0f;
    G.y0 = live ? r[SHAPE_REC_Y0] : 0.0f;
    G.a11 = (float)(1.0 - g1);
    G.a12 = (float)(-g2);
    G.a22 = (float)(1.0 + g1);
    G.invD = (float)(1.0 / (1.0 - g1 * g1 - g2 * g2));
    G.sky = live ? r[SHAPE_REC_SKY0] : 0.0f;
    float cf[W], cr[W];
    {
      const void* sp = stamp_base<DT>(b, st);
#pragma unroll
      for (int m = 0; m < W; ++m) {
        cf[m] = live ? load_rel<DT>(sp, (uint32_t)(m * W + j), st.scale) - G.sky : 0.0f;
        cr[m] = star_r2(G, m, j);
      }
    }
    float w = live ? (float)start_width<PROFILE>(r, beta_fixed) : 1.0f;
    float size = w, beta = PROFILE == 2 ? (float)beta_fixed : 0.0f, r0 = 0.0f, s0_ok = 0.0f;
    const float tolt = (float)tol;
    uint32_t stt = 0;
    int it = 0;
    bool done = !live || !own;
    for (int step = 0; step < max_iter; ++step) {
      if (!__any(!done)) break;
      const float c = weight_const<PROFILE>(w);
      float u[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // r0, r2, r4 (and a pad)
#pragma unroll
      for (int m = 0; m < W; ++m) star_accumulate<PROFILE>(cf[m], cr[m], c, u);
      half_sum_n(u);
      if (!done) {
        ++it;
        r0 = u[0];
        float ns;
        if (!star_step<PROFILE>(u[0], u[1], u[2], beta, ns, stt)) {
          done = true;
        } else {
          const bool small = fabsf(ns - w) < tolt * ns;   // fractional change below tol
          size = ns;
          w = ns;
          s0_ok = u[0];
          if (small) {
            stt |= SHAPE_ST_CONVERGED;
            done = true;
          }
        }
      }
    }
    if (!own) continue;
    if (!live) {
      if (j < 4) out[s * 4 + j] = qnan();
      if (j == 0) {
        iters[s] = 0;
        status[s] = st.bad ? st.bad : SHAPE_ST_BAD_INPUT;
      }
      continue;
    }
    double I0 = 0.0;
    if (s0_ok > 0.0f)
      I0 = (PROFILE == 0 ? (double)s0_ok : (double)s0_ok * ((double)beta + 2.0)) /
           (kPi * (double)size * (double)size);
    if (!(stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_SINGULAR)))
      stt |= SHAPE_ST_MAX_ITER;
    if (j == 0) {
      out[s * 4 + 0] = size;
      out[s * 4 + 1] = beta;
      out[s * 4 + 2] = (float)I0;
      out[s * 4 + 3] = r0;
      iters[s] = it;
      status[s] = stt;
    }
  }
}

template <int DT, int PROFILE>
void launch_one(const shape_batch& b, const float* rec, double tol, int max_iter, double beta,
                float* out, int32_t* iters, uint32_t* status, hipStream_t stream) {
  const int64_t cap = 1ll << 30;
  const dim3 grid((unsigned)(b.n < cap ? b.n : cap));
  if (tol >= kStarExactTol && !b.side && b.side0 == kPairSide) {
    const int64_t n2 = (b.n + 1) / 2;
    hipLaunchKernelGGL((star_pair_kernel<DT, PROFILE>), dim3((unsigned)(n2 < cap ? n2 : cap)),
                       dim3(kWave), 0, stream, b, rec, tol, max_iter, beta, out, iters, status);
  } else if (tol >= kStarExactTol)
    hipLaunchKernelGGL((star_kernel<DT, PROFILE, float>), grid, dim3(kWave), 0, stream, b, rec,
                       tol, max_iter, beta, out, iters, status);
  else
    hipLaunchKernelGGL((star_kernel<DT, PROFILE, double>), grid, dim3(kWave), 0, stream, b, rec,
                       tol, max_iter, beta, out, iters, status);
}

template <int DT>
void launch_dtype(const shape_batch& b, int profile, const float* rec, double tol, int max_iter,
                  double beta, float* out, int32_t* iters, uint32_t* status, hipStream_t stream) {
  switch (profile) {
    case 0: launch_one<DT, 0>(b, rec, tol, max_iter, beta, out, iters, status, stream); break;
    case 1: launch_one<DT, 1>(b, rec, tol, max_iter, beta, out, iters, status, stream); break;
    default: launch_one<DT, 2>(b, rec, tol, max_iter, beta, out, iters, status, stream);
  }
}

}  // namespace

hipError_t launch_stars(const shape_batch& b, int profile, const float* rec, double tol,
                        int max_iter, double beta, float* out, int32_t* iters, uint32_t* status,
                        hipStream_t stream) {
  if (b.dtype == SHAPE_F32)
    launch_dtype<SHAPE_F32>(b, profile, rec, tol, max_iter, beta, out, iters, status, stream);
  else
    launch_dtype<SHAPE_F16_SCALED>(b, profile, rec, tol, max_iter, beta, out, iters, status,
                                   stream);
  return hipGetLastError();
}

}  // namespace shape
