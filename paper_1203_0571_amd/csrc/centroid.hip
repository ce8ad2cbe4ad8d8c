// Starting estimates and the circular-weight centroid (one wave per stamp).
//
// Sec. 4.1 (starting point): the brightest pixel, and r50 from the growth
// curve about it; Sec. 2: Gaussian-weighted first moments, the centre moving
// by (<x>/N)/k with the fixed gain k.
#include "kernels.hpp"

namespace shape {
namespace {

constexpr int kMaxRings = 184;  // ring index of a 128-px stamp is at most 180

// Smallest r >= 0 with r * r >= d2 (the ring holding a pixel at distance^2 d2).
__device__ inline int ring_of(int d2) {
  int r = (int)ceilf(sqrtf((float)d2));
  while (r * r < d2) ++r;
  while (r > 0 && (r - 1) * (r - 1) >= d2) --r;
  return r;
}

template <int DT, int SIDE>
__global__ __launch_bounds__(kWave) void centroid_kernel(shape_batch b, KOpts o, float* rec,
                                                         int32_t* iters, uint32_t* status) {
  // Growth curve: ring sums in fixed point, so the atomics are exact and the
  // result does not depend on the order in which lanes add.
  __shared__ unsigned long long ring[kMaxRings];
  const int lane = threadIdx.x;
  for (int64_t s = blockIdx.x; s < b.n; s += gridDim.x) {
    const Stamp st = stamp_info(b, s);
    float* out = rec + s * SHAPE_REC_LEN;
    if (st.bad) {
      if (lane < SHAPE_REC_LEN) out[lane] = qnan();
      if (lane == 0) {
        iters[s] = 0;
        status[s] = st.bad;
      }
      continue;
    }
    const int W = SIDE ? SIDE : st.side;
    // Passes 1 and 2 read the stamp from memory; the iterations of pass 3
    // sweep it from registers when the batch's side allows (StampPixels).
    const StampPixels<DT, 0> mem(b, st, lane);

    // Pass 1: finiteness, border sum, brightest pixel, largest |I|.
    double border = 0.0;
    float best = -__builtin_huge_valf();
    int besti = 0x7fffffff;
    float amax = 0.0f;
    bool nonfinite = false;
    mem.each([&](float v, int k, int i, int j) {
      nonfinite |= !__builtin_isfinite(v);
      if (i == 0 || j == 0 || i == W - 1 || j == W - 1) border += (double)v;
      if (v > best) {  // k increases, so ties keep the lowest index
        best = v;
        besti = k;
      }
      amax = fmaxf(amax, fabsf(v));
    });
    if (wave_any(nonfinite)) {
      if (lane < SHAPE_REC_LEN) out[lane] = qnan();
      if (lane == 0) {
        iters[s] = 0;
        status[s] = SHAPE_ST_NONFINITE_INPUT;
      }
      continue;
    }
    border = wave_sum(border);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      float ov = __shfl_xor(best, m, kWave);
      int oi = __shfl_xor(besti, m, kWave);
      if (ov > best || (ov == best && oi < besti)) {
        best = ov;
        besti = oi;
      }
      amax = fmaxf(amax, __shfl_xor(amax, m, kWave));
    }
    const double sky0 = border / (4.0 * W - 4.0);
    const int i0 = besti / W, j0 = besti - (besti / W) * W;

    // Pass 2: ring sums of f = I - sky0 about the brightest pixel.  The fixed-
    // point scale is a power of two with |f| * scale * npix < 2.3e18 (so 2 * sum fits).
    const int nrings = ring_of(2 * (W - 1) * (W - 1)) + 1;
    const double fmaxabs = (double)amax + fabs(sky0) + 1.0;
    const double fix = exp2(floor(log2(2.3e18 / ((double)st.npix * fmaxabs))));
    for (int r = lane; r < nrings; r += kWave) ring[r] = 0ull;
    __syncthreads();
    mem.each([&](float v, int, int i, int j) {
      double f = (double)v - sky0;
      int d2 = (i - i0) * (i - i0) + (j - j0) * (j - j0);
      long long q = __double2ll_rn(f * fix);
      atomicAdd(&ring[ring_of(d2)], (unsigned long long)q);
    });
    __syncthreads();
    // Every lane scans the rings (LDS broadcast reads) and reaches the same r50.
    long long F = 0;
#pragma unroll 1
    for (int r = 0; r < nrings; ++r) F += (long long)ring[r];
    uint32_t stt = 0;
    double r50 = 0.125 * W;
    if (F > 0) {
      long long cum = (long long)ring[0], prev = 0;
#pragma unroll 1
      for (int r = 1; r < nrings; ++r) {
        cum += (long long)ring[r];
        if (2 * cum >= F) {  // first crossing of half the total flux
          r50 = (r - 1) + (0.5 * (double)F - (double)prev) / (double)(cum - prev);
          break;
        }
        prev = cum;
      }
    } else {
      stt |= SHAPE_ST_NONPOSITIVE_FLUX;
    }
    __syncthreads();  // ring[] is reused by the next stamp of this wave
    double sigw = r50 / sqrt(2.0 * kLn2);
    sigw = fmin(fmax(sigw, 1.0), 0.25 * W);

    // Pass 3: centroid iteration from the brightest pixel.
    const StampPixels<DT, SIDE> px(b, st, lane);
    double x = j0, y = i0;
    const float c2 = (float)(kLog2e / (2.0 * sigw * sigw));
    const float skyf = (float)sky0;
    int it = 0;
    while (it < o.max_iter_centroid) {
      double N = 0.0, Sx = 0.0, Sy = 0.0;
      const float xf = (float)x, yf = (float)y;
      px.each([&](float v, int, int i, int j) {
        float t1 = (float)j - xf, t2 = (float)i - yf;
        float w = fast_exp2(-(t1 * t1 + t2 * t2) * c2);
        float fw = (v - skyf) * w;
        N += (double)fw;
        Sx += (double)(fw * t1);
        Sy += (double)(fw * t2);
      });
      N = wave_sum(N);
      Sx = wave_sum(Sx);
      Sy = wave_sum(Sy);
      ++it;
      if (!(N > 0.0)) {
        stt |= SHAPE_ST_NONPOSITIVE_FLUX;
        break;
      }
      double dx = Sx / (o.k_gain * N), dy = Sy / (o.k_gain * N);
      x += dx;
      y += dy;
      if (x < 0.0 || y < 0.0 || x > W - 1 || y > W - 1) {
        stt |= SHAPE_ST_LOST;
        break;
      }
      if (fabs(dx) < o.tol_x && fabs(dy) < o.tol_x) {
        stt |= SHAPE_ST_CONVERGED;
        break;
      }
    }
    if (!(stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_LOST)))
      stt |= SHAPE_ST_MAX_ITER;
    if (lane == 0) {
      out[SHAPE_REC_X0] = (float)x;
      out[SHAPE_REC_Y0] = (float)y;
      out[SHAPE_REC_E1] = 0.0f;
      out[SHAPE_REC_E2] = 0.0f;
      out[SHAPE_REC_SIGW] = (float)sigw;
      out[SHAPE_REC_R50] = (float)r50;
      out[SHAPE_REC_SKY0] = (float)sky0;
      out[SHAPE_REC_FLUX] = (float)((double)F / fix);
      iters[s] = it;
      status[s] = stt;
    }
  }
}

template <int DT>
void launch_side(int side, int64_t grid, const shape_batch& b, const KOpts& o, float* rec,
                 int32_t* iters, uint32_t* status, hipStream_t stream) {
  const dim3 g((unsigned)grid), t(kWave);
  switch (side) {
    case 8: hipLaunchKernelGGL((centroid_kernel<DT, 8>), g, t, 0, stream, b, o, rec, iters, status); break;
    case 16: hipLaunchKernelGGL((centroid_kernel<DT, 16>), g, t, 0, stream, b, o, rec, iters, status); break;
    case 32: hipLaunchKernelGGL((centroid_kernel<DT, 32>), g, t, 0, stream, b, o, rec, iters, status); break;
    case 64: hipLaunchKernelGGL((centroid_kernel<DT, 64>), g, t, 0, stream, b, o, rec, iters, status); break;
    default: hipLaunchKernelGGL((centroid_kernel<DT, 0>), g, t, 0, stream, b, o, rec, iters, status);
  }
}

}  // namespace

hipError_t launch_centroid(const shape_batch& b, const KOpts& o, float* rec, int32_t* iters,
                           uint32_t* status, hipStream_t stream) {
  const int64_t grid = b.n < (1ll << 30) ? b.n : (1ll << 30);
  // A batch of one side that divides 64 keeps each stamp in registers.
  const int side = (!b.side && register_side(b.side0)) ? b.side0 : 0;
  if (b.dtype == SHAPE_F32)
    launch_side<SHAPE_F32>(side, grid, b, o, rec, iters, status, stream);
  else
    launch_side<SHAPE_F16_SCALED>(side, grid, b, o, rec, iters, status, stream);
  return hipGetLastError();
}

}  // namespace shape
