// Starting estimates and the circular-weight centroid (one wave per stamp).
//
// Sec. 4.1 (starting point): the brightest pixel, and r50 from the growth
// curve about it; Sec. 2: Gaussian-weighted first moments, the centre moving
// by (<x>/N)/k with the fixed gain k.
#include "columns.hpp"
#include "kernels.hpp"

namespace shape {
namespace {

constexpr int kMaxRings = 184;  // ring index of a 128-px stamp is at most 180

// Smallest r >= 0 with r * r >= d2 (the ring holding a pixel at distance^2
// d2), for 0 <= d2 < 2^16.  The hardware square root is within an ulp, and a
// non-square d2 lies at least 1 / 512 from the nearest square root, so the
// ceiling can only be off at a perfect square, and then by one.
__device__ inline int ring_of(int d2) {
  int r = (int)ceilf(__builtin_amdgcn_sqrtf((float)d2));
  r += __mul24(r, r) < d2;
  r -= (r > 0 && __mul24(r - 1, r - 1) >= d2);
  return r;
}

// 1.5 * 2^52: adding it to a double of magnitude below 2^51 rounds that value
// to an integer held in the low mantissa bits.
constexpr double kRoundMagic = 6755399441055744.0;

// Waves per SIMD the register budget is sized for: at five a 64 x 64 stamp
// held in registers fits 96 VGPRs with a few spilled values (reloaded about
// once per step, not per pixel), and the kernel runs about 8% faster than at
// four (128 VGPRs, no spills).  The other sides need under 80 VGPRs either
// way.
#ifndef SHAPE_CENTROID_WAVES_PER_SIMD
#define SHAPE_CENTROID_WAVES_PER_SIMD (SIDE == 64 ? 5 : 4)
#endif
template <int DT, int SIDE>
__global__ __launch_bounds__(kWave, SHAPE_CENTROID_WAVES_PER_SIMD) void centroid_kernel(
    shape_batch b, KOpts o, float* rec, int32_t* iters, uint32_t* status) {
  // Growth curve: ring sums in fixed point, so the atomics are exact and the
  // result does not depend on the order in which lanes add.
  __shared__ unsigned long long ring[kMaxRings];
  __shared__ float wy_row[kWave];   // the weight's row factor (register stamps)
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
    // The stamp: in registers for a side that divides 64 (px), read from
    // memory column by column on every pass otherwise (cols).
    StampPixels<DT, SIDE> px(b, st, lane);
    const StampColumns<DT> cols(b, st, lane);
    constexpr int kR = SIDE ? kWave / SIDE : 1;   // rows between a lane's slots
    const int il = SIDE ? lane / SIDE : 0, jl = SIDE ? (lane & (SIDE - 1)) : 0;

    // Pass 1: finiteness, border sum, brightest pixel, largest |I|.
    double border = 0.0;
    float best = -__builtin_huge_valf();
    int besti = 0x7fffffff;
    float amax = 0.0f;
    bool nonfinite = false;
    if constexpr (SIDE > 0) {
      constexpr int kSlots = StampPixels<DT, SIDE>::kSlots;
      float vmin = __builtin_huge_valf();
#pragma unroll
      for (int m = 0; m < kSlots; ++m) {
        const float v = px.v[m];
        nonfinite |= !__builtin_isfinite(v);
        if (v > best) {  // the index increases with m, so ties keep the lowest
          best = v;
          besti = lane + kWave * m;
        }
        vmin = fminf(vmin, v);
      }
      amax = fmaxf(fabsf(best), fabsf(vmin));  // max |I| = max(max I, -min I)
      // the border: whole columns 0 and W - 1, the rest of rows 0 and W - 1
      if (jl == 0 || jl == SIDE - 1) {
#pragma unroll
        for (int m = 0; m < kSlots; ++m) border += (double)px.v[m];
      } else {
        if (il == 0) border += (double)px.v[0];
        if (il == kR - 1) border += (double)px.v[kSlots - 1];
      }
    } else {
      for (int c = 0; c < cols.ncol; ++c) {
        const int j = cols.col(c);
        const bool bcol = j == 0 || j == W - 1;
#pragma unroll 4
        for (int m = 0; m < cols.rows; ++m) {
          bool in;
          const float v = cols.at(c, m, in);
          if (in) {
            const int i = cols.row(m), k = i * W + j;
            nonfinite |= !__builtin_isfinite(v);
            if (bcol || i == 0 || i == W - 1) border += (double)v;
            if (v > best || (v == best && k < besti)) {  // ties keep the lowest index
              best = v;
              besti = k;
            }
            amax = fmaxf(amax, fabsf(v));
          }
        }
      }
    }
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

    // Pass 2: ring sums of f = I - sky0 about the brightest pixel, in fixed
    // point: f * fix rounded to an integer, with fix a power of two such that
    // |f| * fix < 2^50 (so kRoundMagic rounds it) and |f| * fix * npix < 2.3e18
    // (so twice a sum fits in 63 bits).
    const int nrings = ring_of(2 * (W - 1) * (W - 1)) + 1;
    const double fmaxabs = (double)amax + fabs(sky0) + 1.0;
    const double fix = ldexp(1.0, ilogb(fmin(2.3e18 / (double)st.npix, 0x1p50) / fmaxabs));
    // (I - sky0) fix + magic in one FMA: fix * I + (magic - sky0 fix)
    const double kofs = kRoundMagic - sky0 * fix;
    const long long magic_bits = __builtin_bit_cast(long long, kRoundMagic);
    for (int r = lane; r < nrings; r += kWave) ring[r] = 0ull;
    __syncthreads();
    auto deposit = [&](float v, int d2) {
      const double t = fma((double)v, fix, kofs);
      const long long q = __builtin_bit_cast(long long, t) - magic_bits;
      atomicAdd(&ring[ring_of(d2)], (unsigned long long)q);
    };
    if constexpr (SIDE > 0) {
      constexpr int kSlots = StampPixels<DT, SIDE>::kSlots;
      const int dj2 = __mul24(jl - j0, jl - j0);
      constexpr int kGrp = kSlots < 8 ? kSlots : 8;
#pragma unroll
      for (int m0 = 0; m0 < kSlots; m0 += kGrp) {
        // Groups of 8 slots behind an opaque copy that also orders them after
        // the previous group's atomics: otherwise every slot's fixed-point
        // value is formed (as a double) before the first atomic.
        float v[kGrp];
#pragma unroll
        for (int q = 0; q < kGrp; ++q) v[q] = px.v[m0 + q];
        asm volatile("" : "+v"(v[0]), "+v"(v[1 % kGrp]), "+v"(v[2 % kGrp]), "+v"(v[3 % kGrp]),
                     "+v"(v[4 % kGrp]), "+v"(v[5 % kGrp]), "+v"(v[6 % kGrp]), "+v"(v[7 % kGrp])
                     :
                     : "memory");
#pragma unroll
        for (int q = 0; q < kGrp; ++q) {
          const int di = il + kR * (m0 + q) - i0;
          deposit(v[q], __mul24(di, di) + dj2);
        }
      }
    } else {
      for (int c = 0; c < cols.ncol; ++c) {
        const int j = cols.col(c), dj2 = __mul24(j - j0, j - j0);
#pragma unroll 4
        for (int m = 0; m < cols.rows; ++m) {
          bool in;
          const float v = cols.at(c, m, in);
          const int di = cols.row(m) - i0;
          if (in) deposit(v, __mul24(di, di) + dj2);
        }
      }
    }
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
    double x = j0, y = i0;
    const float c2 = (float)(kLog2e / (2.0 * sigw * sigw));
    const float skyf = (float)sky0;
    // the register stamp becomes f = I - sky0 once, for every step
    if constexpr (SIDE > 0) {
#pragma unroll
      for (int m = 0; m < StampPixels<DT, SIDE>::kSlots; ++m) px.v[m] -= skyf;
    }
    // Sums N = sum f W, Sx = sum f W theta1, Sy = sum f W theta2 about (x, y).
    auto sweep = [&](double& N, double& Sx, double& Sy) {
      const float xf = (float)x, yf = (float)y;
      if constexpr (SIDE > 0) {
        // A lane holds one column (jl) at rows il + kR m.  The circular
        // weight factors as W = wx(theta1) wy(theta2), so the lane sums
        // f wy and f wy theta2 down its column and applies wx (and theta1)
        // once; the column sums run in FP32 over blocks of up to 8 rows and
        // in FP64 across blocks and lanes.
        // The row factor wy is the same for every column: lane r forms it
        // for row r and the wave reads it back from LDS.
        constexpr int kSlots = StampPixels<DT, SIDE>::kSlots;
        constexpr int kBlk = kSlots < kColumnBlock ? kSlots : kColumnBlock;
        wave_sync();  // the previous step's reads of wy_row are done
        {
          const float tr = (float)lane - yf;
          wy_row[lane] = fast_exp2(-(tr * tr) * c2);
        }
        wave_sync();
        float ilf = (float)il, jlf = (float)jl;
        asm volatile("" : "+v"(ilf), "+v"(jlf));
        // theta2 = delta + kR k with k = m - kC (a constant of the unrolled
        // slot), so the lane sums f wy k and forms the theta2 sum once.
        constexpr int kC = kSlots / 2;
        const float t1 = jlf - xf;
        const float* wy = wy_row + il;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int m0 = 0; m0 < kSlots; m0 += kBlk) {
          float b0 = 0.0f, b1 = 0.0f;
#pragma unroll
          for (int m = m0; m < m0 + kBlk; ++m) {
            const float fe = px.v[m] * wy[kR * m];
            b0 += fe;
            b1 = fmaf(fe, (float)(m - kC), b1);
          }
          s0 += (double)b0;
          s1 += (double)b1;
        }
        const double wx = (double)fast_exp2(-(t1 * t1) * c2);
        const double dl = (double)ilf + (double)(kR * kC) - y;
        N = wx * s0;
        Sx = wx * (double)t1 * s0;
        Sy = wx * (dl * s0 + (double)kR * s1);
      } else {
        // the same factoring down each column the lane owns in memory
        N = Sx = Sy = 0.0;
        for (int c = 0; c < cols.ncol; ++c) {
          const float t1 = (float)cols.col(c) - xf;
          double s0 = 0.0, s1 = 0.0;
          for (int m0 = 0; m0 < cols.rows; m0 += kColumnBlock) {
            float b0 = 0.0f, b1 = 0.0f;
#pragma unroll
            for (int q = 0; q < kColumnBlock; ++q) {
              bool in;
              const float v = cols.at_clamped(c, m0 + q, in);
              const float t2 = (float)cols.row(m0 + q) - yf;
              const float w = fast_exp2(-(t2 * t2) * c2);
              const float fe = (v - skyf) * (in ? w : 0.0f);
              b0 += fe;
              b1 = fmaf(fe, t2, b1);
            }
            s0 += (double)b0;
            s1 += (double)b1;
          }
          const double wx = (double)fast_exp2(-(t1 * t1) * c2);
          N += wx * s0;
          Sx += wx * (double)t1 * s0;
          Sy += wx * s1;
        }
      }
    };
    int it = 0;
    while (it < o.max_iter_centroid) {
      double N, Sx, Sy;
      sweep(N, Sx, Sy);
      {
        double u[4] = {N, Sx, Sy, 0.0};
        wave_sum_n(u);
        N = u[0];
        Sx = u[1];
        Sy = u[2];
      }
      ++it;
      if (!(N > 0.0)) {
        stt |= SHAPE_ST_NONPOSITIVE_FLUX;
        break;
      }
      const double iN = rcp_f64(o.k_gain * N);   // N > 0 here
      double dx = Sx * iN, dy = Sy * iN;
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
      out[SHAPE_REC_SIZE] = qnan();
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
