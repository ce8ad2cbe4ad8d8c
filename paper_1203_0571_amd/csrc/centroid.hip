// Starting estimates and the circular-weight centroid.
//
// Sec. 4.1 (starting point): the brightest pixel, and r50 from the growth
// curve about it; Sec. 2: Gaussian-weighted first moments, the centre moving
// by (<x>/N)/k with the fixed gain k.
//
// Two forms, both reading each stamp from memory once into registers:
// centroid_kernel for a batch of one side that divides 64 (one wave per
// stamp, pixel l + 64 m in slot m of lane l), centroid_any_kernel for any
// side (a SlotMap column layout; one wave per stamp up to side 64, a team of
// three or four waves above).
#include "slots.hpp"
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

// The growth curve in fixed point: f = I - sky0 times fix, rounded to an
// integer, with fix a power of two such that |f| fix < 2^50 (so kRoundMagic
// rounds it) and |f| fix npix < 2.3e18 (so twice a sum fits in 63 bits).  The
// ring sums are then exact and do not depend on the order lanes add in.
struct FixedPoint {
  double fix, kofs;
  long long magic_bits;
  __device__ FixedPoint(double amax, double sky0, int npix) {
    const double fmaxabs = amax + fabs(sky0) + 1.0;
    fix = ldexp(1.0, ilogb(fmin(2.3e18 / (double)npix, 0x1p50) / fmaxabs));
    // (I - sky0) fix + magic in one FMA: fix * I + (magic - sky0 fix)
    kofs = kRoundMagic - sky0 * fix;
    magic_bits = __builtin_bit_cast(long long, kRoundMagic);
  }
  __device__ __forceinline__ void deposit(unsigned long long* ring, float v, int d2) const {
    const double t = fma((double)v, fix, kofs);
    const long long q = __builtin_bit_cast(long long, t) - magic_bits;
    atomicAdd(&ring[ring_of(d2)], (unsigned long long)q);
  }
};

// r50: the first ring r >= 1 where the cumulative fixed-point flux reaches
// half the total, interpolated linearly over [r - 1, r] (rings 0 and 1
// together span [0, 1]).  Lane l takes rings 3l .. 3l + 2 (nrings <= 192), a
// wave scan gives every ring's cumulative sum, and a ballot finds the first
// crossing; every lane of the wave gets the same values.
__device__ inline double r50_from_rings(const unsigned long long* ring, int nrings, int W,
                                        long long& F, uint32_t& stt) {
  const int lane = threadIdx.x & (kWave - 1), r0 = 3 * lane;
  const long long a0 = r0 < nrings ? (long long)ring[r0] : 0;
  const long long a1 = r0 + 1 < nrings ? (long long)ring[r0 + 1] : 0;
  const long long a2 = r0 + 2 < nrings ? (long long)ring[r0 + 2] : 0;
  const long long loc = a0 + a1 + a2;
  const long long incl = wave_total(loc);   // inclusive scan over the lanes
  F = readlane64(incl, kWave - 1);
  if (!(F > 0)) {
    stt |= SHAPE_ST_NONPOSITIVE_FLUX;
    return 0.125 * W;
  }
  const long long e = incl - loc, c0 = e + a0, c1 = c0 + a1, c2 = c1 + a2;
  const bool h0 = r0 >= 1 && r0 < nrings && 2 * c0 >= F;
  const bool h1 = r0 + 1 < nrings && 2 * c1 >= F;
  const bool h2 = r0 + 2 < nrings && 2 * c2 >= F;
  // the last ring's sum is F > 0, so some lane crosses
  const int L = __builtin_ctzll(__ballot(h0 || h1 || h2));
  const long long cum = h0 ? c0 : h1 ? c1 : c2, before = h0 ? e : h1 ? c0 : c1;
  const int r = __builtin_amdgcn_readlane(r0 + (h0 ? 0 : h1 ? 1 : 2), L);
  const long long cr = readlane64(cum, L), pr = r == 1 ? 0 : readlane64(before, L);
  return (r - 1) + (0.5 * (double)F - (double)pr) / (double)(cr - pr);
}

// One centroid step from the summed N, Sx, Sy (Sec. 2): x += Sx / (k N).
// Returns true when the iteration stops (status bits in stt).
__device__ __forceinline__ bool centroid_step(double N, double Sx, double Sy, double& x, double& y,
                                              int W, const KOpts& o, uint32_t& stt) {
  if (!(N > 0.0)) {
    stt |= SHAPE_ST_NONPOSITIVE_FLUX;
    return true;
  }
  const double iN = rcp_f64(o.k_gain * N);   // N > 0 here
  const double dx = Sx * iN, dy = Sy * iN;
  x += dx;
  y += dy;
  if (x < 0.0 || y < 0.0 || x > W - 1 || y > W - 1) {
    stt |= SHAPE_ST_LOST;
    return true;
  }
  if (fabs(dx) < o.tol_x && fabs(dy) < o.tol_x) {
    stt |= SHAPE_ST_CONVERGED;
    return true;
  }
  return false;
}

__device__ inline void write_record(float* out, double x, double y, double sigw, double r50,
                                    double sky0, double flux, int it, uint32_t stt,
                                    int32_t* iters, uint32_t* status, int64_t s) {
  out[SHAPE_REC_X0] = (float)x;
  out[SHAPE_REC_Y0] = (float)y;
  out[SHAPE_REC_E1] = 0.0f;
  out[SHAPE_REC_E2] = 0.0f;
  out[SHAPE_REC_SIGW] = (float)sigw;
  out[SHAPE_REC_R50] = (float)r50;
  out[SHAPE_REC_SKY0] = (float)sky0;
  out[SHAPE_REC_FLUX] = (float)flux;
  out[SHAPE_REC_SIZE] = qnan();
  iters[s] = it;
  status[s] = stt;
}

__device__ inline void write_failed(float* out, int t, int32_t* iters, uint32_t* status, int64_t s,
                                    uint32_t why) {
  if (t < SHAPE_REC_LEN) out[t] = qnan();
  if (t == 0) {
    iters[s] = 0;
    status[s] = why;
  }
}

// The weight's scale from r50: sigma_w = r50 / sqrt(2 ln 2), kept in [1, W / 4].
__device__ __forceinline__ double weight_sigma(double r50, int W) {
  const double sigw = r50 / sqrt(2.0 * kLn2);
  return fmin(fmax(sigw, 1.0), 0.25 * W);
}

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
  static_assert(SIDE == 8 || SIDE == 16 || SIDE == 32 || SIDE == 64, "side must divide 64");
  __shared__ unsigned long long ring[kMaxRings];
  __shared__ float wy_row[kWave];   // the weight's row factor
  const int lane = threadIdx.x;
  for (int64_t s = blockIdx.x; s < b.n; s += gridDim.x) {
    const Stamp st = stamp_info(b, s);
    float* out = rec + s * SHAPE_REC_LEN;
    if (st.bad) {
      write_failed(out, lane, iters, status, s, st.bad);
      continue;
    }
    constexpr int W = SIDE;
    constexpr int kSlots = StampPixels<DT, SIDE>::kSlots;
    constexpr int kR = kWave / SIDE;   // rows between a lane's slots
    StampPixels<DT, SIDE> px(b, st, lane);
    const int il = lane / SIDE, jl = lane & (SIDE - 1);

    // Pass 1: finiteness, border sum, brightest pixel, largest |I|.
    double border = 0.0;
    float best = -__builtin_huge_valf();
    int besti = 0x7fffffff;
    bool nonfinite = false;
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
    float amax = fmaxf(fabsf(best), fabsf(vmin));  // max |I| = max(max I, -min I)
    // the border: whole columns 0 and W - 1, the rest of rows 0 and W - 1
    if (jl == 0 || jl == SIDE - 1) {
#pragma unroll
      for (int m = 0; m < kSlots; ++m) border += (double)px.v[m];
    } else {
      if (il == 0) border += (double)px.v[0];
      if (il == kR - 1) border += (double)px.v[kSlots - 1];
    }
    if (wave_any(nonfinite)) {
      write_failed(out, lane, iters, status, s, SHAPE_ST_NONFINITE_INPUT);
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

    // Pass 2: ring sums of f = I - sky0 about the brightest pixel.
    const int nrings = ring_of(2 * (W - 1) * (W - 1)) + 1;
    const FixedPoint fp((double)amax, sky0, st.npix);
    for (int r = lane; r < nrings; r += kWave) ring[r] = 0ull;
    __syncthreads();
    {
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
          fp.deposit(ring, v[q], __mul24(di, di) + dj2);
        }
      }
    }
    __syncthreads();
    long long F;
    uint32_t stt = 0;
    const double r50 = r50_from_rings(ring, nrings, W, F, stt);
    __syncthreads();  // ring[] is reused by the next stamp of this wave
    const double sigw = weight_sigma(r50, W);

    // Pass 3: centroid iteration from the brightest pixel.
    double x = j0, y = i0;
    const float c2 = (float)(kLog2e / (2.0 * sigw * sigw));
    const float skyf = (float)sky0;
    // the register stamp becomes f = I - sky0 once, for every step
#pragma unroll
    for (int m = 0; m < kSlots; ++m) px.v[m] -= skyf;
    int it = 0;
    while (it < o.max_iter_centroid) {
      // Sums N = sum f W, Sx = sum f W theta1, Sy = sum f W theta2 about
      // (x, y).  A lane holds one column (jl) at rows il + kR m.  The
      // circular weight factors as W = wx(theta1) wy(theta2), so the lane
      // sums f wy and f wy theta2 down its column and applies wx (and
      // theta1) once; the column sums run in FP32 over blocks of up to 8 rows
      // and in FP64 across blocks and lanes.  The row factor wy is the same
      // for every column: lane r forms it for row r and the wave reads it
      // back from LDS.
      const float xf = (float)x, yf = (float)y;
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
      double u[4] = {wx * s0, wx * (double)t1 * s0, wx * (dl * s0 + (double)kR * s1), 0.0};
      wave_sum_n(u);
      ++it;
      if (centroid_step(u[0], u[1], u[2], x, y, W, o, stt)) break;
    }
    if (!(stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_LOST)))
      stt |= SHAPE_ST_MAX_ITER;
    if (lane == 0)
      write_record(out, x, y, sigw, r50, sky0, (double)F / fp.fix, it, stt, iters, status, s);
  }
}

// Two 32 x 32 stamps per wave (stamps 2 w and 2 w + 1 of workgroup w's turn;
// lanes 32 g + j hold column j of stamp g, all 32 rows): the same three passes
// as centroid_kernel with every reduction taken per half-wave, and the
// iteration running until both stamps stop (a stopped stamp's lanes idle).
// A lane then sums 32 pixels per step, where the one-stamp form sums 16 and
// each stamp's step pays the whole wave's reductions.
constexpr int kPairRings = 48;   // ring_of(2 * 31^2) + 1 = 45, rounded up
template <int DT>
__global__ __launch_bounds__(kWave, 5) void centroid_pair_kernel(shape_batch b, KOpts o,
                                                                 float* rec, int32_t* iters,
                                                                 uint32_t* status) {
  constexpr int W = kPairSide, kSlots = kPairSide;
  __shared__ unsigned long long ring[2 * kPairRings];
  __shared__ float wy_row[2 * W];
  const int lane = threadIdx.x, g = lane >> 5, jl = lane & (W - 1);
  const bool hi = g != 0;
  for (int64_t s0 = 2 * (int64_t)blockIdx.x; s0 < b.n; s0 += 2 * (int64_t)gridDim.x) {
    const int64_t s = s0 + g < b.n ? s0 + g : s0;   // a missing second stamp repeats the first
    const bool own = s0 + g < b.n;                  // and writes nothing
    const Stamp st = stamp_info(b, s);
    float* out = rec + s * SHAPE_REC_LEN;
    float v[kSlots];
    {
      const void* sp = stamp_base<DT>(b, st);
      const bool ok = !st.bad;
#pragma unroll
      for (int m = 0; m < kSlots; ++m)
        v[m] = ok ? load_rel<DT>(sp, (uint32_t)(m * W + jl), st.scale) : 0.0f;
    }
    // Pass 1: finiteness, border sum, brightest pixel, largest |I|.
    double border = 0.0;
    float best = -__builtin_huge_valf(), vmin = __builtin_huge_valf();
    int besti = 0x7fffffff;
    bool nonfinite = false;
#pragma unroll
    for (int m = 0; m < kSlots; ++m) {
      nonfinite |= !__builtin_isfinite(v[m]);
      if (v[m] > best) {  // the index increases with m, so ties keep the lowest
        best = v[m];
        besti = m * W + jl;
      }
      vmin = fminf(vmin, v[m]);
    }
    float amax = fmaxf(fabsf(best), fabsf(vmin));
    if (jl == 0 || jl == W - 1) {
#pragma unroll
      for (int m = 0; m < kSlots; ++m) border += (double)v[m];
    } else {
      border = (double)v[0] + (double)v[kSlots - 1];
    }
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) {
      const float ov = __shfl_xor(best, m, kWave);
      const int oi = __shfl_xor(besti, m, kWave);
      if (ov > best || (ov == best && oi < besti)) {
        best = ov;
        besti = oi;
      }
      amax = fmaxf(amax, __shfl_xor(amax, m, kWave));
    }
    {
      double bu[2] = {border, 0.0};
      half_sum_n(bu);
      border = bu[0];
    }
    uint32_t stt = st.bad ? st.bad : (half_any(nonfinite) ? SHAPE_ST_NONFINITE_INPUT : 0u);
    const bool live = stt == 0u;
    const double sky0 = border / (4.0 * W - 4.0);
    const int i0 = besti / W, j0 = besti - (besti / W) * W;

    // Pass 2: ring sums of f = I - sky0 about the brightest pixel, per half.
    constexpr int nrings = 45;   // ring_of(2 * (W - 1)^2) + 1
    unsigned long long* rg = ring + g * kPairRings;
    const FixedPoint fp((double)amax, sky0, st.npix);
    for (int r = jl; r < kPairRings; r += W) rg[r] = 0ull;
    __syncthreads();
    if (live) {
      const int dj2 = __mul24(jl - j0, jl - j0);
#pragma unroll
      for (int m0 = 0; m0 < kSlots; m0 += 8) {
        float w8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) w8[q] = v[m0 + q];
        asm volatile("" : "+v"(w8[0]), "+v"(w8[1]), "+v"(w8[2]), "+v"(w8[3]), "+v"(w8[4]),
                     "+v"(w8[5]), "+v"(w8[6]), "+v"(w8[7])
                     :
                     : "memory");
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int di = m0 + q - i0;
          fp.deposit(rg, w8[q], __mul24(di, di) + dj2);
        }
      }
    }
    __syncthreads();
    // r50 per half: lane j takes rings 3 j .. 3 j + 2 of its stamp
    long long F;
    double r50;
    {
      const int r0 = 3 * jl;
      const long long a0 = r0 < nrings ? (long long)rg[r0] : 0;
      const long long a1 = r0 + 1 < nrings ? (long long)rg[r0 + 1] : 0;
      const long long a2 = r0 + 2 < nrings ? (long long)rg[r0 + 2] : 0;
      const long long loc = a0 + a1 + a2;
      const long long incl = half_scan(loc);
      F = half_pick(incl, 31, 63);
      const long long e = incl - loc, c0 = e + a0, c1 = c0 + a1, c2 = c1 + a2;
      const bool h0 = r0 >= 1 && r0 < nrings && 2 * c0 >= F;
      const bool h1 = r0 + 1 < nrings && 2 * c1 >= F;
      const bool h2 = r0 + 2 < nrings && 2 * c2 >= F;
      const uint64_t m = __ballot(F > 0 && (h0 || h1 || h2));
      const uint32_t m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
      // (a half with F > 0 crosses at its last ring; the other half's lane
      // index is then unused)
      const int L0 = m0 ? __builtin_ctz(m0) : 0, L1 = 32 + (m1 ? __builtin_ctz(m1) : 0);
      const long long cum = h0 ? c0 : h1 ? c1 : c2, before = h0 ? e : h1 ? c0 : c1;
      const int r = half_pick(r0 + (h0 ? 0 : h1 ? 1 : 2), L0, L1);
      const long long cr = half_pick(cum, L0, L1), pr = r == 1 ? 0 : half_pick(before, L0, L1);
      if (F > 0) {
        r50 = (r - 1) + (0.5 * (double)F - (double)pr) / (double)(cr - pr);
      } else {
        stt |= live ? SHAPE_ST_NONPOSITIVE_FLUX : 0u;
        r50 = 0.125 * W;
      }
    }
    __syncthreads();  // ring[] is reused by the next pair of stamps
    const double sigw = weight_sigma(r50, W);

    // Pass 3: centroid iterations from the brightest pixels; a lane sums f wy
    // and f wy theta2 down its column (as centroid_kernel, one slot per row).
    double x = j0, y = i0;
    const float c2 = (float)(kLog2e / (2.0 * sigw * sigw));
    const float skyf = (float)sky0;
#pragma unroll
    for (int m = 0; m < kSlots; ++m) v[m] -= skyf;
    bool done = !live || !own;
    int it = 0;
    for (int step = 0; step < o.max_iter_centroid; ++step) {
      if (!__any(!done)) break;
      const float xf = (float)x, yf = (float)y;
      constexpr int kC = kSlots / 2;
      wave_sync();  // the previous step's reads of wy_row are done
      {
        const float tr = (float)jl - yf;
        wy_row[lane] = fast_exp2(-(tr * tr) * c2);
      }
      wave_sync();
      float jlf = (float)jl;
      asm volatile("" : "+v"(jlf));
      const float t1 = jlf - xf;
      const float* wy = wy_row + g * W;
      double s0d = 0.0, s1d = 0.0;
#pragma unroll
      for (int m0 = 0; m0 < kSlots; m0 += kColumnBlock) {
        float b0 = 0.0f, b1 = 0.0f;
#pragma unroll
        for (int m = m0; m < m0 + kColumnBlock; ++m) {
          const float fe = v[m] * wy[m];
          b0 += fe;
          b1 = fmaf(fe, (float)(m - kC), b1);
        }
        s0d += (double)b0;
        s1d += (double)b1;
      }
      const double wx = (double)fast_exp2(-(t1 * t1) * c2);
      const double dl = (double)kC - y;
      double u[4] = {wx * s0d, wx * (double)t1 * s0d, wx * (dl * s0d + s1d), 0.0};
      half_sum_n(u);
      if (!done) {
        ++it;
        done = centroid_step(u[0], u[1], u[2], x, y, W, o, stt);
      }
    }
    if (live && !(stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_LOST)))
      stt |= SHAPE_ST_MAX_ITER;
    if (own && jl == 0) {
      if (live)
        write_record(out, x, y, sigw, r50, sky0, (double)F / fp.fix, it, stt, iters, status, s);
    }
    if (own && !live) write_failed(out, jl, iters, status, s, stt);
  }
}

// LDS of the any-side form.
template <int TEAM>
struct AnyShared {
  unsigned long long ring[kMaxRings];
  float wy_row[kRowTable];          // the weight's row factor (0 past the stamp)
  double part[2 * TEAM * 4];        // a team's per-wave step sums
  struct Pass1 {
    double border;
    float best, amax;
    int besti, nonfinite;
  } p1[TEAM];
};

// One stamp of the any-side form, its slots unrolled K wide.
template <int DT, int TEAM, int K>
__device__ __forceinline__ void centroid_any(const shape_batch& b, const KOpts& o, const Stamp& st,
                                             int64_t s, float* rec, int32_t* iters,
                                             uint32_t* status, AnyShared<TEAM>& sh, int& parity) {
  const int t = threadIdx.x, lane = t & (kWave - 1);
  float* out = rec + s * SHAPE_REC_LEN;
  const SlotMap<TEAM> mp(st.side, t);
  constexpr int RC = fixed_rows_groups<TEAM, K>();
  const int W = mp.W, R = RC ? RC : mp.R, il = mp.il, jl = mp.jl, rows = mp.rows;
  float v[K];
  load_slots<DT, TEAM, K>(v, stamp_base<DT>(b, st), mp, st.scale);

  // Pass 1: finiteness, border sum, brightest pixel (lowest index on ties),
  // largest |I|, over the pixels of the stamp.
  double border = 0.0;
  float best = -__builtin_huge_valf(), amax = 0.0f;
  int besti = 0x7fffffff;
  bool nonfinite = false;
  {
    const bool bcol = jl == 0 || jl == W - 1;
#pragma unroll
    for (int m0 = 0; m0 < K; m0 += kColumnBlock) {
      if (m0 < rows) {
#pragma unroll
        for (int m = m0; m < m0 + kColumnBlock; ++m) {
          // selects, not branches: a slot outside the stamp changes nothing
          const bool ok = mp.valid(m);
          const float x = v[m];
          const int i = mp.row(m);
          nonfinite |= ok && !__builtin_isfinite(x);
          const float xb = ok ? x : -__builtin_huge_valf();
          if (xb > best) {  // a lane's index increases with m
            best = xb;
            besti = i * W + jl;
          }
          amax = fmaxf(amax, ok ? fabsf(x) : 0.0f);
          border += (ok && (bcol || i == 0 || i == W - 1)) ? (double)x : 0.0;
        }
      }
    }
  }
  const bool bad = TEAM > 1 ? false : wave_any(nonfinite);
  if (TEAM == 1 && bad) {
    write_failed(out, t, iters, status, s, SHAPE_ST_NONFINITE_INPUT);
    return;
  }
  border = wave_sum(border);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const float ov = __shfl_xor(best, m, kWave);
    const int oi = __shfl_xor(besti, m, kWave);
    if (ov > best || (ov == best && oi < besti)) {
      best = ov;
      besti = oi;
    }
    amax = fmaxf(amax, __shfl_xor(amax, m, kWave));
  }
  if constexpr (TEAM > 1) {
    const int nf = wave_any(nonfinite) ? 1 : 0;
    const int w = t / kWave;
    if (lane == 0) sh.p1[w] = {border, best, amax, besti, nf};
    __syncthreads();
    border = sh.p1[0].border;
    best = sh.p1[0].best;
    amax = sh.p1[0].amax;
    besti = sh.p1[0].besti;
    int anynf = sh.p1[0].nonfinite;
#pragma unroll
    for (int q = 1; q < TEAM; ++q) {
      const auto& p = sh.p1[q];
      border += p.border;
      if (p.best > best || (p.best == best && p.besti < besti)) {
        best = p.best;
        besti = p.besti;
      }
      amax = fmaxf(amax, p.amax);
      anynf |= p.nonfinite;
    }
    __syncthreads();   // p1 is rewritten by the next stamp
    if (anynf) {
      write_failed(out, t, iters, status, s, SHAPE_ST_NONFINITE_INPUT);
      return;
    }
  }
  const double sky0 = border / (4.0 * W - 4.0);
  const int i0 = besti / W, j0 = besti - (besti / W) * W;

  // Pass 2: ring sums of f = I - sky0 about the brightest pixel.
  const int nrings = ring_of(2 * (W - 1) * (W - 1)) + 1;
  const FixedPoint fp((double)amax, sky0, st.npix);
  for (int r = t; r < nrings; r += kWave * TEAM) sh.ring[r] = 0ull;
  __syncthreads();
  {
    const int dj2 = __mul24(jl - j0, jl - j0);
#pragma unroll
    for (int m0 = 0; m0 < K; m0 += kColumnBlock) {
      if (m0 < rows) {
        float g[kColumnBlock];
#pragma unroll
        for (int q = 0; q < kColumnBlock; ++q) g[q] = v[m0 + q];
        asm volatile("" : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]),
                     "+v"(g[6]), "+v"(g[7])
                     :
                     : "memory");
#pragma unroll
        for (int q = 0; q < kColumnBlock; ++q) {
          const int m = m0 + q;
          const int di = mp.row(m) - i0;
          if (mp.valid(m)) fp.deposit(sh.ring, g[q], __mul24(di, di) + dj2);
        }
      }
    }
  }
  __syncthreads();
  long long F;
  uint32_t stt = 0;
  const double r50 = r50_from_rings(sh.ring, nrings, W, F, stt);
  __syncthreads();  // ring[] is reused by the next stamp
  const double sigw = weight_sigma(r50, W);

  // Pass 3: centroid iteration from the brightest pixel, with the column
  // factoring of the register form: theta2 = dl + R k down a lane's column
  // (k = m - K / 2 a constant of the unrolled slot).
  double x = j0, y = i0;
  const float c2 = (float)(kLog2e / (2.0 * sigw * sigw));
  const float skyf = (float)sky0;
#pragma unroll
  for (int m = 0; m < K; ++m) v[m] = mp.valid(m) ? v[m] - skyf : 0.0f;
  constexpr int kC = K / 2;
  const float* wy = sh.wy_row + il;
  // Rows past the stamp that a lane's unrolled blocks reach weigh 0.
  const int rtab = min(kRowTable, R * (kColumnBlock * ((rows + kColumnBlock - 1) / kColumnBlock) + 1));
  for (int r = W + t; r < rtab; r += kWave * TEAM) sh.wy_row[r] = 0.0f;
  int it = 0;
  while (it < o.max_iter_centroid) {
    const float xf = (float)x, yf = (float)y;
    // The previous step's reads of wy_row are done: a team passed the
    // barrier of its step sums after them, a wave needs them ordered.
    if constexpr (TEAM == 1) wave_sync();
    for (int r = t; r < W; r += kWave * TEAM) {
      const float tr = (float)r - yf;
      sh.wy_row[r] = fast_exp2(-(tr * tr) * c2);
    }
    team_sync<TEAM>();
    const float t1 = (float)jl - xf;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int m0 = 0; m0 < K; m0 += kColumnBlock) {
      if (m0 < rows) {
        float b0 = 0.0f, b1 = 0.0f;
#pragma unroll
        for (int m = m0; m < m0 + kColumnBlock; ++m) {
          const float fe = v[m] * wy[R * m];
          b0 += fe;
          b1 = fmaf(fe, (float)(m - kC), b1);
        }
        s0 += (double)b0;
        s1 += (double)b1;
      }
    }
    const double wx = (double)fast_exp2(-(t1 * t1) * c2);
    const double dl = (double)il + (double)(R * kC) - y;
    double u[4] = {wx * s0, wx * (double)t1 * s0, wx * (dl * s0 + (double)R * s1), 0.0};
    team_sum_n<TEAM>(u, sh.part, parity);
    ++it;
    if (centroid_step(u[0], u[1], u[2], x, y, W, o, stt)) break;
  }
  if (!(stt & (SHAPE_ST_CONVERGED | SHAPE_ST_NONPOSITIVE_FLUX | SHAPE_ST_LOST)))
    stt |= SHAPE_ST_MAX_ITER;
  if (t == 0) write_record(out, x, y, sigw, r50, sky0, (double)F / fp.fix, it, stt, iters, status, s);
}

// One form per team size (team_takes: one wave up to side 64, three waves
// for 65..96, four for 97..128); each skips the others' stamps.  Stamps that
// cannot be processed are reported by the one-wave form, or by a team form
// launched without it (take_bad).
#ifndef SHAPE_CENTROID_ANY_WAVES_PER_SIMD
#define SHAPE_CENTROID_ANY_WAVES_PER_SIMD 4
#endif
template <int DT, int TEAM>
__global__ __launch_bounds__(kWave * TEAM, SHAPE_CENTROID_ANY_WAVES_PER_SIMD) void
centroid_any_kernel(shape_batch b, KOpts o, float* rec, int32_t* iters, uint32_t* status,
                    int take_bad, int chunk) {
  __shared__ AnyShared<TEAM> sh;
  int parity = 0;
  for (int64_t s0 = (int64_t)blockIdx.x * chunk; s0 < b.n; s0 += (int64_t)gridDim.x * chunk)
  for (uint64_t mine = chunk_mask<TEAM>(b, s0, chunk, take_bad); mine; mine &= mine - 1) {
    const int64_t s = s0 + __builtin_ctzll(mine);
    const Stamp st = stamp_info(b, s);
    if (st.bad) {
      write_failed(rec + s * SHAPE_REC_LEN, threadIdx.x, iters, status, s, st.bad);
      continue;
    }
    if constexpr (TEAM > 1) {
      centroid_any<DT, TEAM, 64>(b, o, st, s, rec, iters, status, sh, parity);
    } else {
      switch (slot_class(SlotMap<TEAM>(st.side, 0).rows)) {
        case 8: centroid_any<DT, TEAM, 8>(b, o, st, s, rec, iters, status, sh, parity); break;
        case 16: centroid_any<DT, TEAM, 16>(b, o, st, s, rec, iters, status, sh, parity); break;
        case 32: centroid_any<DT, TEAM, 32>(b, o, st, s, rec, iters, status, sh, parity); break;
        default: centroid_any<DT, TEAM, 64>(b, o, st, s, rec, iters, status, sh, parity);
      }
    }
  }
}

template <int DT>
void launch_dtype(const shape_batch& b, const KOpts& o, float* rec, int32_t* iters,
                  uint32_t* status, hipStream_t stream) {
  const int64_t cap = 1ll << 30;
  const dim3 one(kWave);
  if (!b.side && register_side(b.side0)) {
    const dim3 g((unsigned)(b.n < cap ? b.n : cap));
    switch (b.side0) {
      case 8: hipLaunchKernelGGL((centroid_kernel<DT, 8>), g, one, 0, stream, b, o, rec, iters, status); break;
      case 16: hipLaunchKernelGGL((centroid_kernel<DT, 16>), g, one, 0, stream, b, o, rec, iters, status); break;
      case 32: {
        const int64_t n2 = (b.n + 1) / 2;
        hipLaunchKernelGGL((centroid_pair_kernel<DT>), dim3((unsigned)(n2 < cap ? n2 : cap)), one, 0,
                           stream, b, o, rec, iters, status);
        break;
      }
      default: hipLaunchKernelGGL((centroid_kernel<DT, 64>), g, one, 0, stream, b, o, rec, iters, status);
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
    hipLaunchKernelGGL((centroid_any_kernel<DT, 1>), grid(c), dim3(kWave), 0, stream, b, o, rec, iters, status, 1, c);
  }
  if (f3) {
    const int c = mixed ? chunk_of<3>() : 1;
    hipLaunchKernelGGL((centroid_any_kernel<DT, 3>), grid(c), dim3(3 * kWave), 0, stream, b, o, rec, iters, status, f1 ? 0 : 1, c);
  }
  if (f4) {
    const int c = mixed ? chunk_of<4>() : 1;
    hipLaunchKernelGGL((centroid_any_kernel<DT, 4>), grid(c), dim3(4 * kWave), 0, stream, b, o, rec, iters, status, f1 ? 0 : 1, c);
  }
}

}  // namespace

hipError_t launch_centroid(const shape_batch& b, const KOpts& o, float* rec, int32_t* iters,
                           uint32_t* status, hipStream_t stream) {
  if (b.dtype == SHAPE_F32)
    launch_dtype<SHAPE_F32>(b, o, rec, iters, status, stream);
  else
    launch_dtype<SHAPE_F16_SCALED>(b, o, rec, iters, status, stream);
  return hipGetLastError();
}

}  // namespace shape
