// Front end on whole frames (Sec. 4.1, the paragraph on the starting point):
// the brightest pixel of each frame, r50 by summing the pixels outward from
// it until half the total flux, and the square of side 6 r50 around it cut
// out into a packed stamp batch.
//
// One workgroup per frame for detection:
//   pass 0  border mean -> sky (FP64, fixed reduction order);
//   pass 1  one read of the frame: finiteness, brightest pixel (first index
//           among equals), total F = sum (I - sky) in FP64, max |I - sky|;
//   pass 2  ring sums about the peak over a square window of half-size R
//           (R = 16, 32, ... until the growth curve crosses F/2 or the window
//           covers the frame), in fixed point (int64 LDS atomics with a
//           power-of-two scale from max |I - sky|, so the sums do not depend
//           on the order of the atomics), rings r - 1 < d <= r, the peak
//           pixel counted with ring 1;
// then the crossing radius is interpolated and the box placed.  A frame is
// read about once: pass 2 touches only the window, typically a few r50.
#include "kernels.hpp"

namespace shape {
namespace {

constexpr int kFrameThreads = 256;
constexpr int kFrameWaves = kFrameThreads / kWave;
constexpr int kR0 = 16;

template <int DT>
__device__ __forceinline__ float frame_px(const shape_frames& f, int64_t base, int64_t k,
                                          float scale) {
  if constexpr (DT == SHAPE_F32) {
    return static_cast<const float*>(f.pixels)[base + k];
  } else {
    return static_cast<float>(static_cast<const _Float16*>(f.pixels)[base + k]) * scale;
  }
}

// Four consecutive pixels from a 4-aligned index (frames whose pixel count
// is a multiple of 4 on a 16-byte aligned buffer).
template <int DT>
__device__ __forceinline__ void load4(const shape_frames& f, int64_t base, int64_t k, float scale,
                                      float (&v)[4]) {
  if constexpr (DT == SHAPE_F32) {
    const float4 q = *reinterpret_cast<const float4*>(static_cast<const float*>(f.pixels) + base + k);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  } else {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    const h4 q = *reinterpret_cast<const h4*>(static_cast<const _Float16*>(f.pixels) + base + k);
    v[0] = (float)q[0] * scale;
    v[1] = (float)q[1] * scale;
    v[2] = (float)q[2] * scale;
    v[3] = (float)q[3] * scale;
  }
}

// Sum over the workgroup in a fixed order (wave DPP sums, then waves 0..3).
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x, w = tid / kWave;
  v = wave_sum(v);
  __syncthreads();
  if ((tid & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kFrameWaves; ++q) s += red[q];
  return s;
}

// Smallest r >= 0 with r^2 >= d2.
__device__ __forceinline__ int ceil_sqrt(int64_t d2) {
  int r = (int)ceil(sqrt((double)d2));
  while ((int64_t)r * r < d2) ++r;
  while (r > 0 && (int64_t)(r - 1) * (r - 1) >= d2) --r;
  return r;
}

template <int DT>
__global__ __launch_bounds__(kFrameThreads) void detect_kernel(shape_frames f, int max_side,
                                                               int nbins, bool vec4, float* info,
                                                               int32_t* peak, int32_t* box,
                                                               uint32_t* status) {
  extern __shared__ long long bins[];   // nbins
  __shared__ double red[kFrameWaves];
  __shared__ float bval[kFrameThreads];
  __shared__ int64_t bidx[kFrameThreads];
  __shared__ int found_r;
  __shared__ double found_prev, found_cum;
  const int tid = threadIdx.x;
  const int H = f.height, W = f.width;
  const int64_t npix = (int64_t)H * W;
  for (int64_t fr = blockIdx.x; fr < f.n; fr += gridDim.x) {
    const int64_t base = fr * npix;
    const float scale = (DT == SHAPE_F16_SCALED) ? f.scale[fr] : 1.0f;
    // pass 0: border mean
    const int nb = 2 * W + 2 * H - 4;
    double bs = 0.0;
    for (int q = tid; q < nb; q += kFrameThreads) {
      int64_t k;
      if (q < W) k = q;                                   // top row
      else if (q < 2 * W) k = (int64_t)(H - 1) * W + (q - W);   // bottom row
      else {
        const int r = q - 2 * W;                          // left, right columns
        const int row = 1 + (r >> 1);
        k = (int64_t)row * W + ((r & 1) ? W - 1 : 0);
      }
      bs += (double)frame_px<DT>(f, base, k, scale);
    }
    const double sky = block_sum(bs, red) / (double)nb;
    // pass 1: finiteness, brightest pixel, total, extent
    float best = -__builtin_inff();
    int64_t bk = npix;
    bool finite = true;
    double tot = 0.0, amax = 0.0;
    auto visit = [&](float v, int64_t k) {
      finite = finite && __builtin_isfinite(v);
      if (v > best) {  // each thread's k increases: ties keep the first index
        best = v;
        bk = k;
      }
      const double d = (double)v - sky;
      tot += d;
      amax = fmax(amax, fabs(d));
    };
    if (vec4) {
      // four pixels per load (16 B FP32 / 8 B FP16), four loads in flight
      const int64_t n4 = npix >> 2;
#pragma unroll 4
      for (int64_t q = tid; q < n4; q += kFrameThreads) {
        float v[4];
        load4<DT>(f, base, q * 4, scale, v);
#pragma unroll
        for (int c = 0; c < 4; ++c) visit(v[c], q * 4 + c);
      }
    } else {
      for (int64_t k = tid; k < npix; k += kFrameThreads) visit(frame_px<DT>(f, base, k, scale), k);
    }
    const bool all_finite = __syncthreads_and(finite);
    if (!all_finite) {
      if (tid == 0) {
        info[fr * 3 + 0] = info[fr * 3 + 1] = info[fr * 3 + 2] = qnan();
        peak[fr * 2 + 0] = peak[fr * 2 + 1] = -1;
        box[fr * 3 + 0] = box[fr * 3 + 1] = box[fr * 3 + 2] = 0;
        status[fr] = SHAPE_ST_NONFINITE_INPUT;
      }
      __syncthreads();
      continue;
    }
    const double F = block_sum(tot, red);
    // max |I - sky| (exact: max is order independent)
    {
      double m = amax;
      for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
      if ((tid & (kWave - 1)) == 0) bins[tid / kWave] = __builtin_bit_cast(long long, m);
    }
    bval[tid] = best;
    bidx[tid] = bk;
    __syncthreads();
    for (int s = kFrameThreads / 2; s >= 1; s >>= 1) {
      if (tid < s) {
        const float v2 = bval[tid + s];
        const int64_t k2 = bidx[tid + s];
        if (v2 > bval[tid] || (v2 == bval[tid] && k2 < bidx[tid])) {
          bval[tid] = v2;
          bidx[tid] = k2;
        }
      }
      __syncthreads();
    }
    double mabs = 0.0;
#pragma unroll
    for (int q = 0; q < kFrameWaves; ++q)
      mabs = fmax(mabs, __builtin_bit_cast(double, bins[q]));
    const int64_t pk = bidx[0];
    const int i0 = (int)(pk / W), j0 = (int)(pk - (int64_t)i0 * W);
    __syncthreads();
    uint32_t stt = 0;
    const int mind = H < W ? H : W;
    double rr = 0.125 * mind;
    if (F > 0.0) {
      // fixed point: |sum| <= npix * mabs * scale < 2^62
      int ex;
      __builtin_frexp((double)npix * fmax(mabs, 1e-300), &ex);
      const double fs = __builtin_ldexp(1.0, 62 - ex);
      const double half = 0.5 * F;
      const int rmax = ceil_sqrt((int64_t)(H - 1) * (H - 1) + (int64_t)(W - 1) * (W - 1));
      int R = kR0;
      for (;;) {
        if (R > rmax) R = rmax;
        const int Rc = R + 1 < nbins ? R + 1 : nbins;
        for (int q = tid; q < Rc; q += kFrameThreads) bins[q] = 0;
        if (tid == 0) found_r = -1;
        __syncthreads();
        const int ia = i0 - R > 0 ? i0 - R : 0, ib = i0 + R < H - 1 ? i0 + R : H - 1;
        const int ja = j0 - R > 0 ? j0 - R : 0, jb = j0 + R < W - 1 ? j0 + R : W - 1;
        const int ww = jb - ja + 1;
        const int nw = (ib - ia + 1) * ww;   // < 2^31 for sides up to 4096
        const int64_t R2 = (int64_t)R * R;
        for (int q = tid; q < nw; q += kFrameThreads) {
          const int i = ia + q / ww, j = ja + q % ww;
          const int64_t d2 = (int64_t)(i - i0) * (i - i0) + (int64_t)(j - j0) * (j - j0);
          if (d2 > R2) continue;
          const int r = ceil_sqrt(d2);
          const double d = (double)frame_px<DT>(f, base, (int64_t)i * W + j, scale) - sky;
          atomicAdd((unsigned long long*)&bins[r < 1 ? 1 : r],
                    (unsigned long long)__builtin_llrint(d * fs));
        }
        __syncthreads();
        // first crossing of F/2 by the growth curve C(r), r = 1..R (wave 0)
        if (tid < kWave) {
          long long carry = 0;
          for (int c0 = 1; c0 <= R; c0 += kWave) {
            const int r = c0 + tid;
            long long v = r <= R ? bins[r] : 0;
            // inclusive scan over the wave
            for (int o = 1; o < kWave; o <<= 1) {
              const long long u = __shfl_up(v, o);
              if (tid >= o) v += u;
            }
            const long long cum = carry + v;
            const bool hit = r <= R && (double)cum / fs >= half;
            const unsigned long long m = __ballot(hit);
            if (m) {
              const int l = __builtin_ctzll(m);
              if (tid == l) {
                const long long prev = cum - bins[r];
                found_r = r;
                found_prev = (r == 1) ? 0.0 : (double)prev / fs;
                found_cum = (double)cum / fs;
              }
              break;
            }
            carry += __shfl(v, kWave - 1);
          }
        }
        __syncthreads();
        const int fr_r = found_r;
        if (fr_r > 0) {
          rr = (fr_r - 1) + (half - found_prev) / (found_cum - found_prev);
          break;
        }
        if (R >= rmax) {
          // rounding left the last ring a hair short of F/2: it crosses there
          rr = (double)rmax;
          break;
        }
        R *= 2;
        __syncthreads();
      }
    } else {
      stt |= SHAPE_ST_NONPOSITIVE_FLUX;
    }
    if (tid == 0) {
      int smax = max_side < mind ? max_side : mind;
      long long side = __builtin_llround(6.0 * rr);
      if (side < 4) side = 4;
      if (side > smax) side = smax;
      int ox = j0 - (int)side / 2, oy = i0 - (int)side / 2;
      if (ox > W - side) ox = W - (int)side;
      if (oy > H - side) oy = H - (int)side;
      if (ox < 0) ox = 0;
      if (oy < 0) oy = 0;
      info[fr * 3 + 0] = (float)sky;
      info[fr * 3 + 1] = (float)rr;
      info[fr * 3 + 2] = (float)F;
      peak[fr * 2 + 0] = j0;
      peak[fr * 2 + 1] = i0;
      box[fr * 3 + 0] = ox;
      box[fr * 3 + 1] = oy;
      box[fr * 3 + 2] = (int)side;
      status[fr] = stt;
    }
    __syncthreads();
  }
}

// Exclusive prefix sum of side^2 over the boxes (one workgroup of 1024).
__global__ __launch_bounds__(1024) void offsets_kernel(const int32_t* box, int64_t n,
                                                       int64_t* offset, int64_t* total) {
  __shared__ long long part[1024 / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  long long carry = 0;
  for (int64_t c0 = 0; c0 < n; c0 += 1024) {
    const int64_t k = c0 + tid;
    const long long s = k < n ? (long long)box[k * 3 + 2] : 0;
    long long v = s * s;
    for (int o = 1; o < kWave; o <<= 1) {
      const long long u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    if (lane == kWave - 1) part[w] = v;
    __syncthreads();
    long long before = 0, all = 0;
    for (int q = 0; q < 1024 / kWave; ++q) {
      if (q < w) before += part[q];
      all += part[q];
    }
    if (k < n) offset[k] = carry + before + v - s * s;
    carry += all;
    __syncthreads();
  }
  if (tid == 0) *total = carry;
}

// Copy each box into the packed stamps (FP32), one workgroup per frame.
// A box outside its frame, or whose cut-out would not fit in the capacity,
// copies nothing and gets side 0 (its stamp is then rejected downstream).
template <int DT>
__global__ __launch_bounds__(kFrameThreads) void cut_kernel(shape_frames f, const int32_t* box,
                                                            const int64_t* offset, float* stamps,
                                                            int64_t capacity, int32_t* sides) {
  const int W = f.width;
  const int64_t npix = (int64_t)f.height * W;
  for (int64_t fr = blockIdx.x; fr < f.n; fr += gridDim.x) {
    const int ox = box[fr * 3 + 0], oy = box[fr * 3 + 1];
    int s = box[fr * 3 + 2];
    const int64_t o0 = offset[fr];
    const bool fits = s > 0 && ox >= 0 && oy >= 0 && ox <= W - s && oy <= f.height - s &&
                      o0 >= 0 && o0 <= capacity - (int64_t)s * s;
    if (!fits) s = 0;
    if (threadIdx.x == 0 && sides) sides[fr] = s;
    if (s == 0) continue;
    const float scale = (DT == SHAPE_F16_SCALED) ? f.scale[fr] : 1.0f;
    const int64_t base = fr * npix + (int64_t)oy * W + ox, o = o0;
    const int n = s * s;
    for (int q = threadIdx.x; q < n; q += kFrameThreads) {
      const int i = q / s, j = q - i * s;
      stamps[o + q] = frame_px<DT>(f, base, (int64_t)i * W + j, scale);
    }
  }
}

}  // namespace

int frame_bins(int height, int width) {
  // rings 0 .. ceil(sqrt((H-1)^2 + (W-1)^2))
  const double d = sqrt((double)(height - 1) * (height - 1) + (double)(width - 1) * (width - 1));
  return (int)ceil(d) + 2;
}

hipError_t launch_frame_detect(const shape_frames& f, int max_side, float* info, int32_t* peak,
                               int32_t* box, uint32_t* status, hipStream_t stream) {
  const int nbins = frame_bins(f.height, f.width);
  const size_t lds = (size_t)nbins * sizeof(long long);
  const int64_t grid = f.n < (1ll << 30) ? f.n : (1ll << 30);
  const int64_t npix = (int64_t)f.height * f.width;
  const size_t align = f.dtype == SHAPE_F32 ? 16 : 8;
  const bool vec4 = npix % 4 == 0 && reinterpret_cast<uintptr_t>(f.pixels) % align == 0;
  if (f.dtype == SHAPE_F32)
    hipLaunchKernelGGL(detect_kernel<SHAPE_F32>, dim3((unsigned)grid), dim3(kFrameThreads), lds,
                       stream, f, max_side, nbins, vec4, info, peak, box, status);
  else
    hipLaunchKernelGGL(detect_kernel<SHAPE_F16_SCALED>, dim3((unsigned)grid), dim3(kFrameThreads),
                       lds, stream, f, max_side, nbins, vec4, info, peak, box, status);
  return hipGetLastError();
}

hipError_t launch_frame_offsets(const int32_t* box, int64_t n, int64_t* offset, int64_t* total,
                                hipStream_t stream) {
  hipLaunchKernelGGL(offsets_kernel, dim3(1), dim3(1024), 0, stream, box, n, offset, total);
  return hipGetLastError();
}

hipError_t launch_frame_cut(const shape_frames& f, const int32_t* box, const int64_t* offset,
                            float* stamps, int64_t capacity, int32_t* sides, hipStream_t stream) {
  const int64_t grid = f.n < (1ll << 30) ? f.n : (1ll << 30);
  if (f.dtype == SHAPE_F32)
    hipLaunchKernelGGL(cut_kernel<SHAPE_F32>, dim3((unsigned)grid), dim3(kFrameThreads), 0,
                       stream, f, box, offset, stamps, capacity, sides);
  else
    hipLaunchKernelGGL(cut_kernel<SHAPE_F16_SCALED>, dim3((unsigned)grid), dim3(kFrameThreads), 0,
                       stream, f, box, offset, stamps, capacity, sides);
  return hipGetLastError();
}

}  // namespace shape
