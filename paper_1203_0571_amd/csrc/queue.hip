// Work-queue form of the profile fit for batches of uneven stamps.
//
// The stamps are ordered by model (Sersic, then Moffat) and, within a model,
// largest side first (a counting sort on the device); every stamp's LM state
// lives in the caller's workspace, and a step advances every still-active
// stamp by exactly one LM trial (lm_iterate, the same code the fused kernel
// loops over).  A step is one persistent launch per model present, each
// popping stamps of its own model's range from atomic cursors: stamps at or
// above `team_min_side` are taken by the whole workgroup (TEAM waves on one
// stamp), the rest by single waves.  One kernel per model keeps each kernel's
// registers to its own sweep (a kernel holding both sweeps needs ~243 VGPRs,
// two waves per SIMD).  A hipGraph of {reset, steps} replays one LM iteration.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "lm.hpp"

namespace shape {
namespace {

// Histogram over (model, side): bucket = side for Sersic, 256 + side for
// Moffat; stamps that cannot be processed go to bucket 0 (Sersic range).
// (kBuckets, kCursors, kCursorStride, kCursorBytes: kernels.hpp)
constexpr int kChunk = 8;      // stamps per cursor pop
// Cursors per (model, phase): workgroup g pops from cursor g % kCursors, and
// cursor c hands out the chunks c, c + kCursors, c + 2 kCursors, ... of the
// range, so every cursor sees the whole size mix.  Each cursor has its own
// 128-byte line: pops on different cursors do not contend (consecutive
// workgroups also land on different XCDs).

struct QHeader {
  uint32_t reserved0, reserved1;
  uint32_t active;         // stamps still iterating after the last step
  uint32_t reserved3;
  uint32_t begin[2];       // order[begin[m], end[m]) holds model m's stamps
  uint32_t nbig[2];        // ... of which [begin[m], nbig[m]) go to teams
  uint32_t end[2];
  uint32_t pad[54];
};
static_assert(sizeof(QHeader) == 256, "header is one 256-byte block");

struct QState {
  double sums[kSums];  // current point's amplitude-profiled sums
  double p[8];
  double lambda;
  int32_t it, nsweep;
  uint32_t stt;
  int32_t done;
};
static_assert(sizeof(QState) % 64 == 0, "state rows stay 64-byte aligned");
static_assert(sizeof(QState) == kQueueStateBytes, "workspace formula and state row agree");

struct QView {
  QHeader* hdr;
  uint32_t* cursors;  // [model][phase: 0 team, 1 single][kCursors][kCursorStride]
  uint32_t* buckets;
  int32_t* order;
  QState* state;
};


__host__ __device__ inline QView view(void* ws, int64_t n) {
  char* c = static_cast<char*>(ws);
  QView v;
  v.hdr = reinterpret_cast<QHeader*>(c);
  v.cursors = reinterpret_cast<uint32_t*>(c + 256);
  c += 256 + kCursorBytes;
  v.buckets = reinterpret_cast<uint32_t*>(c);
  v.order = reinterpret_cast<int32_t*>(c + align256(kBuckets * 4));
  v.state = reinterpret_cast<QState*>(c + align256(kBuckets * 4) + align256(n * 4));
  return v;
}

__device__ inline int bucket_of(const shape_batch& b, int64_t s) {
  const Stamp st = stamp_info(b, s);
  return st.bad ? 0 : st.side + (st.model == SHAPE_MOFFAT ? 256 : 0);
}

// ---- ordering (largest side first) ----------------------------------------

__global__ void clear_kernel(QHeader* hdr, uint32_t* buckets) {
  const int t = threadIdx.x;
  if (t < 64) reinterpret_cast<uint32_t*>(hdr)[t] = 0u;
  for (int k = t; k < kBuckets; k += blockDim.x) buckets[k] = 0u;
}

// Counts per side: a histogram per workgroup in LDS, then one global atomic
// per non-empty bucket (a uniform batch would otherwise serialise every
// stamp on one address).
__global__ void hist_kernel(shape_batch b, uint32_t* buckets) {
  __shared__ uint32_t h[kBuckets];
  for (int k = threadIdx.x; k < kBuckets; k += blockDim.x) h[k] = 0u;
  __syncthreads();
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < b.n;
       s += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[bucket_of(b, s)], 1u);
  __syncthreads();
  for (int k = threadIdx.x; k < kBuckets; k += blockDim.x)
    if (h[k]) atomicAdd(&buckets[k], h[k]);
}

// One thread turns the histogram into start cursors: the Sersic range
// (largest side first, unprocessable stamps last), then the Moffat range.
__global__ void scan_kernel(QHeader* hdr, uint32_t* buckets, int team_min_side) {
  if (threadIdx.x != 0) return;
  uint32_t pos = 0;
  for (int m = 0; m < 2; ++m) {
    hdr->begin[m] = pos;
    uint32_t nbig = pos;
    for (int side = 255; side >= (m == 0 ? 0 : 1); --side) {
      const int k = side + 256 * m;
      const uint32_t c = buckets[k];
      buckets[k] = pos;
      pos += c;
      if (side >= team_min_side && side > 0) nbig = pos;
    }
    hdr->nbig[m] = nbig;
    hdr->end[m] = pos;
  }
}

// Places every stamp at its side's cursor: each workgroup counts its own
// stamps per side in LDS, reserves one range per side with a single global
// atomic, then hands out places inside its ranges with LDS atomics.
__global__ void scatter_kernel(shape_batch b, uint32_t* buckets, int32_t* order) {
  __shared__ uint32_t h[kBuckets];
  for (int k = threadIdx.x; k < kBuckets; k += blockDim.x) h[k] = 0u;
  __syncthreads();
  const int64_t s0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t ds = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = s0; s < b.n; s += ds) atomicAdd(&h[bucket_of(b, s)], 1u);
  __syncthreads();
  for (int k = threadIdx.x; k < kBuckets; k += blockDim.x)
    h[k] = h[k] ? atomicAdd(&buckets[k], h[k]) : 0u;
  __syncthreads();
  for (int64_t s = s0; s < b.n; s += ds) order[atomicAdd(&h[bucket_of(b, s)], 1u)] = (int32_t)s;
}

// ---- per-stamp work -------------------------------------------------------

// State row <-> the team's LDS block (W.sums[0] holds the current point).
template <int TEAM>
__device__ inline void load_state(const QState* q, LmShared& W, int tid) {
  team_sync<TEAM>();
  for (int k = tid; k < kSums; k += kWave * TEAM) W.sums[0][k] = q->sums[k];
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) W.L.p[k] = q->p[k];
    W.L.lambda = q->lambda;
    W.L.it = q->it;
    W.L.nsweep = q->nsweep;
    W.L.stt = q->stt;
    W.L.done = q->done;
    W.cur = 0;
  }
  team_sync<TEAM>();
}

template <int TEAM>
__device__ inline void store_state(QState* q, const LmShared& W, bool sums, int tid) {
  if (sums)
    for (int k = tid; k < kSums; k += kWave * TEAM) q->sums[k] = W.sums[W.cur][k];
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) q->p[k] = W.L.p[k];
    q->lambda = W.L.lambda;
    q->it = W.L.it;
    q->nsweep = W.L.nsweep;
    q->stt = W.L.stt;
    q->done = W.L.done;
  }
  team_sync<TEAM>();
}

__device__ inline LmState load_lm(const QState* q) {
  LmState L;
#pragma unroll
  for (int k = 0; k < 8; ++k) L.p[k] = q->p[k];
  L.lambda = q->lambda;
  L.it = q->it;
  L.nsweep = q->nsweep;
  L.stt = q->stt;
  L.done = q->done;
  return L;
}

// Starting point of one stamp (lm_start), written to its state row.
template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT = kLayoutAny>
__device__ inline void start_one(const shape_batch& b, const KOpts& o, const float* p_init,
                                 const float* rec, QState* state, int64_t s, LmShared& W,
                                 double* xs, int tid) {
  const Stamp st = stamp_info(b, s);
  QState* q = state + s;
  if (st.bad) {
    team_sync<TEAM>();
    if (tid == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k) W.L.p[k] = 0.0;
      W.L.lambda = o.lambda0;
      W.L.it = W.L.nsweep = 0;
      W.L.stt = st.bad;
      W.L.done = 1;
      W.cur = 0;
    }
    team_sync<TEAM>();
    store_state<TEAM>(q, W, false, tid);
    return;
  }
  lm_start<DT, MODEL, MASK, TEAM, LAYOUT>(b, o, st, p_init, rec, s, W, xs, tid);
  if (tid == 0 && !W.L.done && W.L.it >= o.max_iter_lm) W.L.done = 1;
  team_sync<TEAM>();
  store_state<TEAM>(q, W, true, tid);
}

// One LM trial of one stamp, state in and out of its row.  Returns whether
// the stamp is still active afterwards.
template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT = kLayoutAny>
__device__ inline bool step_one(const shape_batch& b, const KOpts& o, QState* state, int64_t s,
                                LmShared& W, double* xs, int tid) {
  QState* q = state + s;
  if (q->done) return false;
  const Stamp st = stamp_info(b, s);
  load_state<TEAM>(q, W, tid);
  lm_iterate<DT, MODEL, MASK, TEAM, LAYOUT>(b, o, st, W, xs, tid);
  if (tid == 0 && !W.L.done && W.L.it >= o.max_iter_lm) W.L.done = 1;
  team_sync<TEAM>();
  const bool active = !W.L.done;
  store_state<TEAM>(q, W, W.cur != 0, tid);
  return active;
}

// Persistent pass over one model's range of the queue: team phase over
// order[begin, nbig), then every wave on its own over order[nbig, end).
// Every workgroup leaves once both cursors have passed the end, so the grid
// always drains.  Four waves per SIMD, as the fused fit.  LAYOUT applies to
// the single-wave phase (kLayoutRows only for batches of one side that
// divides 64, as in the fused fit).
template <int DT, int MODEL, uint32_t MASK, int TEAM, bool START, int LAYOUT>
__global__ __launch_bounds__(kWave* TEAM, 4) void queue_kernel(shape_batch b, KOpts o, void* ws,
                                                               const float* p_init,
                                                               const float* rec) {
  __shared__ LmShared W[TEAM];
  __shared__ double xs[TEAM * kSums];
  __shared__ uint32_t s_idx;
  const QView v = view(ws, b.n);
  const uint32_t begin = v.hdr->begin[MODEL], end = v.hdr->end[MODEL];
  const uint32_t nbig = TEAM > 1 ? v.hdr->nbig[MODEL] : begin;
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid & (kWave - 1);
  const uint32_t cur = blockIdx.x % kCursors;
  uint32_t* big_cursor = v.cursors + ((MODEL * 2 + 0) * kCursors + cur) * kCursorStride;
  uint32_t* small_cursor = v.cursors + ((MODEL * 2 + 1) * kCursors + cur) * kCursorStride;
  uint32_t still = 0;  // active stamps seen by this thread (thread 0 / lane 0 only)
  // Stamps are popped kChunk at a time: one atomic on a shared cursor costs
  // about as much as a stamp's LM step, and most stamps of a late step are
  // already done (their rows are skipped after a flag read).
  if constexpr (TEAM > 1) {
    for (;;) {
      if (tid == 0) s_idx = atomicAdd(big_cursor, 1u);
      __syncthreads();
      const uint32_t first = begin + (s_idx * kCursors + cur) * kChunk;
      __syncthreads();
      if (first >= nbig) break;
      for (uint32_t idx = first; idx < first + kChunk && idx < nbig; ++idx) {
        const int64_t s = v.order[idx];
        if (START) {
          start_one<DT, MODEL, MASK, TEAM>(b, o, p_init, rec, v.state, s, W[0], xs, tid);
          __syncthreads();
        } else if (step_one<DT, MODEL, MASK, TEAM>(b, o, v.state, s, W[0], xs, tid)) {
          if (tid == 0) ++still;
        }
      }
    }
  }
  for (;;) {
    uint32_t first = 0;
    if (lane == 0) first = atomicAdd(small_cursor, 1u);
    first = nbig + (__builtin_amdgcn_readfirstlane(first) * kCursors + cur) * kChunk;
    if (first >= end) break;
    // lanes 0 .. kChunk-1 look up the chunk's stamps and whether they still iterate
    int32_t sl = 0;
    bool todo = false;
    if (lane < kChunk && first + lane < end) {
      sl = v.order[first + lane];
      todo = START || !v.state[sl].done;
    }
    uint64_t mask = __ballot(todo);
    while (mask) {
      const int l = __builtin_ctzll(mask);
      mask &= mask - 1;
      const int64_t s = __builtin_amdgcn_readlane(sl, l);
      if (START) {
        start_one<DT, MODEL, MASK, 1, LAYOUT>(b, o, p_init, rec, v.state, s, W[wave], nullptr,
                                              lane);
        wave_sync();
      } else if (step_one<DT, MODEL, MASK, 1, LAYOUT>(b, o, v.state, s, W[wave], nullptr, lane)) {
        if (lane == 0) ++still;
      }
    }
  }
  if (!START && lane == 0 && still) atomicAdd(&v.hdr->active, still);
}

__global__ void reset_kernel(QHeader* hdr, uint32_t* cursors) {
  const int t = threadIdx.x;
  if (t < 4 * kCursors) cursors[t * kCursorStride] = 0u;
  if (t == 0) hdr->active = 0u;
}

// Outputs from the state rows, one thread per stamp.
template <uint32_t MASK>
__global__ void finish_kernel(shape_batch b, KOpts o, void* ws, float* p_out, float* chi2,
                              float* perr, int32_t* iters, uint32_t* status, int32_t* sweeps) {
  const QView v = view(ws, b.n);
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < b.n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const Stamp st = stamp_info(b, s);
    const QState* q = v.state + s;
    LmState L = load_lm(q);
    if (st.bad) {
      for (int k = 0; k < 8; ++k) {
        p_out[s * 8 + k] = qnan();
        if (perr) perr[s * 8 + k] = qnan();
      }
      chi2[s] = qnan();
      iters[s] = 0;
      status[s] = st.bad;
      if (sweeps) sweeps[s] = 0;
      continue;
    }
    if (st.model == SHAPE_SERSIC)
      lm_finish<SHAPE_SERSIC, MASK>(o, st, L, q->sums, s, p_out, chi2, perr, iters, status,
                                    sweeps, 0);
    else
      lm_finish<SHAPE_MOFFAT, MASK>(o, st, L, q->sums, s, p_out, chi2, perr, iters, status,
                                    sweeps, 0);
  }
}

template <int DT, int MODEL, uint32_t MASK, int TEAM, bool START, int LAYOUT = kLayoutAny>
const void* queue_kernel_ptr() {
  return reinterpret_cast<const void*>(&queue_kernel<DT, MODEL, MASK, TEAM, START, LAYOUT>);
}

template <int MODEL, bool START>
const void* pick_kernel(int dtype, uint32_t mask, int team, bool rows) {
  if constexpr (MODEL == SHAPE_SERSIC) {
    if (rows && team == 1) {
      if (dtype == SHAPE_F32 && mask == kMaskAll)
        return queue_kernel_ptr<SHAPE_F32, MODEL, kMaskAll, 1, START, kLayoutRows>();
      if (dtype == SHAPE_F32 && mask == kMaskSize)
        return queue_kernel_ptr<SHAPE_F32, MODEL, kMaskSize, 1, START, kLayoutRows>();
      if (dtype == SHAPE_F16_SCALED && mask == kMaskAll)
        return queue_kernel_ptr<SHAPE_F16_SCALED, MODEL, kMaskAll, 1, START, kLayoutRows>();
      if (dtype == SHAPE_F16_SCALED && mask == kMaskSize)
        return queue_kernel_ptr<SHAPE_F16_SCALED, MODEL, kMaskSize, 1, START, kLayoutRows>();
    }
  }
#define SHAPE_Q(DT, M, T) \
  if (dtype == DT && mask == M && team == T) return queue_kernel_ptr<DT, MODEL, M, T, START>();
  SHAPE_Q(SHAPE_F32, kMaskAll, 1)
  SHAPE_Q(SHAPE_F32, kMaskAll, 2)
  SHAPE_Q(SHAPE_F32, kMaskAll, 4)
  SHAPE_Q(SHAPE_F32, kMaskSize, 1)
  SHAPE_Q(SHAPE_F16_SCALED, kMaskAll, 1)
  SHAPE_Q(SHAPE_F16_SCALED, kMaskAll, 2)
  SHAPE_Q(SHAPE_F16_SCALED, kMaskAll, 4)
  SHAPE_Q(SHAPE_F16_SCALED, kMaskSize, 1)
#undef SHAPE_Q
  return nullptr;
}

// Workgroups that fit on the device at once for this kernel (persistent grid).
hipError_t resident_grid(const void* fn, int team, int* grid) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWave * team, 0);
  if (e != hipSuccess) return e;
  *grid = cus * (per_cu > 0 ? per_cu : 1);
  return hipSuccess;
}

hipError_t launch_queue_pass(const shape_batch& b, const KOpts& o, void* ws, const float* p_init,
                             const float* rec, const QCfg& cfg, bool start, hipStream_t stream) {
  // Sersic always (it also retires unprocessable stamps); Moffat when the
  // batch carries a model array.
  const int models = b.model ? 2 : 1;
  const bool rows = !b.side && !b.model && rows_layout_fits(b.side0);
  for (int m = 0; m < models; ++m) {
    const void* fn;
    if (m == 0)
      fn = start ? pick_kernel<SHAPE_SERSIC, true>(b.dtype, o.free_mask, cfg.team, rows)
                 : pick_kernel<SHAPE_SERSIC, false>(b.dtype, o.free_mask, cfg.team, rows);
    else
      fn = start ? pick_kernel<SHAPE_MOFFAT, true>(b.dtype, o.free_mask, cfg.team, rows)
                 : pick_kernel<SHAPE_MOFFAT, false>(b.dtype, o.free_mask, cfg.team, rows);
    if (!fn) return hipErrorInvalidValue;
    int grid = cfg.grid;
    if (grid <= 0) {
      hipError_t e = resident_grid(fn, cfg.team, &grid);
      if (e != hipSuccess) return e;
    }
    // every cursor needs a workgroup of its own to drain it
    if (grid < kCursors) grid = kCursors;
    void* args[] = {(void*)&b, (void*)&o, &ws, (void*)&p_init, (void*)&rec};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kWave * cfg.team), args, 0, stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_queue_start(const shape_batch& b, const KOpts& o, void* ws, const float* p_init,
                              const float* rec, const QCfg& cfg, hipStream_t stream) {
  const QView v = view(ws, b.n);
  const int threads = 256;
  const int blocks = (int)((b.n + threads - 1) / threads < 4096 ? (b.n + threads - 1) / threads : 4096);
  hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(threads), 0, stream, v.hdr, v.buckets);
  hipLaunchKernelGGL(hist_kernel, dim3(blocks), dim3(threads), 0, stream, b, v.buckets);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kWave), 0, stream, v.hdr, v.buckets,
                     cfg.team > 1 ? cfg.team_min_side : kBuckets);
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(threads), 0, stream, b, v.buckets,
                     v.order);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(kWave), 0, stream, v.hdr, v.cursors);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_queue_pass(b, o, ws, p_init, rec, cfg, true, stream);
}

hipError_t launch_queue_step(const shape_batch& b, const KOpts& o, void* ws, const QCfg& cfg,
                             hipStream_t stream) {
  const QView v = view(ws, b.n);
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(kWave), 0, stream, v.hdr, v.cursors);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_queue_pass(b, o, ws, nullptr, nullptr, cfg, false, stream);
}

hipError_t launch_queue_finish(const shape_batch& b, const KOpts& o, void* ws, float* p_out,
                               float* chi2, float* perr, int32_t* iters, uint32_t* status,
                               int32_t* sweeps, hipStream_t stream) {
  const int threads = 64;
  const int64_t blocks64 = (b.n + threads - 1) / threads;
  const int blocks = (int)(blocks64 < 65536 ? blocks64 : 65536);
  if (o.free_mask == kMaskAll)
    hipLaunchKernelGGL(finish_kernel<kMaskAll>, dim3(blocks), dim3(threads), 0, stream, b, o, ws,
                       p_out, chi2, perr, iters, status, sweeps);
  else
    hipLaunchKernelGGL(finish_kernel<kMaskSize>, dim3(blocks), dim3(threads), 0, stream, b, o, ws,
                       p_out, chi2, perr, iters, status, sweeps);
  return hipGetLastError();
}

}  // namespace shape
