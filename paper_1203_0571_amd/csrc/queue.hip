// Work-queue form of the profile fit (Sec. 4.1), batched: the LM iteration of
// every stamp is split into its two kinds of work, each run where it suits
// the device.
//
//   sweep kernels   one wave (or a team of waves) per stamp renders the model
//                   and its Jacobian at the stamp's trial point and reduces
//                   chi^2, J^T r and J^T J (the adjoint sums of chi^2,
//                   sweep.hpp).  Persistent: workgroups pop stamps of the
//                   current list from atomic cursors, largest side first.
//   decide kernel   one lane per stamp: profiles the amplitudes of the sweep,
//                   accepts or rejects the trial, forms the damped Schur
//                   complement, solves it (FP64 L D L^T within the lane)
//                   and either finishes the stamp or forms the next trial's
//                   constants and appends the stamp to the next list.
//
// The sweeps carry no LM arithmetic, and the LM arithmetic runs 64 stamps to
// a wave instead of one.  The per-stamp arithmetic is the fused fit's own
// (lm.hpp), so the results equal the fused kernel's bit for bit.
//
// A step = {sweep kernel per model, decide kernel per model, advance}; it
// judges one swept trial of every active stamp (trials rejected before a
// sweep are taken inside the decide kernel) and is captured once into a
// hipGraph.  The lists are compacted every step, so a late step costs what
// its active stamps cost.  shape_queue_start sorts the stamps (model, then
// side, largest first; sides >= team_min_side form the team classes), forms
// the starting points and runs the two start sweeps (amplitudes at unit
// scale, then the first full sweep) with their decisions.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "lm.hpp"

namespace shape {
namespace {

constexpr uint32_t kMaxChunk = 8;   // stamps per cursor pop at most, by default
constexpr int kDecideBlock = 256;
// The decide pass's FP64 bookkeeping holds a stamp's 45 sums and its damped
// system in one lane: waves per SIMD against register spills.
#ifndef SHAPE_DECIDE_WAVES_PER_SIMD
#define SHAPE_DECIDE_WAVES_PER_SIMD 2
#endif

// Stamp phases.
constexpr int32_t kPhLin = 0;     // the amplitude sweep at unit scale is pending
constexpr int32_t kPhFirst = 1;   // the first full sweep is pending
constexpr int32_t kPhTrial = 2;   // a trial's sweep is pending
constexpr int32_t kPhDone = 3;

struct QHeader {
  uint32_t reserved0, reserved1;
  uint32_t active;               // byte 8: stamps in the next step's list
  uint32_t step;                 // lists swapped so far (its parity names the current list)
  uint32_t begin[kClasses];      // class ranges of the order and of both lists
  uint32_t end[kClasses];
  uint32_t count[2][kClasses];   // entries of each list per class
  uint32_t drain[kClasses];      // drain pass cursor per class
  uint32_t pad[64 - 4 - 5 * kClasses];
};
static_assert(sizeof(QHeader) == 256, "header is one 256-byte block");

// The workspace: header, cursor lines, histogram, order, two lists and the
// per-stamp state, every quantity an array over the stamps ([k][n]), so that
// the decide pass (one lane per stamp) reads and writes it coalesced.
struct QView {
  QHeader* hdr;
  uint32_t* cursors;  // [class][kCursors][kCursorStride]
  uint32_t* buckets;
  int32_t* order;
  int32_t* list[2];
  double* p;          // [8][n]
  double* pt;         // [8][n]
  double* cur;        // [kSums][n]: the current point's profiled sums
  double* lambda;     // [n]
  double* smax;       // [n]
  int32_t* it;        // [n]
  int32_t* nsweep;    // [n]
  uint32_t* stt;      // [n]
  int32_t* phase;     // [n]
  double* trial;      // [kSums][n]: the last sweep's sums
  float* consts;      // [kConstRow][n]: the pending sweep's constants (TrialF)
  int64_t n;
};

__host__ __device__ inline QView view(void* ws, int64_t n) {
  char* c = static_cast<char*>(ws);
  const size_t m = (size_t)n;
  QView v;
  v.n = n;
  v.hdr = reinterpret_cast<QHeader*>(c);
  c += 256;
  v.cursors = reinterpret_cast<uint32_t*>(c);
  c += kCursorBytes;
  v.buckets = reinterpret_cast<uint32_t*>(c);
  c += align256(kBuckets * 4);
  v.order = reinterpret_cast<int32_t*>(c);
  c += align256(m * 4);
  v.list[0] = reinterpret_cast<int32_t*>(c);
  c += align256(m * 4);
  v.list[1] = reinterpret_cast<int32_t*>(c);
  c += align256(m * 4);
  v.p = reinterpret_cast<double*>(c);
  c += align256(m * 64);
  v.pt = reinterpret_cast<double*>(c);
  c += align256(m * 64);
  v.cur = reinterpret_cast<double*>(c);
  c += align256(m * 45 * 8);
  v.lambda = reinterpret_cast<double*>(c);
  c += align256(m * 8);
  v.smax = reinterpret_cast<double*>(c);
  c += align256(m * 8);
  v.it = reinterpret_cast<int32_t*>(c);
  c += align256(m * 4);
  v.nsweep = reinterpret_cast<int32_t*>(c);
  c += align256(m * 4);
  v.stt = reinterpret_cast<uint32_t*>(c);
  c += align256(m * 4);
  v.phase = reinterpret_cast<int32_t*>(c);
  c += align256(m * 4);
  v.trial = reinterpret_cast<double*>(c);
  c += align256(m * 45 * 8);
  v.consts = reinterpret_cast<float*>(c);
  return v;
}
static_assert(kSums == 45, "the workspace formula holds 45 sums per stamp");

// List 0 or 1 (a select: indexing the view's array with a run-time value
// would place the whole view in private memory).
__device__ inline int32_t* list_of(const QView& v, int which) {
  return which ? v.list[1] : v.list[0];
}
static_assert(kConstRow * sizeof(float) >= sizeof(TrialF), "the constant arrays hold a trial");
constexpr int kConsts = (int)(sizeof(TrialF) / sizeof(float));

__device__ inline int bucket_of(const shape_batch& b, int64_t s) {
  const Stamp st = stamp_info(b, s);
  return st.bad ? 0 : st.side + (st.model == SHAPE_MOFFAT ? 256 : 0);
}

// Class of a stamp: 2 model + (0: a team of waves, 1: a single wave).
__host__ __device__ constexpr int cls(int model, bool team) { return 2 * model + (team ? 0 : 1); }

// ---- ordering (largest side first) ----------------------------------------

__global__ void clear_kernel(QHeader* hdr, uint32_t* buckets, uint32_t* cursors) {
  const int t = threadIdx.x;
  if (t < 64) reinterpret_cast<uint32_t*>(hdr)[t] = 0u;
  for (int k = t; k < kBuckets; k += blockDim.x) buckets[k] = 0u;
  for (int k = t; k < kClasses * kCursors; k += blockDim.x) cursors[k * kCursorStride] = 0u;
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

// One thread turns the histogram into start positions: the Sersic classes
// (team: side >= team_min_side, then single; largest side first,
// unprocessable stamps last), then the Moffat classes.
__global__ void scan_kernel(QHeader* hdr, uint32_t* buckets, int team_min_side) {
  if (threadIdx.x != 0) return;
  uint32_t pos = 0;
  for (int m = 0; m < 2; ++m) {
    hdr->begin[cls(m, true)] = pos;
    bool single = false;
    for (int side = 255; side >= (m == 0 ? 0 : 1); --side) {
      if (!single && (side < team_min_side || side == 0)) {
        hdr->end[cls(m, true)] = pos;
        hdr->begin[cls(m, false)] = pos;
        single = true;
      }
      const int k = side + 256 * m;
      const uint32_t c = buckets[k];
      buckets[k] = pos;
      pos += c;
    }
    if (!single) {
      hdr->end[cls(m, true)] = pos;
      hdr->begin[cls(m, false)] = pos;
    }
    hdr->end[cls(m, false)] = pos;
  }
}

// Places every stamp at its side's position: each workgroup counts its own
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

// ---- per-stamp state ------------------------------------------------------

// The per-stamp state is indexed by the stamp's rank r in the queue order
// (the lists hold ranks), so the lanes of a wave touch consecutive entries.
__device__ inline LmState load_lm(const QView& v, int64_t r) {
  LmState L;
#pragma unroll
  for (int k = 0; k < 8; ++k) L.p[k] = v.p[k * v.n + r];
  L.lambda = v.lambda[r];
  L.it = v.it[r];
  L.nsweep = v.nsweep[r];
  L.stt = v.stt[r];
  L.done = v.phase[r] == kPhDone;
  return L;
}

__device__ inline void store_lm(const QView& v, int64_t r, const LmState& L) {
#pragma unroll
  for (int k = 0; k < 8; ++k) v.p[k * v.n + r] = L.p[k];
  v.lambda[r] = L.lambda;
  v.it[r] = L.it;
  v.nsweep[r] = L.nsweep;
  v.stt[r] = L.stt;
}

// (whole-struct copies through a float array keep the trial in registers)
__device__ inline void store_consts(const QView& v, int64_t r, const TrialF& t) {
  float f[kConsts];
  __builtin_memcpy(f, &t, sizeof(TrialF));
#pragma unroll
  for (int k = 0; k < kConsts; ++k) v.consts[k * v.n + r] = f[k];
}

// The pending sweep's constants of the stamp of rank r (r is the same in
// every lane, so these are scalar loads).
__device__ inline TrialF load_consts(const QView& v, int64_t r) {
  float f[kConsts];
#pragma unroll
  for (int k = 0; k < kConsts; ++k) f[k] = v.consts[k * v.n + r];
  TrialF t;
  __builtin_memcpy(&t, f, sizeof(TrialF));
  return t;
}

// Stamps (ranks) appended to a list, compacted per workgroup (kDecideBlock
// threads): every thread offers at most one stamp of class c; thread order is kept
// within the workgroup and one global atomic reserves the workgroup's range.
// Every thread of the workgroup must call it.
__device__ inline void append(const QView& v, int which, int c, bool take, int32_t s) {
  __shared__ uint32_t wsum[kDecideBlock / kWave];
  __shared__ uint32_t base;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const uint64_t m = __ballot(take);
  const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  if (tid == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kDecideBlock / kWave; ++w) {
      const uint32_t x = wsum[w];
      wsum[w] = tot;
      tot += x;
    }
    base = tot ? atomicAdd(&v.hdr->count[which][c], tot) : 0u;
  }
  __syncthreads();
  if (take) list_of(v, which)[v.hdr->begin[c] + base + wsum[wave] + below] = s;
  __syncthreads();
}

// ---- start ----------------------------------------------------------------

// Starting points (lm.hpp start_point), one lane per stamp in queue order;
// the stamps to sweep go to list 0 for the amplitude sweep at unit scale.
__global__ __launch_bounds__(kDecideBlock) void start_kernel(shape_batch b, KOpts o, void* ws,
                                                              const float* p_init,
                                                              const float* rec) {
  const QView v = view(ws, b.n);
  for (int64_t base = (int64_t)blockIdx.x * kDecideBlock; base < b.n;
       base += (int64_t)gridDim.x * kDecideBlock) {
    const int64_t i = base + threadIdx.x;
    bool take = false;
    int32_t s = 0;
    int c = 0;
    if (i < b.n) {
      s = v.order[i];
      const Stamp st = stamp_info(b, s);
      for (int k = 0; k < kClasses; ++k)
        if (i >= v.hdr->begin[k] && i < v.hdr->end[k]) c = k;
      LmState L;
      if (st.bad) {
#pragma unroll
        for (int k = 0; k < 8; ++k) L.p[k] = 0.0;
        L.lambda = o.lambda0;
        L.it = L.nsweep = 0;
        L.stt = st.bad;
        L.done = 1;
      } else {
        L = st.model == SHAPE_SERSIC ? start_point<SHAPE_SERSIC>(o, st, p_init, rec, s)
                                     : start_point<SHAPE_MOFFAT>(o, st, p_init, rec, s);
      }
      if (!L.done) {
        // the linear start: one sweep at unit amplitude / zero sky (I0 and
        // sky are the free amplitudes of every supported mask)
        L.p[6] = 1.0;
        L.p[7] = 0.0;
        store_consts(v, i, make_trial<float, false>(L.p, st.model, o.moffat_beta));
        take = true;
      }
      store_lm(v, i, L);
      v.phase[i] = L.done ? kPhDone : kPhLin;
    }
    for (int k = 0; k < kClasses; ++k) append(v, 0, k, take && c == k, (int32_t)i);
  }
}

// ---- sweeps ---------------------------------------------------------------

// The next chunk of list positions for one wave or team, taken by its lead
// thread: cursor q hands out the positions q, q + kCursors, q + 2 kCursors,
// ... of the class (every cursor sees the whole size mix); a wave starts on
// cursor (its index mod kCursors, so consecutive workgroups, which go to
// different XCDs, use different cursors) and moves on when that one is
// drained, so the grid drains every cursor.  Chunks shrink from maxc (the
// configuration's chunk) to one stamp as a cursor's part runs out.  Returns (q << 40 | cnt << 32 | j):
// positions q + kCursors (j .. j + cnt - 1), or ~0 when all are drained.
__device__ inline uint64_t pop_chunk(uint32_t* cursors, uint32_t count, int& q, int& tried,
                                     uint32_t per, uint32_t maxc) {
  while (tried < kCursors) {
    const uint32_t part = count > (uint32_t)q ? (count - q + kCursors - 1) / kCursors : 0u;
    uint32_t* cur = cursors + q * kCursorStride;
    const uint32_t seen = __hip_atomic_load(cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (seen < part) {
      uint32_t k = (part - seen) / (2u * per);
      k = k < 1u ? 1u : (k > maxc ? maxc : k);
      const uint32_t j = atomicAdd(cur, k);
      if (j < part) {
        const uint32_t cnt = part - j < k ? part - j : k;
        return ((uint64_t)q << 40) | ((uint64_t)cnt << 32) | j;
      }
    }
    q = (q + 1) % kCursors;
    ++tried;
  }
  return ~0ull;
}

// One sweep of the stamp of rank r (st: its stamp) at its pending constants
// into its trial sums; the amplitude sweep (phase kPhLin) sums the amplitude
// columns only.
template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT>
__device__ __forceinline__ void sweep_one(const shape_batch& b, const Stamp& st, const QView& v,
                                          int64_t r, double* xs, int tid, void* stage) {
  constexpr uint32_t EM = eff_mask(MASK, MODEL);
  constexpr uint32_t LIN = EM & 0xC0u;
  const TrialF t = load_consts(v, r);
  double* dst = v.trial + r;
  if (v.phase[r] == kPhLin)
    sweep_sums<DT, MODEL, LIN, TEAM, LAYOUT>(b, st, t, dst, xs, tid, v.n, stage);
  else
    sweep_sums<DT, MODEL, EM, TEAM, LAYOUT>(b, st, t, dst, xs, tid, v.n, stage);
}

// Persistent sweep pass over one model's classes of the current list: the
// team class (TEAM waves per stamp), then every wave alone on the single
// class.  Every stamp comes from memory (each step visits each stamp once,
// so none is in the caches): a team streams its stamp through an LDS buffer
// in blocks (kLayoutStaged); a wave alone takes the fused fit's layout
// (single_wave_layout; FP16 stamps of a batch of one side that divides 64
// staged whole in LDS, the lane-stride walk through an LDS buffer), so its
// sums are the fused fit's bit for bit.  Four waves per
// SIMD, as the fused fit.
template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT>
__global__ __launch_bounds__(kWave* TEAM, 4) void sweep_kernel(shape_batch b, void* ws,
                                                               uint32_t chunk) {
  __shared__ double xs[TEAM * kSums];
  __shared__ uint64_t s_pop;
  __shared__ __align__(16) unsigned char stage[TEAM][kStageBytes];
  const QView v = view(ws, b.n);
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid & (kWave - 1);
  const int which = v.hdr->step & 1;
  if constexpr (TEAM > 1) {
    const int c = cls(MODEL, true);
    const uint32_t count = v.hdr->count[which][c];
    const int32_t* lst = list_of(v, which) + v.hdr->begin[c];
    uint32_t* cursors = v.cursors + c * kCursors * kCursorStride;
    const uint32_t per = (gridDim.x + kCursors - 1) / kCursors;
    int q = blockIdx.x % kCursors, tried = 0;
    for (;;) {
      if (tid == 0) s_pop = pop_chunk(cursors, count, q, tried, per, chunk);
      __syncthreads();
      const uint64_t pk = s_pop;
      __syncthreads();
      if (pk == ~0ull) break;
      const uint32_t j = (uint32_t)pk, cnt = (uint32_t)(pk >> 32) & 0xFFu;
      const int qq = (int)(pk >> 40);
      for (uint32_t e = 0; e < cnt; ++e) {
        const int64_t r = lst[qq + kCursors * (j + e)];
        sweep_one<DT, MODEL, MASK, TEAM, kLayoutStaged>(b, stamp_info(b, v.order[r]), v, r, xs,
                                                        tid, stage[0]);
      }
    }
  }
  const int c = cls(MODEL, false);
  const uint32_t count = v.hdr->count[which][c];
  const int32_t* lst = list_of(v, which) + v.hdr->begin[c];
  uint32_t* cursors = v.cursors + c * kCursors * kCursorStride;
  const uint32_t per = (gridDim.x * TEAM + kCursors - 1) / kCursors;
  int q = (int)((blockIdx.x * TEAM + wave) % kCursors), tried = 0;
  for (;;) {
    uint64_t pk = 0;
    if (lane == 0) pk = pop_chunk(cursors, count, q, tried, per, chunk);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)pk);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(pk >> 32));
    if (lo == ~0u && hi == ~0u) break;
    const uint32_t j = lo, cnt = hi & 0xFFu;
    const int qq = (int)(hi >> 8);
    for (uint32_t e = 0; e < cnt; ++e) {
      const int64_t r = lst[qq + kCursors * (j + e)];
      const Stamp st = stamp_info(b, v.order[r]);
      if constexpr (LAYOUT == kLayoutRows) {
        if constexpr (DT == SHAPE_F16_SCALED) {
          // the whole stamp (at most 64 x 64 FP16, 8 KiB) in LDS for the row layout
          _Float16* lds_px = reinterpret_cast<_Float16*>(stage[wave]);
          const uint4* src = reinterpret_cast<const uint4*>(static_cast<const _Float16*>(b.pixels) +
                                                            st.off);
          wave_sync();   // the previous stamp's reads of the buffer are done
          for (int k = lane; k < st.npix / 8; k += kWave) reinterpret_cast<uint4*>(lds_px)[k] = src[k];
          wave_sync();
          shape_batch bl = b;
          bl.pixels = lds_px;
          Stamp sl = st;
          sl.off = 0;
          sweep_one<DT, MODEL, MASK, 1, kLayoutRows>(bl, sl, v, r, nullptr, lane, nullptr);
        } else {
          sweep_one<DT, MODEL, MASK, 1, kLayoutRows>(b, st, v, r, nullptr, lane, nullptr);
        }
      } else {
        // the fused fit's layout: column segments, or the lane-stride walk
        // (through the LDS buffer: the same sums)
        constexpr int kL = LAYOUT == kLayoutSegs ? kLayoutSegsStaged : kLayoutStaged;
        sweep_one<DT, MODEL, MASK, 1, kL>(b, st, v, r, nullptr, lane, stage[wave]);
      }
    }
  }
}

// ---- decisions --------------------------------------------------------------

// One stamp's LM bookkeeping after its sweep (stamp s of rank r), in one lane
// (the lm.hpp routines the fused fit runs): the amplitude start, the first
// sweep's sums, or the verdict on a trial; then new trials until one needs a
// sweep (returns true: its constants are stored) or the fit is done.
template <int MODEL, uint32_t MASK>
__device__ bool decide_one(const shape_batch& b, const KOpts& o, const QView& v, int64_t s,
                           int64_t r) {
  constexpr uint32_t EM = eff_mask(MASK, MODEL);
  constexpr uint32_t LIN = EM & 0xC0u;
  constexpr uint32_t NL = EM & 0x3Fu;
  constexpr int NN = popcount(NL);
  const Stamp st = stamp_info(b, s);
  LmState L = load_lm(v, r);
  const int32_t ph = v.phase[r];
  const double* T = v.trial + r;   // entry k at T[k * n]
  if (ph == kPhLin) {
    // the amplitudes' optimum at the starting shape, then the first full sweep
    if (!__builtin_isfinite(T[0])) {
      L.stt = SHAPE_ST_NONFINITE_INPUT;
      L.done = 1;
    } else {
      double S[kSums];
#pragma unroll
      for (int k = 0; k < kSums; ++k) S[k] = T[k * v.n];
      const AmpStep a = amp_solve<LIN>(S);
      if (!a.ok) L.stt |= SHAPE_ST_SINGULAR;
      L.p[6] += a.d6;
      L.p[7] += a.d7;
      if (!(L.p[6] > 0.0)) L.stt |= SHAPE_ST_NONPOSITIVE_FLUX;
      L.nsweep = 1;
      store_consts(v, r, make_trial<float, false>(L.p, MODEL, o.moffat_beta));
    }
    store_lm(v, r, L);
    v.phase[r] = L.done ? kPhDone : kPhFirst;
    return !L.done;
  }
  double C[kSums];
  bool changed = true;
  if (ph == kPhFirst) {
#pragma unroll
    for (int k = 0; k < kSums; ++k) C[k] = T[k * v.n];
    if (!__builtin_isfinite(C[0])) {
      L.stt = SHAPE_ST_NONFINITE_INPUT;
      L.done = 1;
    }
  } else {
    // the verdict on the swept trial
    double Tt[kSums];
#pragma unroll
    for (int k = 0; k < kSums; ++k) Tt[k] = T[k * v.n];
    double pt[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) pt[k] = v.pt[k * v.n + r];
    AmpStep a{true, 0.0, 0.0};
    if (LIN != 0u) {
      a = amp_solve<LIN>(Tt);
      if (a.ok) amp_apply<EM, LIN>(Tt, a, pt[6]);
    }
    const double c2c = v.cur[r];
    changed = lm_judge<LIN>(L, pt, a, v.smax[r], Tt[0], c2c, o);
    if (changed) {
#pragma unroll
      for (int k = 0; k < kSums; ++k) C[k] = Tt[k];
    } else {
#pragma unroll
      for (int k = 0; k < kSums; ++k) C[k] = v.cur[k * v.n + r];
    }
  }
  // the current point's sums go to memory when they changed; what the new
  // trials need of them is the undamped Schur complement (lower triangle)
  // and the step's right-hand side, so the sums need not stay in registers
  if (changed) {
#pragma unroll
    for (int k = 0; k < kSums; ++k) v.cur[k * v.n + r] = C[k];
  }
  constexpr int NT = NN * (NN + 1) / 2;
  double M[NT];
#pragma unroll
  for (int a = 0, e = 0; a < NN; ++a)
#pragma unroll
    for (int c = 0; c <= a; ++c, ++e) M[e] = schur_entry<LIN>(C, nth_bit(NL, a), nth_bit(NL, c));
  const StepRhs<NN> R = step_rhs<NL, NN>(C);
  // new trials until one needs a sweep
  bool sweep = false;
  while (!L.done) {
    if (L.it >= o.max_iter_lm) {
      L.done = 1;
      break;
    }
    // the damped system and the step
    double A[NT], x[NN];
#pragma unroll
    for (int a = 0, e = 0; a < NN; ++a) {
#pragma unroll
      for (int c = 0; c <= a; ++c, ++e) {
        double d = M[e];
        if (a == c) d *= 1.0 + L.lambda;
        A[e] = d;
      }
      x[a] = R.g[a];
    }
    const bool solved = ldl_solve<NN>(A, x);
    double pt[8];
    const double smax = lm_propose<MODEL, NL, LIN, NN>(L, R, x, solved, o, st, pt);
    if (smax >= 0.0) {
#pragma unroll
      for (int k = 0; k < 8; ++k) v.pt[k * v.n + r] = pt[k];
      v.smax[r] = smax;
      store_consts(v, r, make_trial<float, false>(pt, MODEL, o.moffat_beta));
      sweep = true;
      break;
    }
  }
  store_lm(v, r, L);
  v.phase[r] = sweep ? kPhTrial : kPhDone;
  return sweep;
}

// The decide pass over one model's classes of the current list; stamps that
// need a sweep go to the other list (same class).
template <int MODEL, uint32_t MASK>
__global__ __launch_bounds__(kDecideBlock, SHAPE_DECIDE_WAVES_PER_SIMD) void decide_kernel(shape_batch b, KOpts o, void* ws) {
  const QView v = view(ws, b.n);
  const int which = v.hdr->step & 1;
  for (int k = 0; k < 2; ++k) {
    const int c = cls(MODEL, k == 0);
    const uint32_t count = v.hdr->count[which][c];
    const int32_t* lst = list_of(v, which) + v.hdr->begin[c];
    for (uint32_t base = blockIdx.x * kDecideBlock; base < count; base += gridDim.x * kDecideBlock) {
      const uint32_t i = base + threadIdx.x;
      bool take = false;
      int32_t r = 0;
      if (i < count) {
        r = lst[i];
        take = decide_one<MODEL, MASK>(b, o, v, v.order[r], r);
      }
      append(v, which ^ 1, c, take, r);
    }
  }
}

// End of a step: swap the lists, count the active stamps, clear the list to
// be filled next and the cursors.
__global__ void advance_kernel(QHeader* hdr, uint32_t* cursors) {
  const int t = threadIdx.x;
  __shared__ uint32_t next;
  if (t == 0) {
    next = (hdr->step + 1) & 1;
    uint32_t active = 0;
    for (int c = 0; c < kClasses; ++c) active += hdr->count[next][c];
    hdr->active = active;
    hdr->step = hdr->step + 1;
  }
  __syncthreads();
  if (t < kClasses) hdr->count[next ^ 1][t] = 0u;
  if (t < kClasses) hdr->drain[t] = 0u;
  for (int k = t; k < kClasses * kCursors; k += blockDim.x) cursors[k * kCursorStride] = 0u;
}

// ---- drain ----------------------------------------------------------------

// The stamps of the current list finished in one launch per model: each
// stamp's pending trial (its sweep and verdict), then LM trials until it is
// done -- lm.hpp's loop, the fused fit's, with the state moved between the
// workspace and LDS.  Team-class stamps are taken by the whole workgroup
// (TEAM waves), the rest by single waves, as in the steps, so the results
// equal those of further steps bit for bit.  For the end of a fit, where a
// step would cost a launch, a decide pass and a straggler's sweep for a few
// stamps.
template <int TEAM>
__device__ inline void drain_load(const QView& v, int64_t r, LmShared& W, int tid) {
  team_sync<TEAM>();
  if (tid < kSums) W.sums[0][tid] = v.cur[tid * v.n + r];
  if (tid < 8) W.pt[tid] = v.pt[tid * v.n + r];
  if (tid == 0) {
    W.L = load_lm(v, r);
    W.smax = v.smax[r];
    W.cur = 0;
  }
  team_sync<TEAM>();
}

template <int TEAM>
__device__ inline void drain_store(const QView& v, int64_t r, const LmShared& W, int tid) {
  if (tid < kSums) v.cur[tid * v.n + r] = W.sums[W.cur][tid];
  if (tid == 0) {
    store_lm(v, r, W.L);
    v.phase[r] = kPhDone;
  }
  team_sync<TEAM>();
}

template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT>
__global__ __launch_bounds__(kWave* TEAM, 4) void drain_kernel(shape_batch b, KOpts o, void* ws) {
  __shared__ LmShared W[TEAM];
  __shared__ double xs[TEAM * kSums];
  __shared__ uint32_t s_e;
  const QView v = view(ws, b.n);
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid & (kWave - 1);
  const int which = v.hdr->step & 1;
  const int32_t* lst = list_of(v, which);
  if constexpr (TEAM > 1) {
    const int c = cls(MODEL, true);
    const uint32_t cnt = v.hdr->count[which][c];
    for (;;) {
      if (tid == 0) s_e = atomicAdd(&v.hdr->drain[c], 1u);
      __syncthreads();
      const uint32_t e = s_e;
      __syncthreads();
      if (e >= cnt) break;
      const int64_t r = lst[v.hdr->begin[c] + e];
      const Stamp st = stamp_info(b, v.order[r]);
      drain_load<TEAM>(v, r, W[0], tid);
      lm_sweep_judge<DT, MODEL, MASK, TEAM, kLayoutAny>(b, o, st, W[0], xs, tid);
      while (!W[0].L.done && W[0].L.it < o.max_iter_lm)
        lm_iterate<DT, MODEL, MASK, TEAM, kLayoutAny>(b, o, st, W[0], xs, tid);
      drain_store<TEAM>(v, r, W[0], tid);
    }
  }
  const int c = cls(MODEL, false);
  const uint32_t cnt = v.hdr->count[which][c];
  for (;;) {
    uint32_t e = 0;
    if (lane == 0) e = atomicAdd(&v.hdr->drain[c], 1u);
    e = __builtin_amdgcn_readfirstlane(e);
    if (e >= cnt) break;
    const int64_t r = lst[v.hdr->begin[c] + e];
    const Stamp st = stamp_info(b, v.order[r]);
    drain_load<1>(v, r, W[wave], lane);
    if constexpr (DT == SHAPE_F16_SCALED && LAYOUT == kLayoutRows && TEAM == 1) {
      // the stamp in LDS for all its remaining sweeps, as in the fused fit
      __shared__ __align__(16) _Float16 lds_px[kWave * kWave];
      const uint4* src = reinterpret_cast<const uint4*>(static_cast<const _Float16*>(b.pixels) +
                                                        st.off);
      for (int k = lane; k < st.npix / 8; k += kWave) reinterpret_cast<uint4*>(lds_px)[k] = src[k];
      wave_sync();
      shape_batch bl = b;
      bl.pixels = lds_px;
      Stamp sl = st;
      sl.off = 0;
      lm_sweep_judge<DT, MODEL, MASK, 1, LAYOUT>(bl, o, sl, W[wave], nullptr, lane);
      while (!W[wave].L.done && W[wave].L.it < o.max_iter_lm)
        lm_iterate<DT, MODEL, MASK, 1, LAYOUT>(bl, o, sl, W[wave], nullptr, lane);
    } else {
      lm_sweep_judge<DT, MODEL, MASK, 1, LAYOUT>(b, o, st, W[wave], nullptr, lane);
      while (!W[wave].L.done && W[wave].L.it < o.max_iter_lm)
        lm_iterate<DT, MODEL, MASK, 1, LAYOUT>(b, o, st, W[wave], nullptr, lane);
    }
    drain_store<1>(v, r, W[wave], lane);
  }
}

// After the drain: the current list is empty.
__global__ void drained_kernel(QHeader* hdr) {
  const int t = threadIdx.x;
  if (t < kClasses) hdr->count[hdr->step & 1][t] = 0u;
  if (t == 0) hdr->active = 0u;
}

// Outputs from the state, one lane per stamp (lm.hpp lm_finish).
template <uint32_t MASK>
__global__ void finish_kernel(shape_batch b, KOpts o, void* ws, float* p_out, float* chi2,
                              float* perr, int32_t* iters, uint32_t* status, int32_t* sweeps) {
  const QView v = view(ws, b.n);
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < b.n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = v.order[r];
    const Stamp st = stamp_info(b, s);
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
    const LmState L = load_lm(v, r);
    double C[kSums];
    for (int k = 0; k < kSums; ++k) C[k] = v.cur[k * v.n + r];
    if (st.model == SHAPE_SERSIC)
      lm_finish<SHAPE_SERSIC, MASK>(o, st, L, C, s, p_out, chi2, perr, iters, status, sweeps, 0);
    else
      lm_finish<SHAPE_MOFFAT, MASK>(o, st, L, C, s, p_out, chi2, perr, iters, status, sweeps, 0);
  }
}

// ---- host side ------------------------------------------------------------

template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT>
const void* sweep_ptr() {
  return reinterpret_cast<const void*>(&sweep_kernel<DT, MODEL, MASK, TEAM, LAYOUT>);
}

template <int MODEL>
const void* pick_sweep(int dtype, uint32_t mask, int team, int layout) {
  if constexpr (MODEL == SHAPE_SERSIC) {
    if (layout == kLayoutRows && team == 1) {
      if (dtype == SHAPE_F32 && mask == kMaskAll)
        return sweep_ptr<SHAPE_F32, MODEL, kMaskAll, 1, kLayoutRows>();
      if (dtype == SHAPE_F32 && mask == kMaskSize)
        return sweep_ptr<SHAPE_F32, MODEL, kMaskSize, 1, kLayoutRows>();
      if (dtype == SHAPE_F16_SCALED && mask == kMaskAll)
        return sweep_ptr<SHAPE_F16_SCALED, MODEL, kMaskAll, 1, kLayoutRows>();
      if (dtype == SHAPE_F16_SCALED && mask == kMaskSize)
        return sweep_ptr<SHAPE_F16_SCALED, MODEL, kMaskSize, 1, kLayoutRows>();
    }
  }
#define SHAPE_Q(DT, M, T)                                                   \
  if (dtype == DT && mask == M && team == T)                                \
    return layout == kLayoutSegs ? sweep_ptr<DT, MODEL, M, T, kLayoutSegs>() \
                                 : sweep_ptr<DT, MODEL, M, T, kLayoutAny>();
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

int decide_grid(int64_t n) {
  const int64_t g = (n + kDecideBlock - 1) / kDecideBlock;
  return (int)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

// One step: the sweeps of the current list, the decisions, the swap.
hipError_t launch_step(const shape_batch& b, const KOpts& o, void* ws, const QCfg& cfg,
                       hipStream_t stream) {
  const QView v = view(ws, b.n);
  const int models = b.model ? 2 : 1;
  for (int m = 0; m < models; ++m) {
    const void* fn =
        m == 0 ? pick_sweep<SHAPE_SERSIC>(b.dtype, o.free_mask, cfg.team,
                                          single_wave_layout(b, SHAPE_SERSIC))
               : pick_sweep<SHAPE_MOFFAT>(b.dtype, o.free_mask, cfg.team,
                                          single_wave_layout(b, SHAPE_MOFFAT));
    if (!fn) return hipErrorInvalidValue;
    int grid = cfg.grid;
    if (grid <= 0) {
      hipError_t e = resident_grid(fn, cfg.team, &grid);
      if (e != hipSuccess) return e;
    }
    uint32_t chunk = cfg.chunk > 0 ? (uint32_t)cfg.chunk : kMaxChunk;
    void* args[] = {(void*)&b, &ws, &chunk};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kWave * cfg.team), args, 0, stream);
    if (e != hipSuccess) return e;
  }
  const dim3 dg(decide_grid(b.n)), dt(kDecideBlock);
  if (o.free_mask == kMaskAll) {
    hipLaunchKernelGGL((decide_kernel<SHAPE_SERSIC, kMaskAll>), dg, dt, 0, stream, b, o, ws);
    if (b.model)
      hipLaunchKernelGGL((decide_kernel<SHAPE_MOFFAT, kMaskAll>), dg, dt, 0, stream, b, o, ws);
  } else {
    hipLaunchKernelGGL((decide_kernel<SHAPE_SERSIC, kMaskSize>), dg, dt, 0, stream, b, o, ws);
    if (b.model)
      hipLaunchKernelGGL((decide_kernel<SHAPE_MOFFAT, kMaskSize>), dg, dt, 0, stream, b, o, ws);
  }
  hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(kWave), 0, stream, v.hdr, v.cursors);
  return hipGetLastError();
}

template <int DT, int MODEL, uint32_t MASK, int TEAM, int LAYOUT>
const void* drain_ptr() {
  return reinterpret_cast<const void*>(&drain_kernel<DT, MODEL, MASK, TEAM, LAYOUT>);
}

template <int MODEL>
const void* pick_drain(int dtype, uint32_t mask, int team, int layout) {
  if constexpr (MODEL == SHAPE_SERSIC) {
    if (layout == kLayoutRows && team == 1) {
      if (dtype == SHAPE_F32 && mask == kMaskAll)
        return drain_ptr<SHAPE_F32, MODEL, kMaskAll, 1, kLayoutRows>();
      if (dtype == SHAPE_F32 && mask == kMaskSize)
        return drain_ptr<SHAPE_F32, MODEL, kMaskSize, 1, kLayoutRows>();
      if (dtype == SHAPE_F16_SCALED && mask == kMaskAll)
        return drain_ptr<SHAPE_F16_SCALED, MODEL, kMaskAll, 1, kLayoutRows>();
      if (dtype == SHAPE_F16_SCALED && mask == kMaskSize)
        return drain_ptr<SHAPE_F16_SCALED, MODEL, kMaskSize, 1, kLayoutRows>();
    }
  }
#define SHAPE_D(DT, M, T)                                                   \
  if (dtype == DT && mask == M && team == T)                                \
    return layout == kLayoutSegs ? drain_ptr<DT, MODEL, M, T, kLayoutSegs>() \
                                 : drain_ptr<DT, MODEL, M, T, kLayoutAny>();
  SHAPE_D(SHAPE_F32, kMaskAll, 1)
  SHAPE_D(SHAPE_F32, kMaskAll, 2)
  SHAPE_D(SHAPE_F32, kMaskAll, 4)
  SHAPE_D(SHAPE_F32, kMaskSize, 1)
  SHAPE_D(SHAPE_F16_SCALED, kMaskAll, 1)
  SHAPE_D(SHAPE_F16_SCALED, kMaskAll, 2)
  SHAPE_D(SHAPE_F16_SCALED, kMaskAll, 4)
  SHAPE_D(SHAPE_F16_SCALED, kMaskSize, 1)
#undef SHAPE_D
  return nullptr;
}

}  // namespace

hipError_t launch_queue_drain(const shape_batch& b, const KOpts& o, void* ws, const QCfg& cfg,
                              hipStream_t stream) {
  const QView v = view(ws, b.n);
  const int models = b.model ? 2 : 1;
  for (int m = 0; m < models; ++m) {
    const void* fn =
        m == 0 ? pick_drain<SHAPE_SERSIC>(b.dtype, o.free_mask, cfg.team,
                                          single_wave_layout(b, SHAPE_SERSIC))
               : pick_drain<SHAPE_MOFFAT>(b.dtype, o.free_mask, cfg.team,
                                          single_wave_layout(b, SHAPE_MOFFAT));
    if (!fn) return hipErrorInvalidValue;
    int grid = 0;
    hipError_t e = resident_grid(fn, cfg.team, &grid);
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&b, (void*)&o, &ws};
    e = hipLaunchKernel(fn, dim3(grid), dim3(kWave * cfg.team), args, 0, stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(drained_kernel, dim3(1), dim3(kWave), 0, stream, v.hdr);
  return hipGetLastError();
}

hipError_t launch_queue_start(const shape_batch& b, const KOpts& o, void* ws, const float* p_init,
                              const float* rec, const QCfg& cfg, hipStream_t stream) {
  const QView v = view(ws, b.n);
  const int threads = 256;
  const int blocks = (int)((b.n + threads - 1) / threads < 4096 ? (b.n + threads - 1) / threads : 4096);
  hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(threads), 0, stream, v.hdr, v.buckets, v.cursors);
  hipLaunchKernelGGL(hist_kernel, dim3(blocks), dim3(threads), 0, stream, b, v.buckets);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kWave), 0, stream, v.hdr, v.buckets,
                     cfg.team > 1 ? cfg.team_min_side : kBuckets);
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(threads), 0, stream, b, v.buckets,
                     v.order);
  hipLaunchKernelGGL(start_kernel, dim3(decide_grid(b.n)), dim3(kDecideBlock), 0, stream, b, o,
                     ws, p_init, rec);
  hipError_t e = hipGetLastError();
  // the amplitude sweep, then the first full sweep and the first trials
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = launch_step(b, o, ws, cfg, stream);
  return e;
}

hipError_t launch_queue_step(const shape_batch& b, const KOpts& o, void* ws, const QCfg& cfg,
                             hipStream_t stream) {
  return launch_step(b, o, ws, cfg, stream);
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
