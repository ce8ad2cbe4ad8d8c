// A stamp of any side held in registers for the centroid and ellipticity
// iterations, whose weighted sums factor over pixel columns: theta1 is fixed
// down a column, so a lane sums f W theta2^q down its column and applies the
// theta1 factors once per column.  The stamp is read from memory once; every
// later sweep runs from registers.
#pragma once

#include "common.hpp"

namespace shape {

// Rows summed in FP32 before a column sum is carried on in FP64.
constexpr int kColumnBlock = 8;
// Most register slots a lane holds (a 64-px column, or 64 rows of a 128-px
// stamp split over two row groups).
constexpr int kMaxSlots = 64;
// Rows of the row-factor table: covers every row index a lane can form,
// padding included (at most 15 + 16 * 7 for one wave, 2 + 2 * 63 for a
// team).
constexpr int kRowTable = 256;

// Team of TEAM waves (L = 64 TEAM lanes) on one stamp of side W <= L:
// R = L / W row groups; thread t owns column t % W at rows t / W + R m
// (slot m, m < rows = ceil(W / R)).  Threads with t / W >= R hold nothing.
// Slots that are not pixels of the stamp hold a stand-in value until the
// kernel zeroes them (SlotMap::valid).
template <int TEAM>
struct SlotMap {
  int W, R, il, jl, rows;
  bool on;
  __device__ __forceinline__ SlotMap(int side, int t) : W(side) {
    R = (kWave * TEAM) / W;
    il = t / W;
    jl = t - il * W;
    on = il < R;
    rows = (W + R - 1) / R;
  }
  __device__ __forceinline__ int row(int m) const { return il + R * m; }
  __device__ __forceinline__ bool valid(int m) const { return on && row(m) < W; }
};

// Slot count a sweep is unrolled for: the smallest of 8, 16, 32, 64 that
// holds `rows`.  Inside it the slots are taken in blocks of kColumnBlock and
// a block at or past `rows` is skipped (a wave-uniform branch).
__device__ __forceinline__ int slot_class(int rows) {
  return rows <= 8 ? 8 : rows <= 16 ? 16 : rows <= 32 ? 32 : 64;
}

// Sides each form takes: one wave up to 64, a team of three waves for
// 65..96, a team of four for 97..128 (the smallest team whose lanes hold two
// row groups of the side's columns).
template <int TEAM>
__host__ __device__ constexpr bool team_takes(int side) {
  return TEAM == 1 ? side <= kWave : TEAM == 3 ? (side > kWave && side <= 96) : side > 96;
}

// The row-group count R that a slot count K implies, where it is unique
// (0 elsewhere).  One wave (L = 64): a side of 33..64 has R = 1 and 33..64
// rows (K = 64); a side of 22..32 has R = 2 and 11..16 rows (K = 16); a side
// of 17..21 has R = 3 and 6..7 rows, and every side below 17 also has at
// most 8 rows (K = 8, R from 3 to 16); no side gives 17..32 rows.  Teams of
// three (L = 192, side 65..96) and four (L = 256, side 97..128) have R = 2
// and 33..64 rows (K = 64).  With R known at compile time, the row offsets
// R m of a lane's slots are constants.
template <int TEAM, int K>
__host__ __device__ constexpr int fixed_rows_groups() {
  if constexpr (TEAM == 1) return K == 64 ? 1 : K == 16 ? 2 : 0;
  else return K == 64 ? 2 : 0;
}

// Load the K slots of this thread.  A slot below the stamp reads the pixel
// of the stamp's last row in its column (so every address is inside the
// stamp and the loads of a block issue back to back, with no select or
// branch between them); the sweeps mask such slots with SlotMap::valid.
// Blocks at or past `rows` are not loaded and hold 0.
template <int DT, int TEAM, int K>
__device__ __forceinline__ void load_slots(float (&v)[K], const void* sp, const SlotMap<TEAM>& mp,
                                           float scale) {
  const int last = mp.W - 1;
#pragma unroll
  for (int m = 0; m < K; ++m) v[m] = 0.0f;
#pragma unroll
  for (int m0 = 0; m0 < K; m0 += kColumnBlock) {
    if (m0 < mp.rows) {
#pragma unroll
      for (int q = 0; q < kColumnBlock; ++q) {
        const int i = min(mp.row(m0 + q), last);
        v[m0 + q] = load_rel<DT>(sp, (uint32_t)(i * mp.W + mp.jl), scale);
      }
    }
  }
}

// Sums of N FP64 values (N a multiple of 4) over the team: the wave sums,
// then, for a team, each wave's totals through LDS, added in wave order so
// every wave holds the same bits.  `buf` holds 2 TEAM N doubles; the two
// halves alternate between calls (`parity`), so one barrier per call keeps a
// fast wave's next write off the half a slow wave still reads.
template <int TEAM, int N>
__device__ __forceinline__ void team_sum_n(double (&u)[N], double* buf, int& parity) {
  wave_sum_n(u);
  if constexpr (TEAM > 1) {
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    double* b = buf + parity * TEAM * N;
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < N; ++j) b[w * N + j] = u[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double a = b[j];
#pragma unroll
      for (int q = 1; q < TEAM; ++q) a += b[q * N + j];
      u[j] = a;
    }
    parity ^= 1;
  }
}

// Stamps a workgroup looks at in a batch of mixed sides, their descriptors
// read in one round: with sides spread evenly in log over 16..128, a chunk
// holds about five stamps of its form (few enough that the last workgroups
// end close together).
template <int TEAM>
constexpr int chunk_of() { return TEAM == 1 ? 8 : 32; }

// Which stamps of the chunk [s0, s0 + chunk) (chunk <= 64) a form takes, as
// a bit mask (team_takes); stamps that cannot be processed go to the
// one-wave form, or to a team form that runs alone (take_bad).  Lane i looks
// at stamp s0 + i, so a chunk's descriptors are read in one round.
template <int TEAM>
__device__ __forceinline__ uint64_t chunk_mask(const shape_batch& b, int64_t s0, int chunk,
                                               int take_bad) {
  const int lane = threadIdx.x & (kWave - 1);
  bool mine = false;
  if (lane < chunk && s0 + lane < b.n) {
    const Stamp st = stamp_info(b, s0 + lane);
    mine = st.bad ? (TEAM == 1 || take_bad != 0) : team_takes<TEAM>(st.side);
  }
  return __ballot(mine);
}

// Barrier over the team (a wave on its own needs only its LDS writes made
// visible to its other lanes).
template <int TEAM>
__device__ __forceinline__ void team_sync() {
  if constexpr (TEAM > 1)
    __syncthreads();
  else
    wave_sync();
}

// Two 32 x 32 stamps per wave: lanes 0-31 hold one stamp, lanes 32-63 the
// next (group g = lane / 32), lane 32 g + j holding column j, slot m = row m.
// With 32 pixels per lane instead of 16, each step's reductions and closed
// forms are shared by two stamps.
constexpr int kPairSide = 32;

// Sums of N FP64 values (N even) within each half-wave, every lane receiving
// its half's N totals: v_permlane16_swap halves the values between the rows
// of a half (rows 0 and 2 then carry entries 0..N/2-1, rows 1 and 3 the
// rest), a scan within each row of 16 finishes them, and the totals are read
// from lanes 15, 31 (first half) and 47, 63 (second half).
template <int N>
__device__ inline void half_sum_n(double (&u)[N]) {
  static_assert(N % 2 == 0, "N must be even");
  constexpr int H = N / 2;
#pragma unroll
  for (int j = 0; j < H; ++j) swap_add16(u[j], u[j + H]);
#pragma unroll
  for (int j = 0; j < H; ++j) {
    u[j] = dpp::add<dpp::kShr1, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr2, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr4, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr8, 0xf>(u[j]);
  }
  const bool hi = (threadIdx.x & (kWave - 1)) >= 32;
  double t[N];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    t[j] = hi ? read_lane_f64(u[j], 47) : read_lane_f64(u[j], 15);
    t[j + H] = hi ? read_lane_f64(u[j], 63) : read_lane_f64(u[j], 31);
  }
#pragma unroll
  for (int j = 0; j < N; ++j) u[j] = t[j];
}

// The same for N FP32 values.
template <int N>
__device__ inline void half_sum_n(float (&u)[N]) {
  static_assert(N % 2 == 0, "N must be even");
  constexpr int H = N / 2;
#pragma unroll
  for (int j = 0; j < H; ++j) swap_add16(u[j], u[j + H]);
#pragma unroll
  for (int j = 0; j < H; ++j) {
    u[j] = dpp::add<dpp::kShr1, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr2, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr4, 0xf>(u[j]);
    u[j] = dpp::add<dpp::kShr8, 0xf>(u[j]);
  }
  const bool hi = (threadIdx.x & (kWave - 1)) >= 32;
  auto rl = [](float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
  };
  float t[N];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    t[j] = hi ? rl(u[j], 47) : rl(u[j], 15);
    t[j + H] = hi ? rl(u[j], 63) : rl(u[j], 31);
  }
#pragma unroll
  for (int j = 0; j < N; ++j) u[j] = t[j];
}

// Inclusive scan of an int64 within each half-wave (row scans, then the last
// lane of rows 0 and 2 added to rows 1 and 3).
__device__ inline long long half_scan(long long v) {
  v = dpp::add<dpp::kShr1, 0xf>(v);
  v = dpp::add<dpp::kShr2, 0xf>(v);
  v = dpp::add<dpp::kShr4, 0xf>(v);
  v = dpp::add<dpp::kShr8, 0xf>(v);
  v = dpp::add<dpp::kBcast15, 0xa>(v);
  return v;
}

// A value as held by lane `l0` for the first half-wave and by lane `l1` for
// the second (l0, l1 wave-uniform).
__device__ __forceinline__ long long half_pick(long long v, int l0, int l1) {
  const bool hi = (threadIdx.x & (kWave - 1)) >= 32;
  const long long a = readlane64(v, l0), b = readlane64(v, l1);
  return hi ? b : a;
}
__device__ __forceinline__ int half_pick(int v, int l0, int l1) {
  const bool hi = (threadIdx.x & (kWave - 1)) >= 32;
  const int a = __builtin_amdgcn_readlane(v, l0), b = __builtin_amdgcn_readlane(v, l1);
  return hi ? b : a;
}

// Whether any lane of this lane's half-wave has p set.
__device__ __forceinline__ bool half_any(bool p) {
  const uint64_t m = __ballot(p);
  const bool hi = (threadIdx.x & (kWave - 1)) >= 32;
  return ((hi ? m >> 32 : m) & 0xffffffffull) != 0;
}

}  // namespace shape
