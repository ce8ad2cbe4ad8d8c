// Column-wise access to a stamp for the centroid and ellipticity sweeps,
// whose weighted sums factor over a lane's pixel column: theta1 is fixed per
// column, so a lane sums f W theta2^q down its column and applies the
// theta1 factors once per column.
#pragma once

#include "common.hpp"

namespace shape {

// A stamp of any side read from memory by columns.  A side W <= 64 packs
// R = 64 / W row groups: lane l < R W owns column l % W at rows l / W + R m
// (lanes past R W idle); a larger side gives lane l the columns l and l + 64
// at every row.  All lanes run the same trip count `rows` per column;
// at(c, m, in) reads the pixel at row(m), col(c), or returns 0 with
// in = false outside the stamp.
template <int DT>
struct StampColumns {
  const void* sp;
  float scale;
  int W, R, il, j0, ncol, rows;
  bool on;
  __device__ __forceinline__ StampColumns(const shape_batch& b, const Stamp& st, int lane)
      : sp(stamp_base<DT>(b, st)), scale(st.scale), W(st.side) {
    if (W <= kWave) {
      R = kWave / W;
      il = lane / W;
      j0 = lane - il * W;
      ncol = 1;
      on = il < R;
    } else {
      R = 1;
      il = 0;
      j0 = lane;
      ncol = 2;
      on = true;
    }
    rows = (W + R - 1) / R;
  }
  __device__ __forceinline__ int col(int c) const { return j0 + kWave * c; }
  __device__ __forceinline__ int row(int m) const { return il + R * m; }
  __device__ __forceinline__ float at(int c, int m, bool& in) const {
    const int i = row(m), j = col(c);
    in = on && i < W && j < W;
    return in ? load_rel<DT>(sp, (uint32_t)(i * W + j), scale) : 0.0f;
  }
  // The pixel at row(m), col(c) clamped into the stamp (slots outside it read
  // its last row or column; in = false there, and the caller zeroes their
  // weight): every slot loads, so a block's loads are issued back to back
  // instead of one masked branch and wait per load.
  __device__ __forceinline__ float at_clamped(int c, int m, bool& in) const {
    const int i = row(m), j = col(c);
    in = on && i < W && j < W;
    const int ic = i < W ? i : W - 1, jc = j < W ? j : W - 1;
    return load_rel<DT>(sp, (uint32_t)(ic * W + jc), scale);
  }
};

// Rows summed in FP32 before a column sum is carried on in FP64.
constexpr int kColumnBlock = 8;

}  // namespace shape
