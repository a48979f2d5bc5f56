// Device helpers shared by the score-step kernels (hg_score.hip,
// hg_score_dense.hip): wave and block reductions and scans, the vertex
// context of a scored vertex and the Section 3 merge test.
#pragma once

#include "hg_internal.h"

namespace hg {
namespace {

// A value that is the same in every lane (e.g. read from LDS at a
// wave-uniform address), moved to a scalar register so that the control flow
// depending on it stays scalar.
// The lane mask of a predicate (HIP's __ballot takes an int, which costs a
// select and a compare per call to turn the predicate back into a mask).
__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ inline int32_t rfl_i32(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline uint32_t rfl_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)x);
}

struct VertexCtx {
  int32_t n;
  int64_t beg, deg;
  int32_t size_n, syn_n, ax_n;
  GraphConst G;
  bool all_valid;
};

// Section 3 limits on the union of n and m; `ov` is the number of original
// axons with a destination in both (0 when the distinct-axon bound cannot
// bind for this vertex).
__device__ inline bool merge_valid(const ScoreArgs& a, const VertexCtx& v, uint32_t m,
                                   int64_t ov) {
  if ((int64_t)v.size_n + a.L.size[m] > v.G.omega) return false;
  if ((int64_t)v.syn_n + a.L.syn[m] > v.G.phi) return false;
  return (int64_t)v.ax_n + a.L.ax[m] - ov <= v.G.delta;
}

template <int THREADS>
__device__ inline uint64_t block_max_u64(uint64_t x, uint64_t* red) {
  constexpr int NW = THREADS / kWave;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    uint64_t o = __shfl_xor(x, d, kWave);
    x = o > x ? o : x;
  }
  int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) red[wid] = x;
  __syncthreads();
  uint64_t r = red[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) r = red[k] > r ? red[k] : r;
  __syncthreads();
  return r;
}

// Inclusive prefix sum over the 64 lanes of a wave with the DPP unit: four
// shifts within rows of 16 lanes, then the row totals carried into the later
// rows with the row broadcasts (lanes shifted in from outside a row, and
// rows a step leaves out, add 0).
__device__ inline int32_t wave_incl_scan(int32_t x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 to rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 to rows 2, 3
  return x;
}

// Exclusive block-wide prefix sums of three per-thread values (in thread
// order) and their totals.  One barrier: the caller synchronises again
// before ws (3 * NW entries) is written by another scan.
template <int THREADS>
__device__ inline void block_scan3(const int32_t (&x)[3], int32_t (&px)[3], int32_t (&tx)[3],
                                   int32_t* ws) {
  constexpr int NW = THREADS / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int32_t ix[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ix[c] = wave_incl_scan(x[c]);
    if (lane == kWave - 1) ws[c * NW + wid] = ix[c];
  }
  __syncthreads();
  // the wave totals, one per lane, scanned again; a wave takes the sum of
  // the waves before it and the total with readlane
  static_assert(NW <= kWave, "one lane per wave");
  int32_t wt[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) wt[c] = lane < NW ? ws[c * NW + lane] : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int32_t inc = wave_incl_scan(wt[c]);
    const int32_t before = wid > 0 ? __builtin_amdgcn_readlane(inc, wid - 1) : 0;
    px[c] = before + ix[c] - x[c];
    tx[c] = __builtin_amdgcn_readlane(inc, NW - 1);
  }
}

template <typename K>
int persistent_grid(K kernel, int threads) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * device_cu_count();
}

}  // namespace
}  // namespace hg
