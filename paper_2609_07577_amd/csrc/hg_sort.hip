// Stable LSD radix sort of (uint64 key, uint64 value) pairs, 8 bits per pass,
// for the refinement's move and event orders.  A pass: per-tile digit counts,
// one exclusive scan over the digit-major count table, and a stable scatter
// in which every tile ranks its items digit by digit in their original order
// (lanes by ballot matching, waves and rounds by LDS counters).
#include "hg_internal.h"

namespace hg {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;  // per thread and tile
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kDigits = 256;
constexpr int kSortWaves = kSortThreads / kWave;

__global__ __launch_bounds__(kSortThreads) void digit_count_kernel(
    const uint64_t* __restrict__ keys, int64_t n, int shift, int64_t n_tiles,
    int32_t* __restrict__ counts) {
  __shared__ int32_t c[kDigits];
  const int tid = threadIdx.x;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    c[tid] = 0;
    __syncthreads();
    const int64_t base = tile * kSortTile;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const int64_t i = base + (int64_t)r * kSortThreads + tid;
      if (i < n) atomicAdd(&c[(uint32_t)(keys[i] >> shift) & 0xFFu], 1);
    }
    __syncthreads();
    counts[(int64_t)tid * n_tiles + tile] = c[tid];
    __syncthreads();
  }
}

// Items of a tile are taken in rounds of 256 (round r, thread t holds item
// r * 256 + t), so that the tile order is (round, wave, lane): a lane's rank
// among earlier items of its digit is the count from earlier rounds, earlier
// waves of its round and earlier lanes of its wave.
__global__ __launch_bounds__(kSortThreads) void digit_scatter_kernel(
    const uint64_t* __restrict__ keys, const uint64_t* __restrict__ vals, int64_t n, int shift,
    int64_t n_tiles, const int64_t* __restrict__ offsets, uint64_t* __restrict__ okeys,
    uint64_t* __restrict__ ovals) {
  __shared__ int64_t base[kDigits];
  __shared__ int32_t wcnt[kSortWaves][kDigits];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    base[tid] = offsets[(int64_t)tid * n_tiles + tile];
    for (int w = 0; w < kSortWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t t0 = tile * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
      const int64_t i = t0 + (int64_t)r * kSortThreads + tid;
      const bool live = i < n;
      uint64_t k = 0, v = 0;
      if (live) {
        k = keys[i];
        v = vals[i];
      }
      const uint32_t d = live ? ((uint32_t)(k >> shift) & 0xFFu) : 0u;
      uint64_t eq = __builtin_amdgcn_ballot_w64(live);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t m = __builtin_amdgcn_ballot_w64(((d >> b) & 1u) != 0);
        eq &= ((d >> b) & 1u) ? m : ~m;
      }
      const int32_t rank = __popcll(eq & below);
      // the first lane of each digit group publishes the group's size
      if (live && rank == 0) wcnt[wid][d] = __popcll(eq);
      __syncthreads();
      if (live) {
        int64_t pos = base[d] + rank;
        for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
        okeys[pos] = k;
        ovals[pos] = v;
      }
      __syncthreads();
      int32_t add = 0;
      for (int w = 0; w < kSortWaves; ++w) {
        add += wcnt[w][tid];
        wcnt[w][tid] = 0;
      }
      base[tid] += add;
      __syncthreads();
    }
  }
}

}  // namespace

int64_t radix_sort_scratch(int64_t n) {
  const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
  return kDigits * (n_tiles > 0 ? n_tiles : 1);
}

// Sorts n pairs by the low `bits` bits of the keys (stable).  The result is
// in (keys, vals); (tk, tv) are buffers of n entries; counts and offsets have
// radix_sort_scratch(n) entries (+1 for offsets); dn is device int64 scratch.
void radix_sort_pairs(uint64_t* keys, uint64_t* vals, uint64_t* tk, uint64_t* tv, int64_t n,
                      int bits, int32_t* counts, int64_t* offsets, int64_t* dn,
                      int64_t* partials, hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
  const int64_t m = kDigits * n_tiles;
  fill_i64(dn, m, 1, s);
  const int grid = (int)(n_tiles < 4096 ? n_tiles : 4096);
  uint64_t *ka = keys, *va = vals, *kb = tk, *vb = tv;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8, ++passes) {
    digit_count_kernel<<<grid, kSortThreads, 0, s>>>(ka, n, shift, n_tiles, counts);
    exclusive_scan_i32(counts, offsets, dn, m, partials, s);
    digit_scatter_kernel<<<grid, kSortThreads, 0, s>>>(ka, va, n, shift, n_tiles, offsets, kb,
                                                       vb);
    uint64_t* t = ka;
    ka = kb;
    kb = t;
    t = va;
    va = vb;
    vb = t;
  }
  if (passes & 1) {
    (void)hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(vals, va, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
  }
}

}  // namespace hg
