// S8: connectivity (paper, Section 3, Eq. 1):
//   Conn = sum over hyperedges e of w(e) * (lambda(e) - 1),
//   lambda(e) = number of distinct part[v] over the pins v of e.
// Four size classes: a wave with one, two or four pins per lane sorts the
// block ids by shuffles (<= 256 pins); a work-group counts distinct ids in
// an LDS hash set of 4096 slots (<= 2048 pins, many work-groups per CU to
// hide the latency of the part lookups) or of 32768 slots (<= 16384 pins,
// 1024 threads); larger hyperedges use a bitmap over the block-id range.
// Sums are int64 and combined with integer atomics, so the result does not
// depend on scheduling.
#include "hg_internal.h"

namespace hg {

namespace {

constexpr int kSmallMax = 4 * kWave;
constexpr int kMediumMax = 2048;
constexpr int kBlockMax = 16384;
constexpr int kThreads = 256;
constexpr uint32_t kEmptySlot = 0xFFFFFFFFu;

__global__ void conn_classify_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
                                     int32_t* __restrict__ list, int32_t* __restrict__ count,
                                     int64_t maxE) {
  const int64_t E = d->E;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // wave-uniform loop: every lane takes part in the list append
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x +
                      __builtin_amdgcn_readfirstlane(threadIdx.x & ~(kWave - 1));
       base < E;
       base += stride) {
    const int64_t i = base + lane;
    int b = -1;
    if (i < E) {
      const int64_t s = eoff[i + 1] - eoff[i];
      // lambda <= 1 contributes nothing
      if (s >= 2) b = s <= kSmallMax ? 0 : (s <= kMediumMax ? 1 : (s <= kBlockMax ? 2 : 3));
    }
    const int32_t pos = wave_bucket_slot<4>(b, count);
    if (b >= 0) list[(int64_t)b * maxE + pos] = (int32_t)i;
  }
}

struct ConnArgs {
  LevelView L;
  const int32_t* part;
  const int32_t* list;
  const int32_t* count;
  int32_t* work;
  int64_t* conn;
  uint32_t* bitmap;
  int64_t bitmap_words;
  int64_t part_words;
  int32_t* err;
  int64_t max_items;
};

// lambda(e) of one hyperedge of at most KPL * 64 pins by a wave: its block
// ids sorted in registers, the heads of the runs counted.
template <int KPL>
__device__ inline int conn_wave(const ConnArgs& a, int64_t s0, int len) {
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t key[KPL];
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    key[r] = 0xFFFFFFFFu;
    if (r * kWave + lane < len) key[r] = (uint32_t)a.part[a.L.pins[s0 + r * kWave + lane] & kIdMask];
  }
  wave_sort<KPL>(key);
  int lambda = 0;
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    uint32_t prev = __shfl_up(key[r], 1, kWave);
    if (r > 0) {
      const uint32_t last = __shfl(key[r > 0 ? r - 1 : 0], kWave - 1, kWave);
      if (lane == 0) prev = last;
    }
    const int pos = r * kWave + lane;
    const bool head = pos < len && (pos == 0 || prev != key[r]);
    lambda += __popcll(__ballot(head));
  }
  return lambda;
}

// Up to 256 pins: a wave per hyperedge, one, two or four keys per lane.
__global__ void conn_small_kernel(ConnArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t cnt = a.count[0] < a.max_items ? a.count[0] : a.max_items;
  int64_t acc = 0;
  for (int64_t it = wave; it < cnt; it += nw) {
    const int64_t e = a.list[it];
    const int64_t s0 = a.L.eoff[e];
    const int len = (int)(a.L.eoff[e + 1] - s0);
    int lambda;
    if (len <= kWave) lambda = conn_wave<1>(a, s0, len);  // wave-uniform
    else if (len <= 2 * kWave) lambda = conn_wave<2>(a, s0, len);
    else lambda = conn_wave<4>(a, s0, len);
    acc += (int64_t)a.L.w[e] * (lambda - 1);  // same value in every lane
  }
  if (lane == 0 && acc) atomicAdd((unsigned long long*)a.conn, (unsigned long long)acc);
}

// Hyperedges of class CLS (at most SLOTS / 2 pins): one work-group each.
template <int SLOTS, int CLS, int THREADS>
__global__ __launch_bounds__(THREADS) void conn_block_kernel(ConnArgs a) {
  __shared__ uint32_t set[SLOTS];
  __shared__ int32_t s_item;
  __shared__ int32_t s_new;
  const int tid = threadIdx.x;
  int32_t cnt = a.count[CLS];
  if (cnt > a.max_items) {
    if (tid == 0) atomicOr(a.err, kErrWorkCount);
    cnt = (int32_t)a.max_items;
  }
  for (int i = tid; i < SLOTS; i += THREADS) set[i] = kEmptySlot;
  int64_t acc = 0;
  while (true) {
    __syncthreads();
    if (tid == 0) {
      s_item = atomicAdd(&a.work[CLS], 1);
      s_new = 0;
    }
    __syncthreads();
    const int32_t item = s_item;
    if (item >= cnt) break;
    const int64_t e = a.list[item];
    const int64_t s0 = a.L.eoff[e], s1 = a.L.eoff[e + 1];
    uint32_t cap = 128;
    while (cap < 2 * (uint64_t)(s1 - s0) && cap < (uint32_t)SLOTS) cap <<= 1;
    const uint32_t mask = cap - 1;
    int mine = 0;
    for (int64_t k = s0 + tid; k < s1; k += THREADS) {
      uint32_t b = (uint32_t)a.part[a.L.pins[k] & kIdMask];
      uint32_t h = (b * 0x9E3779B1u) & mask;
      uint32_t probe = 0;
      for (; probe <= mask; ++probe) {
        uint32_t old = atomicCAS(&set[h], kEmptySlot, b);
        if (old == kEmptySlot) {
          ++mine;
          break;
        }
        if (old == b) break;
        h = (h + 1) & mask;
      }
      if (probe > mask) atomicOr(a.err, kErrSetFull);
    }
    if (mine) atomicAdd(&s_new, mine);
    __syncthreads();
    if (tid == 0) acc += (int64_t)a.L.w[e] * (s_new - 1);
    for (uint32_t i = tid; i < cap; i += THREADS) set[i] = kEmptySlot;
  }
  if (tid == 0 && acc) atomicAdd((unsigned long long*)a.conn, (unsigned long long)acc);
}

__global__ __launch_bounds__(kThreads) void conn_huge_kernel(ConnArgs a) {
  __shared__ int32_t s_item;
  __shared__ int32_t s_new;
  const int tid = threadIdx.x;
  int32_t cnt = a.count[3];
  if (cnt > a.max_items) {
    if (tid == 0) atomicOr(a.err, kErrWorkCount);
    cnt = (int32_t)a.max_items;
  }
  uint32_t* bm = a.bitmap + (int64_t)blockIdx.x * a.bitmap_words;
  for (int64_t w = tid; w < a.part_words; w += kThreads) bm[w] = 0;
  int64_t acc = 0;
  while (true) {
    __syncthreads();
    if (tid == 0) {
      s_item = atomicAdd(&a.work[3], 1);
      s_new = 0;
    }
    __syncthreads();
    const int32_t item = s_item;
    if (item >= cnt) break;
    const int64_t e = a.list[item];
    int mine = 0;
    for (int64_t k = a.L.eoff[e] + tid; k < a.L.eoff[e + 1]; k += kThreads) {
      uint32_t b = (uint32_t)a.part[a.L.pins[k] & kIdMask];
      uint32_t bit = 1u << (b & 31);
      uint32_t old = atomicOr(&bm[b >> 5], bit);
      if (!(old & bit)) ++mine;
    }
    if (mine) atomicAdd(&s_new, mine);
    __syncthreads();
    if (tid == 0) acc += (int64_t)a.L.w[e] * (s_new - 1);
    for (int64_t k = a.L.eoff[e] + tid; k < a.L.eoff[e + 1]; k += kThreads) {
      uint32_t b = (uint32_t)a.part[a.L.pins[k] & kIdMask];
      bm[b >> 5] = 0;
    }
  }
  if (tid == 0 && acc) atomicAdd((unsigned long long*)a.conn, (unsigned long long)acc);
}

}  // namespace

void connectivity(const LevelView& L, int64_t maxE, int64_t part_range, const int32_t* part,
                  int64_t* conn, const ConnScratch& cs, hipStream_t s) {
  fill_i64(conn, 0, 1, s);
  fill_i32(cs.ecount, 0, 4, s);
  fill_i32(cs.work, 0, 4, s);
  conn_classify_kernel<<<grid_for(maxE, 256, 16384), 256, 0, s>>>(L.dims, L.eoff, cs.ebucket,
                                                                  cs.ecount, maxE);
  ConnArgs a{L, part, cs.ebucket, cs.ecount, cs.work, conn, cs.bitmap, cs.bitmap_words,
             (part_range + 31) / 32, cs.err, maxE};
  conn_small_kernel<<<grid_for(maxE, 4, 16384), 256, 0, s>>>(a);
  a.list = cs.ebucket + maxE;
  conn_block_kernel<2 * kMediumMax, 1, kThreads><<<device_cu_count() * 8, kThreads, 0, s>>>(a);
  a.list = cs.ebucket + 2 * maxE;
  conn_block_kernel<2 * kBlockMax, 2, 1024><<<device_cu_count(), 1024, 0, s>>>(a);
  a.list = cs.ebucket + 3 * maxE;
  conn_huge_kernel<<<kHugeWG, kThreads, 0, s>>>(a);
}

}  // namespace hg
