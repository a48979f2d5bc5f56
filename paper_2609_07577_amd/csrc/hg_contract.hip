// S6/S7 and super-node state: contraction G -> G_P (paper, Section 3,
// "Partitioning Definition": A = {rho(e)}, eta(a) = summed weight; Section
// 4.1: the constrained state of every super-node is carried to the next
// level).
//
// S6  per fine hyperedge: relabel pins through vmap, sort by coarse id, merge
//     equal ids (destination flag = OR), drop if fewer than two remain, and
//     hash the resulting (id, flag) list.  Three size classes: one wave in
//     registers (<= 256 pins, one, two or four keys per lane), one work-group in
//     LDS (<= 16384 pins), and a bitmap over the coarse id range for
//     anything larger.
// S7  group identical lists: a global open-addressing table keyed by the
//     64-bit hash elects the smallest fine hyperedge of each hash value; every
//     member is then compared pin by pin with it, and the rare members whose
//     list differs (hash collisions) are grouped among themselves by an exact
//     quadratic pass.  Coarse hyperedges are numbered by their smallest fine
//     hyperedge; weights and multiplicities are summed.
// State: size and syn are sums; v_axons of a coarse vertex is the count of
//     original axons with a destination inside it:
//       sum over members of (ax - sum of mult over hyperedges where the
//       member has the flag)  [axons already internal to a member]
//     + sum over fine hyperedges of mult where the coarse vertex gets the
//       flag after relabelling  [axons with a destination in it, internal to
//       it now or not].
#include "hg_internal.h"

namespace hg {

namespace {

constexpr int kSmallMax = 4 * kWave;
constexpr int kMediumMax = 2048;
constexpr int kBlockMax = 16384;
constexpr int kBlockThreads = 256;
constexpr uint32_t kPad = 0xFFFFFFFFu;

__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline uint32_t key_to_pin(uint32_t k) { return (k >> 1) | ((k & 1u) << 31); }

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// ---------------------------------------------------------------------------
// Coarse vertex state from the fine vertices: sizes and synapses summed; the
// axons start from each member's internal ones (its axons less the
// multiplicity of the hyperedges where it holds the destination flag, which
// scatter_add_flagged summed into dstmult).
__global__ void vertex_state_kernel(LevelView L, const int32_t* __restrict__ vmap,
                                    const int32_t* __restrict__ dstmult, int32_t* __restrict__ osize,
                                    int32_t* __restrict__ osyn, int32_t* __restrict__ oax) {
  int64_t V = L.dims->V;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < V; i += stride) {
    int32_t c = vmap[i];
    atomicAdd(&osize[c], L.size[i]);
    atomicAdd(&osyn[c], L.syn[i]);
    int32_t internal = L.ax[i] - dstmult[i];
    if (internal) atomicAdd(&oax[c], internal);
  }
}

__global__ void classify_edges_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
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
      b = s <= kSmallMax ? 0 : (s <= kMediumMax ? 1 : (s <= kBlockMax ? 2 : 3));
    }
    const int32_t pos = wave_bucket_slot<4>(b, count);
    if (b >= 0) list[(int64_t)b * maxE + pos] = (int32_t)i;
  }
}

struct S6Args {
  LevelView L;
  const int32_t* vmap;
  uint32_t* tpin;
  int32_t* tlen;
  uint64_t* fp;
  int32_t* oax;
  const int32_t* list;
  const int32_t* count;
  int32_t* work;
  uint32_t* bitmap;
  int64_t bitmap_words;
  const int32_t* n_coarse;
  int32_t* err;
  int64_t max_items;
  uint64_t fp_mask;  // fingerprint bits kept (all of them outside tests)
};

// The coarse pins of fine hyperedge e (their flagged multiplicities are added
// to the coarse vertices' axons after S6, by scatter_add_flagged).
__device__ inline void emit_pin(const S6Args& a, int64_t e, int64_t pos, uint32_t pin,
                                int32_t m) {
  (void)m;
  a.tpin[a.L.eoff[e] + pos] = pin;
}

// S6 of one hyperedge of at most KPL * 64 pins by a wave: keys (coarse id,
// flag) sorted in registers, the last key of each run of one id kept (its
// flag is the OR of the run's), emitted at its rank.  Returns the number
// emitted; h gets the sum of their hashes (this lane's part).
template <int KPL>
__device__ inline int s6_wave(const S6Args& a, int64_t e, int64_t s0, int len, int32_t m,
                              uint64_t& h) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t below = (1ull << lane) - 1;
  uint32_t key[KPL];
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    key[r] = kPad;
    if (r * kWave + lane < len) {
      const uint32_t p = a.L.pins[s0 + r * kWave + lane];
      key[r] = ((uint32_t)a.vmap[p & kIdMask] << 1) | (p >> 31);
    }
  }
  wave_sort<KPL>(key);
  int n_out = 0;
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    uint32_t next = __shfl_down(key[r], 1, kWave);
    if (r + 1 < KPL) {
      const uint32_t first = __shfl(key[r + 1 < KPL ? r + 1 : r], 0, kWave);
      if (lane == kWave - 1) next = first;
    }
    const int pos = r * kWave + lane;
    const bool tail = pos < len && (pos == len - 1 || (next >> 1) != (key[r] >> 1));
    const uint64_t tb = __ballot(tail);
    if (tail) {
      const uint32_t pin = key_to_pin(key[r]);
      emit_pin(a, e, n_out + __popcll(tb & below), pin, m);
      h += mix64(pin);
    }
    n_out += __popcll(tb);
  }
  return n_out;
}

// Up to 256 pins: a wave per hyperedge, one, two or four keys per lane.
__global__ void s6_small_kernel(S6Args a) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t cnt = a.count[0] < a.max_items ? a.count[0] : a.max_items;
  for (int64_t it = wave; it < cnt; it += nw) {
    const int64_t e = a.list[it];
    const int64_t s0 = a.L.eoff[e];
    const int len = (int)(a.L.eoff[e + 1] - s0);
    const int32_t m = a.L.mult[e];
    uint64_t h = 0;
    int n_out;
    if (len <= kWave) n_out = s6_wave<1>(a, e, s0, len, m, h);  // wave-uniform
    else if (len <= 2 * kWave) n_out = s6_wave<2>(a, e, s0, len, m, h);
    else n_out = s6_wave<4>(a, e, s0, len, m, h);
    h = wave_sum(h);
    // every lane stores the same values (no lane-only code in this loop)
    a.tlen[e] = n_out;
    a.fp[e] = ((h + mix64(0x5151ull + (uint64_t)n_out)) & a.fp_mask) | 1ull;
  }
}

template <int THREADS = kBlockThreads>
__device__ inline int64_t block_exclusive_scan_i32(int32_t v, int32_t* total, int32_t* wsum) {
  constexpr int NW = THREADS / kWave;
  int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int32_t inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int32_t t = __shfl_up(inc, d, kWave);
    if (lane >= d) inc += t;
  }
  if (lane == kWave - 1) wsum[wid] = inc;
  __syncthreads();
  int32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    if (k < wid) base += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

template <int THREADS = kBlockThreads>
__device__ inline uint64_t block_sum_u64(uint64_t v, uint64_t* red) {
  constexpr int NW = THREADS / kWave;
  v = wave_sum(v);
  int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  uint64_t r = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) r += red[k];
  __syncthreads();
  return r;
}

// Hyperedges of class CLS (at most MAXN pins): one work-group, bitonic sort
// in LDS (the medium class keeps its keys small enough for many work-groups
// per CU, which hide the latency of the vertex-map lookups; the large class
// sorts with 1024 threads, eight compare-exchanges per thread and step at
// 16384 keys).
template <int MAXN, int CLS, int THREADS>
__global__ __launch_bounds__(THREADS) void s6_block_kernel(S6Args a) {
  __shared__ uint32_t keys[MAXN];
  __shared__ int32_t wsum[THREADS / kWave];
  __shared__ uint64_t red[THREADS / kWave];
  __shared__ int32_t s_item;
  const int tid = threadIdx.x;
  int32_t cnt = a.count[CLS];
  if (cnt > a.max_items) {
    if (tid == 0) atomicOr(a.err, kErrWorkCount);
    cnt = (int32_t)a.max_items;
  }
  while (true) {
    __syncthreads();
    if (tid == 0) s_item = atomicAdd(&a.work[CLS], 1);
    __syncthreads();
    const int32_t item = s_item;
    if (item >= cnt) break;
    const int64_t e = a.list[item];
    const int64_t s0 = a.L.eoff[e];
    const int len = (int)(a.L.eoff[e + 1] - s0);
    int N = 128;
    while (N < len && N < MAXN) N <<= 1;
    for (int i = tid; i < N; i += THREADS) {
      uint32_t key = kPad;
      if (i < len) {
        uint32_t p = a.L.pins[s0 + i];
        key = ((uint32_t)a.vmap[p & kIdMask] << 1) | (p >> 31);
      }
      keys[i] = key;
    }
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int t = tid; t < N / 2; t += THREADS) {
          int i = 2 * t - (t & (j - 1));
          int l = i + j;
          uint32_t x = keys[i], y = keys[l];
          bool asc = (i & k) == 0;
          if ((x > y) == asc) {
            keys[i] = y;
            keys[l] = x;
          }
        }
        __syncthreads();
      }
    }
    // compaction of run tails, contiguous chunk per thread
    const int per = (len + THREADS - 1) / THREADS;
    const int lo = tid * per;
    const int hi = lo + per < len ? lo + per : len;
    int32_t c = 0;
    for (int i = lo; i < hi; ++i)
      if (i == len - 1 || (keys[i + 1] >> 1) != (keys[i] >> 1)) ++c;
    int32_t total;
    int64_t pos = block_exclusive_scan_i32<THREADS>(c, &total, wsum);
    const int32_t m = a.L.mult[e];
    uint64_t h = 0;
    for (int i = lo; i < hi; ++i) {
      if (i == len - 1 || (keys[i + 1] >> 1) != (keys[i] >> 1)) {
        uint32_t pin = key_to_pin(keys[i]);
        emit_pin(a, e, pos++, pin, m);
        h += mix64(pin);
      }
    }
    h = block_sum_u64<THREADS>(h, red);
    if (tid == 0) {
      a.tlen[e] = total;
      a.fp[e] = ((h + mix64(0x5151ull + (uint64_t)total)) & a.fp_mask) | 1ull;
    }
  }
}

// > 16384 pins: presence and flag bitmaps over the coarse id range.
__global__ __launch_bounds__(kBlockThreads) void s6_huge_kernel(S6Args a) {
  __shared__ int32_t wsum[kBlockThreads / kWave];
  __shared__ uint64_t red[kBlockThreads / kWave];
  __shared__ int32_t s_item;
  const int tid = threadIdx.x;
  int32_t cnt = a.count[3];
  if (cnt > a.max_items) {
    if (tid == 0) atomicOr(a.err, kErrWorkCount);
    cnt = (int32_t)a.max_items;
  }
  const int64_t words = ((int64_t)*a.n_coarse + 31) / 32;
  uint32_t* present = a.bitmap + (int64_t)blockIdx.x * 2 * a.bitmap_words;
  uint32_t* flag = present + a.bitmap_words;
  for (int64_t w = tid; w < words; w += kBlockThreads) {
    present[w] = 0;
    flag[w] = 0;
  }
  while (true) {
    __syncthreads();
    if (tid == 0) s_item = atomicAdd(&a.work[3], 1);
    __syncthreads();
    const int32_t item = s_item;
    if (item >= cnt) break;
    const int64_t e = a.list[item];
    const int64_t s0 = a.L.eoff[e], s1 = a.L.eoff[e + 1];
    for (int64_t k = s0 + tid; k < s1; k += kBlockThreads) {
      uint32_t p = a.L.pins[k];
      uint32_t c = (uint32_t)a.vmap[p & kIdMask];
      atomicOr(&present[c >> 5], 1u << (c & 31));
      if (p & kDst) atomicOr(&flag[c >> 5], 1u << (c & 31));
    }
    __syncthreads();
    const int32_t m = a.L.mult[e];
    int64_t base = 0;
    uint64_t h = 0;
    for (int64_t w0 = 0; w0 < words; w0 += kBlockThreads) {
      int64_t w = w0 + tid;
      uint32_t bits = w < words ? present[w] : 0u;
      uint32_t fl = w < words ? flag[w] : 0u;
      int32_t total;
      int64_t pos = base + block_exclusive_scan_i32(__popc(bits), &total, wsum);
      while (bits) {
        int b = __ffs(bits) - 1;
        bits &= bits - 1;
        uint32_t id = (uint32_t)(w * 32 + b);
        uint32_t pin = id | (((fl >> b) & 1u) << 31);
        emit_pin(a, e, pos++, pin, m);
        h += mix64(pin);
      }
      if (w < words) {
        present[w] = 0;
        flag[w] = 0;
      }
      base += total;
    }
    h = block_sum_u64(h, red);
    if (tid == 0) {
      a.tlen[e] = (int32_t)base;
      a.fp[e] = ((h + mix64(0x5151ull + (uint64_t)base)) & a.fp_mask) | 1ull;
    }
  }
}

// ---------------------------------------------------------------------------
// S7
struct S7Args {
  const Dims* dims;
  const int64_t* eoff;
  const uint32_t* tpin;
  int32_t* tlen;
  const uint64_t* fp;
  uint64_t* hkey;
  int32_t* hlead;
  int64_t hmask;
  int32_t* slot;
  int32_t* group;
  int32_t* mism;
  int32_t* mcount;
  int32_t* err;
};

__global__ void s7_insert_kernel(S7Args a) {
  int64_t E = a.dims->E;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < E; i += stride) {
    if (a.tlen[i] < 2) continue;
    uint64_t f = a.fp[i];
    int64_t h = (int64_t)((f ^ (f >> 29)) & (uint64_t)a.hmask);
    int64_t probe = 0;
    for (; probe <= a.hmask; ++probe) {
      uint64_t old = atomicCAS((unsigned long long*)&a.hkey[h], 0ull, (unsigned long long)f);
      if (old == 0 || old == f) break;
      h = (h + 1) & a.hmask;
    }
    if (probe > a.hmask) {
      atomicOr(a.err, kErrHashFull);
      a.tlen[i] = 0;  // treated as dropped; the error word reports the failure
      continue;
    }
    a.slot[i] = (int32_t)h;
    atomicMin(&a.hlead[h], (int32_t)i);
  }
}

__device__ inline bool lists_equal_wave(const S7Args& a, int64_t e1, int64_t e2) {
  const int lane = threadIdx.x & (kWave - 1);
  int32_t n1 = a.tlen[e1];
  if (n1 != a.tlen[e2]) return false;
  if (n1 > a.eoff[e1 + 1] - a.eoff[e1] || n1 > a.eoff[e2 + 1] - a.eoff[e2]) {
    atomicOr(a.err, kErrListLength);  // every lane: no lane-only code in wave loops
    return false;
  }
  const uint32_t* p1 = a.tpin + a.eoff[e1];
  const uint32_t* p2 = a.tpin + a.eoff[e2];
  for (int32_t k = 0; k < n1; k += kWave) {
    bool diff = (k + lane < n1) && p1[k + lane] != p2[k + lane];
    if (__ballot(diff)) return false;
  }
  return true;
}

__global__ void s7_verify_kernel(S7Args a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t E = a.dims->E;
  // Every lane of the wave stores the same group value; hash collisions are
  // marked -2 here and listed by s7_collect_kernel.
  for (int64_t e = wave; e < E; e += nw) {
    int32_t g;
    if (a.tlen[e] < 2) {
      g = -1;
    } else {
      int32_t L = a.hlead[a.slot[e]];
      if (L == (int32_t)e) g = (int32_t)e;
      else g = lists_equal_wave(a, e, L) ? L : -2;
    }
    a.group[e] = g;
  }
  (void)lane;
}

__global__ void s7_collect_kernel(S7Args a) {
  int64_t E = a.dims->E;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < E; i += stride) {
    if (a.group[i] == -2) {
      int pos = atomicAdd(a.mcount, 1);
      a.mism[pos] = (int32_t)i;
    }
  }
}

// Hash collisions: group the mismatching hyperedges among themselves by
// exact comparison; leader = smallest id with the same list.
__global__ void s7_fixup_kernel(S7Args a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int32_t k = *a.mcount < (int32_t)a.dims->E ? *a.mcount : (int32_t)a.dims->E;
  for (int32_t i = wid; i < k; i += nw) {
    int32_t e = a.mism[i];
    int32_t best = e;
    for (int32_t j = 0; j < k; ++j) {
      int32_t e2 = a.mism[j];
      if (e2 < best && lists_equal_wave(a, e, e2)) best = e2;
    }
    a.group[e] = best;  // every lane stores the same value
  }
  (void)lane;
}

__global__ void leader_flag_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ group,
                                   int32_t* __restrict__ lflag) {
  int64_t E = d->E;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < E; i += stride) lflag[i] = group[i] == (int32_t)i ? 1 : 0;
}

__global__ void coarse_edges_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ group,
                                    const int64_t* __restrict__ lrank,
                                    const int32_t* __restrict__ tlen, const int32_t* __restrict__ w,
                                    const int32_t* __restrict__ mult, int32_t* __restrict__ leader_at,
                                    int64_t* __restrict__ llen, int32_t* __restrict__ ow,
                                    int32_t* __restrict__ omult) {
  int64_t E = d->E;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < E; i += stride) {
    int32_t g = group[i];
    if (g < 0) continue;
    int64_t r = lrank[g];
    if (g == (int32_t)i) {
      leader_at[r] = (int32_t)i;
      llen[r] = tlen[i];
    }
    atomicAdd(&ow[r], w[i]);
    atomicAdd(&omult[r], mult[i]);
  }
}

__global__ void out_edge_count_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ lrank,
                                      Dims* __restrict__ od) {
  od->E = lrank[d->E];
}

__global__ void copy_pins_kernel(const Dims* __restrict__ od, const int32_t* __restrict__ leader_at,
                                 const int64_t* __restrict__ eoff, const uint32_t* __restrict__ tpin,
                                 const int64_t* __restrict__ oeoff, uint32_t* __restrict__ opins) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t E2 = od->E;
  for (int64_t r = wave; r < E2; r += nw) {
    int64_t e = leader_at[r];
    const uint32_t* src = tpin + eoff[e];
    uint32_t* dst = opins + oeoff[r];
    int64_t n = oeoff[r + 1] - oeoff[r];
    for (int64_t k = lane; k < n; k += kWave) dst[k] = src[k];
  }
}

__global__ void finish_sizes_kernel(const int32_t* __restrict__ n_coarse,
                                    const int64_t* __restrict__ oeoff, Dims* __restrict__ od,
                                    int64_t* __restrict__ sizes) {
  od->V = *n_coarse;
  od->P = oeoff[od->E];
  sizes[0] = od->V;
  sizes[1] = od->E;
  sizes[2] = od->P;
}

}  // namespace

int contract_level(const LevelView& L, int64_t maxV, int64_t maxE, int64_t maxP,
                   const int32_t* vmap, const int32_t* n_coarse, hg_level_out* out,
                   const ContractScratch& cs, hipStream_t s) {
  (void)maxP;
  const int gridV = grid_for(maxV, 256, 16384);
  const int gridE = grid_for(maxE, 256, 16384);
  const int gridEw = grid_for(maxE, 4, 16384);  // a wave per hyperedge
  const int64_t capV = out->cap_vertices;
  const int64_t capE = out->cap_edges;

  // state
  fill_i32(cs.dstmult, 0, maxV, s);
  scatter_add_flagged(L.dims, L.eoff, nullptr, L.pins, L.mult, &L.dims->V, nullptr, maxV, maxE,
                      cs.dstmult, cs.inc, cs.partials, s);
  fill_i32(out->v_size, 0, capV, s);
  fill_i32(out->v_syn, 0, capV, s);
  fill_i32(out->v_axons, 0, capV, s);
  vertex_state_kernel<<<gridV, 256, 0, s>>>(L, vmap, cs.dstmult, out->v_size, out->v_syn,
                                            out->v_axons);

  // S6
  fill_i32(cs.ecount, 0, 8, s);
  fill_i32(cs.work, 0, 4, s);
  classify_edges_kernel<<<gridE, 256, 0, s>>>(L.dims, L.eoff, cs.ebucket, cs.ecount, maxE);
  S6Args a6{L, vmap, cs.tpin, cs.tlen, cs.fp, out->v_axons, nullptr, nullptr, cs.work,
            cs.bitmap, cs.bitmap_words, n_coarse, cs.err, maxE, cs.fp_mask};
  a6.list = cs.ebucket;
  a6.count = cs.ecount;
  s6_small_kernel<<<gridEw, 256, 0, s>>>(a6);
  a6.list = cs.ebucket + maxE;
  s6_block_kernel<kMediumMax, 1, kBlockThreads><<<device_cu_count() * 8, kBlockThreads, 0, s>>>(a6);
  a6.list = cs.ebucket + 2 * maxE;
  s6_block_kernel<kBlockMax, 2, 1024><<<device_cu_count() * 2, 1024, 0, s>>>(a6);
  a6.list = cs.ebucket + 3 * maxE;
  s6_huge_kernel<<<kHugeWG, kBlockThreads, 0, s>>>(a6);
  // the axons of the coarse vertices: + mult of every coarse hyperedge copy
  // (per fine hyperedge) where the vertex holds a destination
  scatter_add_flagged(L.dims, L.eoff, cs.tlen, cs.tpin, L.mult, nullptr, n_coarse, maxV, maxE,
                      out->v_axons, cs.inc, cs.partials, s);

  // S7
  fill_u64(cs.htab_key, 0, cs.htab_cap, s);
  fill_i32(cs.htab_lead, 0x7FFFFFFF, cs.htab_cap, s);
  S7Args a7{L.dims, L.eoff, cs.tpin, cs.tlen, cs.fp, cs.htab_key, cs.htab_lead,
            cs.htab_cap - 1, cs.slot, cs.group, cs.mism, cs.ecount + 4, cs.err};
  s7_insert_kernel<<<gridE, 256, 0, s>>>(a7);
  s7_verify_kernel<<<gridEw, 256, 0, s>>>(a7);
  s7_collect_kernel<<<gridE, 256, 0, s>>>(a7);
  s7_fixup_kernel<<<1, 256, 0, s>>>(a7);
  leader_flag_kernel<<<gridE, 256, 0, s>>>(L.dims, cs.group, cs.lflag);
  exclusive_scan_i32(cs.lflag, cs.lrank, &L.dims->E, maxE, cs.partials, s);
  fill_i32(out->edge_weight, 0, capE, s);
  fill_i32(out->edge_mult, 0, capE, s);
  coarse_edges_kernel<<<gridE, 256, 0, s>>>(L.dims, cs.group, cs.lrank, cs.tlen, L.w, L.mult,
                                            cs.leader_at, cs.llen, out->edge_weight,
                                            out->edge_mult);
  out_edge_count_kernel<<<1, 1, 0, s>>>(L.dims, cs.lrank, cs.out_dims);
  exclusive_scan_i64(cs.llen, out->edge_offsets, &cs.out_dims->E, maxE, cs.partials, s);
  copy_pins_kernel<<<gridEw, 256, 0, s>>>(cs.out_dims, cs.leader_at, L.eoff, cs.tpin,
                                          out->edge_offsets, out->pins);
  finish_sizes_kernel<<<1, 1, 0, s>>>(n_coarse, out->edge_offsets, cs.out_dims, out->sizes);
  return 0;
}

}  // namespace hg
