// S0: incidence lists I(n) (paper, Section 2: in(n) U out(n)); order inside a
// list is not fixed and does not matter to any result (all later uses are
// integer sums or set tests).  Levels of up to 2^25 vertices are transposed
// through buckets of 8192 consecutive vertices with LDS counters only;
// larger ones by global atomic counters.
// S1: expansion sizes X_n = sum over I(n) of |e|, level maxima of the
// super-node state, and the work lists of the scoring kernels.
// Level-0 state (Section 2 model; Section 3 constraint quantities).
#include "hg_internal.h"

namespace hg {

namespace {

__global__ void count_pins_kernel(const Dims* __restrict__ d, const uint32_t* __restrict__ pins,
                                  int32_t* __restrict__ vcount) {
  int64_t P = d->P;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < P; i += stride) atomicAdd(&vcount[pins[i] & kIdMask], 1);
}

// One wave per hyperedge: every pin gets a slot in its vertex's list.
__global__ void scatter_incidence_kernel(const Dims* __restrict__ d,
                                         const int64_t* __restrict__ eoff,
                                         const uint32_t* __restrict__ pins,
                                         const int64_t* __restrict__ voff,
                                         int32_t* __restrict__ cursor,
                                         uint32_t* __restrict__ vinc) {
  int64_t E = d->E;
  int lane = threadIdx.x & (kWave - 1);
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t e = wave; e < E; e += nwaves) {
    int64_t s = eoff[e], t = eoff[e + 1];
    for (int64_t k = s + lane; k < t; k += kWave) {
      uint32_t p = pins[k];
      uint32_t v = p & kIdMask;
      int32_t pos = atomicAdd(&cursor[v], 1);
      vinc[voff[v] + pos] = (uint32_t)e | (p & kDst);
    }
  }
}

// ---- bucketed transpose --------------------------------------------------
constexpr int kIncScatterThreads = 512;
// Work-group g takes the pins [P g / G, P (g + 1) / G).

__device__ inline void pin_share(int64_t P, int64_t& p0, int64_t& p1) {
  p0 = P * (int64_t)blockIdx.x / gridDim.x;
  p1 = P * (int64_t)(blockIdx.x + 1) / gridDim.x;
}

// Pins of the work-group's share per bucket: bcnt[b * G + g].
__global__ __launch_bounds__(256) void inc_count_kernel(const Dims* __restrict__ d,
                                                        const uint32_t* __restrict__ pins,
                                                        int32_t* __restrict__ bcnt,
                                                        int64_t* __restrict__ n_out) {
  __shared__ int32_t h[kIncBuckets];
  const int64_t V = d->V, P = d->P;
  const int bits = incidence_bits(V);
  const int32_t nb = (int32_t)((V + (1ll << bits) - 1) >> bits);
  for (int32_t i = threadIdx.x; i < nb; i += 256) h[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = (int64_t)nb * gridDim.x;
  __syncthreads();
  int64_t p0, p1;
  pin_share(P, p0, p1);
  for (int64_t k = p0 + threadIdx.x; k < p1; k += 256)
    atomicAdd(&h[(pins[k] & kIdMask) >> bits], 1);
  __syncthreads();
  for (int32_t i = threadIdx.x; i < nb; i += 256)
    bcnt[(int64_t)i * gridDim.x + blockIdx.x] = h[i];
}

// The work-group's pins as (vertex << 32 | edge | flag) pairs at its slots of
// each bucket (boff = exclusive scan of bcnt, bucket-major).  Waves walk the
// hyperedges that meet the share, from the one holding its first pin.
__global__ __launch_bounds__(kIncScatterThreads) void inc_scatter_kernel(
    const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
    const uint32_t* __restrict__ pins, const int64_t* __restrict__ boff,
    uint64_t* __restrict__ pairs) {
  __shared__ int32_t cur[kIncBuckets];  // next slot of each bucket (P < 2^31)
  __shared__ int64_t s_e0;
  const int64_t V = d->V, E = d->E, P = d->P;
  const int bits = incidence_bits(V);
  const int32_t nb = (int32_t)((V + (1ll << bits) - 1) >> bits);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  constexpr int NW = kIncScatterThreads / kWave;
  const int64_t G = gridDim.x;
  for (int32_t i = threadIdx.x; i < nb; i += kIncScatterThreads)
    cur[i] = (int32_t)boff[(int64_t)i * G + blockIdx.x];
  int64_t p0, p1;
  pin_share(P, p0, p1);
  if (threadIdx.x == 0) {
    // the last hyperedge starting at or before p0 (eoff[0] = 0 <= p0)
    int64_t lo = 0, hi = E;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (eoff[mid] <= p0) lo = mid;
      else hi = mid - 1;
    }
    s_e0 = lo;
  }
  __syncthreads();
  if (p0 >= p1) return;  // block-uniform, after the last barrier
  for (int64_t e = s_e0 + wid; e < E; e += NW) {
    const int64_t a0 = eoff[e], a1 = eoff[e + 1];
    if (a0 >= p1) break;  // wave-uniform
    const int64_t lo = a0 > p0 ? a0 : p0, hi = a1 < p1 ? a1 : p1;
    for (int64_t k = lo + lane; k < hi; k += kWave) {
      const uint32_t p = pins[k];
      const uint32_t v = p & kIdMask;
      const int32_t at = atomicAdd(&cur[v >> bits], 1);
      pairs[at] = ((uint64_t)v << 32) | (uint64_t)((uint32_t)e | (p & kDst));
    }
  }
}

// One work-group per bucket: its vertices' list lengths (LDS counters), their
// offsets (bucket start + an LDS scan) into voff, and the entries placed.
__global__ __launch_bounds__(1024) void inc_finish_kernel(const Dims* __restrict__ d,
                                                          const int64_t* __restrict__ boff,
                                                          int32_t G,
                                                          const uint64_t* __restrict__ pairs,
                                                          int64_t* __restrict__ voff,
                                                          uint32_t* __restrict__ vinc) {
  constexpr int kIds = 1 << kIncBits;
  constexpr int kPer = kIds / 1024;
  __shared__ int32_t cnt[kIds];
  __shared__ int32_t ws[1024 / kWave];
  const int64_t V = d->V, P = d->P;
  const int bits = incidence_bits(V);
  const int32_t ids = 1 << bits;  // vertices of a bucket (<= kIds)
  const int32_t nb = (int32_t)((V + ids - 1) >> bits);
  const int32_t b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  if (b == 0 && tid == 0) voff[V] = P;
  if (b >= nb) return;  // block-uniform, before any barrier
  const int64_t start = boff[(int64_t)b * G];
  const int64_t end = b + 1 < nb ? boff[(int64_t)(b + 1) * G] : P;
  const int64_t base = (int64_t)b << bits;
  for (int i = tid; i < kIds; i += 1024) cnt[i] = 0;
  __syncthreads();
  // four loads in flight per thread before their LDS updates
  for (int64_t k0 = start + tid; k0 < end; k0 += 4 * 1024) {
    uint64_t pr[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + u * 1024;
      pr[u] = k < end ? pairs[k] : ((uint64_t)base << 32);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k0 + u * 1024 < end) atomicAdd(&cnt[(int32_t)((pr[u] >> 32) - base)], 1);
  }
  __syncthreads();
  // exclusive scan: thread t owns ids [kPer t, kPer t + kPer)
  int32_t loc[kPer], sum = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    loc[i] = sum;
    sum += cnt[kPer * tid + i];
  }
  int32_t inc = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) ws[wid] = inc;
  __syncthreads();
  int32_t before = 0;
  for (int w = 0; w < wid; ++w) before += ws[w];
  const int32_t first = before + inc - sum;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int32_t j = kPer * tid + i;
    cnt[j] = first + loc[i];
    if (j < ids && base + j < V) voff[base + j] = start + first + loc[i];
  }
  __syncthreads();
  for (int64_t k0 = start + tid; k0 < end; k0 += 4 * 1024) {
    uint64_t pr[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + u * 1024;
      pr[u] = k < end ? pairs[k] : ((uint64_t)base << 32);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (k0 + u * 1024 < end) {
        const int32_t at = atomicAdd(&cnt[(int32_t)((pr[u] >> 32) - base)], 1);
        vinc[start + at] = (uint32_t)pr[u];
      }
    }
  }
}

// ---- bucketed sums of flagged pins ------------------------------------------
// The same buckets, over the live pins of each hyperedge (pins[eoff[e] ..
// eoff[e] + len[e]) when `len` is given); only flagged pins take part.

__device__ inline int64_t edge_of_pin(const int64_t* eoff, int64_t E, int64_t p0) {
  int64_t lo = 0, hi = E;  // the last hyperedge starting at or before p0
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (eoff[mid] <= p0) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ inline int64_t acc_vertices(const int64_t* nv64, const int32_t* nv32) {
  return nv64 ? *nv64 : (int64_t)*nv32;
}

template <bool SCATTER>
__global__ __launch_bounds__(kIncScatterThreads) void flagged_bucket_kernel(
    const Dims* __restrict__ d, const int64_t* __restrict__ eoff, const int32_t* __restrict__ len,
    const uint32_t* __restrict__ pins, const int32_t* __restrict__ val,
    const int64_t* __restrict__ nv64, const int32_t* __restrict__ nv32,
    int32_t* __restrict__ bcnt, int64_t* __restrict__ n_out, const int64_t* __restrict__ boff,
    uint64_t* __restrict__ pairs) {
  __shared__ int32_t h[kIncBuckets];
  __shared__ int64_t s_e0;
  const int64_t E = d->E, P = d->P, NV = acc_vertices(nv64, nv32);
  const int bits = incidence_bits(NV);
  const int32_t nb = (int32_t)((NV + (1ll << bits) - 1) >> bits);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  constexpr int NW = kIncScatterThreads / kWave;
  const int64_t G = gridDim.x;
  // counts, or (scatter) the next slot of each bucket (P < 2^31)
  for (int32_t i = threadIdx.x; i < nb; i += kIncScatterThreads)
    h[i] = SCATTER ? (int32_t)boff[(int64_t)i * G + blockIdx.x] : 0;
  if (!SCATTER && blockIdx.x == 0 && threadIdx.x == 0) *n_out = (int64_t)nb * gridDim.x;
  int64_t p0, p1;
  pin_share(P, p0, p1);
  if (threadIdx.x == 0) s_e0 = edge_of_pin(eoff, E, p0);
  __syncthreads();
  if (p0 < p1) {  // block-uniform
    for (int64_t e = s_e0 + wid; e < E; e += NW) {
      const int64_t a0 = eoff[e];
      if (a0 >= p1) break;  // wave-uniform
      const int64_t a1 = len ? a0 + len[e] : eoff[e + 1];
      const int64_t lo = a0 > p0 ? a0 : p0, hi = a1 < p1 ? a1 : p1;
      const int32_t m = val[e];
      for (int64_t k = lo + lane; k < hi; k += kWave) {
        const uint32_t p = pins[k];
        if (!(p & kDst)) continue;
        const uint32_t v = p & kIdMask;
        const int32_t at = atomicAdd(&h[v >> bits], 1);
        if (SCATTER) pairs[at] = ((uint64_t)v << 32) | (uint32_t)m;
      }
    }
  }
  if (!SCATTER) {
    __syncthreads();
    for (int32_t i = threadIdx.x; i < nb; i += kIncScatterThreads)
      bcnt[(int64_t)i * G + blockIdx.x] = h[i];
  }
}

// One work-group per bucket: LDS sums of its pairs added to acc.
__global__ __launch_bounds__(1024) void flagged_sum_kernel(
    const int64_t* __restrict__ nv64, const int32_t* __restrict__ nv32,
    const int64_t* __restrict__ boff, int32_t G, const int64_t* __restrict__ n_pairs_at,
    const uint64_t* __restrict__ pairs, int32_t* __restrict__ acc) {
  constexpr int kIds = 1 << kIncBits;
  __shared__ int32_t sum[kIds];
  const int64_t NV = acc_vertices(nv64, nv32);
  const int bits = incidence_bits(NV);
  const int32_t ids = 1 << bits;
  const int32_t nb = (int32_t)((NV + ids - 1) >> bits);
  const int32_t b = blockIdx.x;
  if (b >= nb) return;  // block-uniform
  const int64_t start = boff[(int64_t)b * G];
  const int64_t end = b + 1 < nb ? boff[(int64_t)(b + 1) * G] : boff[*n_pairs_at];
  const int64_t base = (int64_t)b << bits;
  for (int i = threadIdx.x; i < kIds; i += 1024) sum[i] = 0;
  __syncthreads();
  for (int64_t k = start + threadIdx.x; k < end; k += 1024) {
    const uint64_t pr = pairs[k];
    atomicAdd(&sum[(int32_t)((pr >> 32) - base)], (int32_t)(uint32_t)pr);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ids; i += 1024)
    if (base + i < NV && sum[i]) acc[base + i] += sum[i];
}

__global__ void flagged_atomic_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
                                      const int32_t* __restrict__ len,
                                      const uint32_t* __restrict__ pins,
                                      const int32_t* __restrict__ val, int32_t* __restrict__ acc) {
  const int64_t E = d->E;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t e = wave; e < E; e += nw) {
    const int64_t a0 = eoff[e], a1 = len ? a0 + len[e] : eoff[e + 1];
    const int32_t m = val[e];
    for (int64_t k = a0 + lane; k < a1; k += kWave) {
      const uint32_t p = pins[k];
      if (p & kDst) atomicAdd(&acc[p & kIdMask], m);
    }
  }
}

__global__ void level0_flags_kernel(const Dims* __restrict__ d, const uint32_t* __restrict__ pins,
                                    int32_t* __restrict__ syn) {
  int64_t P = d->P;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < P; i += stride) {
    uint32_t p = pins[i];
    if (p & kDst) atomicAdd(&syn[p & kIdMask], 1);
  }
}

__global__ void level0_finish_kernel(const Dims* __restrict__ d, int32_t* __restrict__ size,
                                     const int32_t* __restrict__ syn, int32_t* __restrict__ ax,
                                     int32_t* __restrict__ mult) {
  int64_t V = d->V, E = d->E;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = i; v < V; v += stride) {
    size[v] = 1;
    ax[v] = syn[v];
  }
  for (int64_t e = i; e < E; e += stride) mult[e] = 1;
}

__global__ void reset_maxima_kernel(GraphConst* gc, int32_t n_graphs, int32_t* bcount,
                                    int64_t* visits) {
  int i = threadIdx.x;
  for (int g = i; g < n_graphs; g += blockDim.x) {
    gc[g].max_size = 0;
    gc[g].max_syn = 0;
    gc[g].max_ax = 0;
    gc[g].nverts = 0;
  }
  if (i < kNumBuckets) {
    bcount[i] = 0;
    visits[i] = 0;
  }
}

// MULTI (a union of graphs): the per-graph maxima and vertex counts are kept
// per wave and written when the graph changes; a single graph's come from
// graph_maxima_kernel instead (per-wave atomics from every wave of the
// expansion would all hit the same four words).
template <bool MULTI>
__global__ void expansion_kernel(LevelView L, const int64_t* __restrict__ voff,
                                 const uint32_t* __restrict__ vinc, int64_t* __restrict__ xn,
                                 GraphConst* __restrict__ gc, Buckets b, int64_t maxV) {
  // A wave per vertex: lanes stride over its incidence list (coarse
  // super-nodes have tens of thousands of incident hyperedges).
  const int64_t V = L.dims->V;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x / kWave) +
                        __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int gcur = -1;
  int32_t msz = 0, msy = 0, max_ = 0, cnt = 0;
  for (int64_t v = wave0; v < V; v += nwaves) {  // wave-uniform
    const int64_t s = voff[v], t = voff[v + 1];
    int64_t x = 0;
    for (int64_t j = s + lane; j < t; j += kWave) {
      const uint32_t a = vinc[j] & kIdMask;
      x += L.eoff[a + 1] - L.eoff[a] - 1;  // neighbours visited through a (n excluded)
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    if (lane == 0) xn[v] = x;
    if (!MULTI) continue;
    const int g = L.gid[v];
    if (g != gcur) {  // wave-uniform
      if (gcur >= 0 && lane == 0) {
        atomicMax(&gc[gcur].max_size, msz);
        atomicMax(&gc[gcur].max_syn, msy);
        atomicMax(&gc[gcur].max_ax, max_);
        atomicAdd(&gc[gcur].nverts, cnt);
      }
      gcur = g;
      msz = msy = max_ = cnt = 0;
    }
    ++cnt;
    const int32_t sz = L.size[v], sy = L.syn[v], ax = L.ax[v];
    msz = sz > msz ? sz : msz;
    msy = sy > msy ? sy : msy;
    max_ = ax > max_ ? ax : max_;
  }
  if (MULTI && gcur >= 0 && lane == 0) {
    atomicMax(&gc[gcur].max_size, msz);
    atomicMax(&gc[gcur].max_syn, msy);
    atomicMax(&gc[gcur].max_ax, max_);
    atomicAdd(&gc[gcur].nverts, cnt);
  }
}

// A single graph's level maxima of size, syn and ax and its vertex count: a
// grid-stride reduction with one atomic per work-group and field.
__global__ __launch_bounds__(256) void graph_maxima_kernel(LevelView L,
                                                           GraphConst* __restrict__ gc) {
  __shared__ int32_t red[3][256 / kWave];
  const int64_t V = L.dims->V;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int32_t m[3] = {0, 0, 0};
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t sz = L.size[v], sy = L.syn[v], ax = L.ax[v];
    m[0] = sz > m[0] ? sz : m[0];
    m[1] = sy > m[1] ? sy : m[1];
    m[2] = ax > m[2] ? ax : m[2];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
      const int32_t o = __shfl_xor(m[c], d, kWave);
      m[c] = o > m[c] ? o : m[c];
    }
    if (lane == 0) red[c][wid] = m[c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int32_t r = 0;
      for (int w = 0; w < 256 / kWave; ++w) r = red[c][w] > r ? red[c][w] : r;
      if (r > 0) atomicMax(c == 0 ? &gc[0].max_size : (c == 1 ? &gc[0].max_syn : &gc[0].max_ax), r);
    }
    if (blockIdx.x == 0) gc[0].nverts = (int32_t)V;
  }
}

// Thread per vertex.  Bucket by a bound on the distinct neighbours (X_n, and
// the graph's vertex count): single pass in the small table (bound <=
// load16/16 of it), single pass in the big table, or multipass; +4
// when the distinct-axon bound can bind for n (ax_n + level max > Delta), so
// the shared inbound count must be accumulated; 8 or 9 (dense windows) for
// neighbourhoods that visit at least one id in dense_ratio of the graph and
// are large or visited at least kDenseMinVisits times.  Vertices with X_n = 0 have
// no neighbour and are in no list.
__global__ void bucket_kernel(LevelView L, const int64_t* __restrict__ xn,
                              const int64_t* __restrict__ voff,
                              const GraphConst* __restrict__ gc, Buckets b, int64_t maxV,
                              int32_t load16, int32_t dense_windows, int32_t dense_ratio) {
  const int64_t V = L.dims->V;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // wave-uniform loop: every lane takes part in the list append
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x +
                      __builtin_amdgcn_readfirstlane(threadIdx.x & ~(kWave - 1));
       base < V;
       base += stride) {
    const int64_t v = base + lane;
    int bk = -1;
    if (v < V) {
      const int64_t x = xn[v];
      const GraphConst G = gc[L.gid ? L.gid[v] : 0];
      // no neighbour, or no vertex of this graph has a candidate any more
      if (x > 0 && !G.done) {
        const bool ov = (int64_t)L.ax[v] + G.max_ax > G.delta;
        // distinct neighbours: at most the visits, and at most the other
        // vertices of the graph (coarse levels revisit few super-nodes often)
        const int64_t dist = x < (int64_t)G.nverts - 1 ? x : (int64_t)G.nverts - 1;
        if (dist <= (int64_t)kSmallSlots * load16 / 16) bk = 0;
        else if (dist <= (int64_t)(ov ? kBigSlotsOv : kBigSlots) * load16 / 16) bk = 1;
        else bk = (voff[v + 1] - voff[v] <= kWinDeg) ? 2 : 3;
        if (ov) bk += 4;
        // dense neighbourhoods (visits at least a dense_ratio-th of the ids):
        // the large ones, and the small ones visited very often
        if (((bk & 3) >= 2 || x >= kDenseMinVisits) && dense_windows > 0 && dense_ratio > 0 &&
            x * dense_ratio >= (int64_t)G.nverts)
          bk = ov ? 9 : 8;
      }
    }
    const int32_t pos = wave_bucket_slot<kNumBuckets>(bk, b.count);
    if (bk >= 0) b.list[(int64_t)bk * maxV + pos] = (int32_t)v;
    // the neighbour visits of each list (a census read back by the host)
    const int64_t xv = (bk >= 0) ? xn[v] : 0;
#pragma unroll
    for (int k = 0; k < kNumBuckets; ++k) {
      if (__builtin_amdgcn_ballot_w64(bk == k) == 0) continue;  // wave-uniform
      int64_t s = bk == k ? xv : 0;
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) s += __shfl_xor(s, d, kWave);
      if (lane == 0) atomicAdd((unsigned long long*)&b.visits[k], (unsigned long long)s);
    }
  }
}

}  // namespace

void build_incidence(const LevelView& L, int64_t maxV, int64_t maxE, int64_t maxP,
                     int32_t* vcount, int64_t* voff, uint32_t* vinc, int64_t* partials,
                     hipStream_t s, const IncScratch& inc) {
  const int64_t nb = incidence_buckets(maxV);
  if (inc.pairs && inc.boff && nb >= 1 && nb <= inc.nb_cap) {
    inc_count_kernel<<<kIncBlocks, 256, 0, s>>>(L.dims, L.pins, inc.bcnt, inc.n);
    exclusive_scan_i32(inc.bcnt, inc.boff, inc.n, nb * kIncBlocks, partials, s);
    inc_scatter_kernel<<<kIncBlocks, kIncScatterThreads, 0, s>>>(L.dims, L.eoff, L.pins,
                                                                 inc.boff, inc.pairs);
    inc_finish_kernel<<<(int)nb, 1024, 0, s>>>(L.dims, inc.boff, kIncBlocks, inc.pairs, voff,
                                               vinc);
    return;
  }
  fill_i32(vcount, 0, maxV, s);
  count_pins_kernel<<<grid_for(maxP, 256 * 8, 8192), 256, 0, s>>>(L.dims, L.pins, vcount);
  exclusive_scan_i32(vcount, voff, &L.dims->V, maxV, partials, s);
  fill_i32(vcount, 0, maxV, s);
  scatter_incidence_kernel<<<grid_for(maxE, 4, 16384), 256, 0, s>>>(L.dims, L.eoff, L.pins,
                                                                     voff, vcount, vinc);
}

void scatter_add_flagged(const Dims* d, const int64_t* eoff, const int32_t* len,
                         const uint32_t* pins, const int32_t* val, const int64_t* nv64,
                         const int32_t* nv32, int64_t maxNV, int64_t maxE, int32_t* acc,
                         const IncScratch& inc, int64_t* partials, hipStream_t s) {
  const int64_t nb = incidence_buckets(maxNV);
  if (inc.pairs && inc.boff && nb >= 1 && nb <= inc.nb_cap) {
    flagged_bucket_kernel<false><<<kIncBlocks, kIncScatterThreads, 0, s>>>(
        d, eoff, len, pins, val, nv64, nv32, inc.bcnt, inc.n, nullptr, nullptr);
    exclusive_scan_i32(inc.bcnt, inc.boff, inc.n, nb * kIncBlocks, partials, s);
    flagged_bucket_kernel<true><<<kIncBlocks, kIncScatterThreads, 0, s>>>(
        d, eoff, len, pins, val, nv64, nv32, nullptr, nullptr, inc.boff, inc.pairs);
    flagged_sum_kernel<<<(int)nb, 1024, 0, s>>>(nv64, nv32, inc.boff, kIncBlocks, inc.n,
                                               inc.pairs, acc);
    return;
  }
  flagged_atomic_kernel<<<grid_for(maxE, 4, 16384), 256, 0, s>>>(d, eoff, len, pins, val, acc);
}

void level0_state(const Dims* d, const int64_t* eoff, const uint32_t* pins, int64_t maxV,
                  int64_t maxE, int32_t* size, int32_t* syn, int32_t* ax, int32_t* mult,
                  hipStream_t s) {
  (void)eoff;
  fill_i32(syn, 0, maxV, s);
  level0_flags_kernel<<<4096, 256, 0, s>>>(d, pins, syn);
  int64_t m = maxV > maxE ? maxV : maxE;
  level0_finish_kernel<<<grid_for(m, 256, 8192), 256, 0, s>>>(d, size, syn, ax, mult);
}

void expansion_and_buckets(const LevelView& L, const int64_t* voff, const uint32_t* vinc,
                           int64_t maxV, int64_t* xn, GraphConst* gc, int32_t n_graphs,
                           Buckets b, Tuning t, hipStream_t s, int32_t dense_windows) {
  reset_maxima_kernel<<<1, 256, 0, s>>>(gc, n_graphs, b.count, b.visits);
  if (L.gid) {
    expansion_kernel<true><<<grid_for(maxV, 4, 16384), 256, 0, s>>>(L, voff, vinc, xn, gc, b, maxV);
  } else {
    expansion_kernel<false><<<grid_for(maxV, 4, 16384), 256, 0, s>>>(L, voff, vinc, xn, gc, b, maxV);
    graph_maxima_kernel<<<grid_for(maxV, 256 * 8, 1024), 256, 0, s>>>(L, gc);
  }
  bucket_kernel<<<grid_for(maxV, 256, 16384), 256, 0, s>>>(L, xn, voff, gc, b, maxV,
                                                          t.load16, dense_windows,
                                                          t.dense_ratio);
}

}  // namespace hg
