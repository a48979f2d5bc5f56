// Refinement of a partition on one level of the hierarchy (paper, Section
// 4.1, "Uncoarsening and Refinement").  One round:
//
//   pins(p, e)  every pin keyed by (hyperedge, part, destination flag) and
//               sorted; runs give, per hyperedge, its parts with their pin
//               counts and destination-flagged pin counts;
//   state       per part: neurons, inbound synapses, distinct inbound axons
//               (axons internal to its vertices plus the multiplicity of the
//               hyperedges in which it holds a flagged pin);
//   proposals   per vertex n in part A, a work-group accumulates over the
//               parts p sharing a hyperedge with n the weight of those
//               hyperedges (conn(n, p)) and the multiplicity of the flagged
//               ones where p holds a flagged pin too (the axons n and p
//               share), in LDS arrays over ranges of part ids;
//               save(n) = weight of hyperedges where n is A's only pin,
//               loss(n, p) = incident weight - conn(n, p), gain = save - loss;
//               the best move with p within the limits after adding n;
//   order       moves sorted by gain (descending), vertex (ascending);
//   gains       each move's gain recomputed as if the moves before it were
//               applied: per (hyperedge, part) the moves' +1 / -1 events in
//               move order, prefix-summed onto the initial pin counts, give
//               the count each move sees; the same for flagged pins gives
//               the moves at which a hyperedge becomes or stops being
//               inbound to a part;
//   validity    per part, its size, synapse and axon events in move order,
//               prefix-summed onto the initial totals; a total crossing its
//               limit upwards (downwards) adds (removes) one violation at
//               that move, for limits the part met before the round; a
//               prefix is valid when the violations summed up to it are 0;
//   selection   the valid prefix with the largest positive cumulative gain
//               (the shortest on ties) is applied.
// Rounds repeat until one applies no move or max_rounds is reached.
#include "hg_host.h"

namespace hg {

void radix_sort_pairs(uint64_t* keys, uint64_t* vals, uint64_t* tk, uint64_t* tv, int64_t n,
                      int bits, int32_t* counts, int64_t* offsets, int64_t* dn,
                      int64_t* partials, hipStream_t s);
int64_t radix_sort_scratch(int64_t n);

namespace {

constexpr int kRange = 8192;     // part ids per pass of the proposal kernel
constexpr int kPropThreads = 256;

__device__ inline int64_t lower_bound_u64(const uint64_t* __restrict__ a, int64_t n, uint64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One key per pin: ((e * k + part) << 1) | flag.  A wave per hyperedge.
__global__ void pin_keys_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
                                const uint32_t* __restrict__ pins,
                                const int32_t* __restrict__ part, int64_t k,
                                uint64_t* __restrict__ keys, uint64_t* __restrict__ vals) {
  const int64_t E = d->E;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t e = wave; e < E; e += nw)
    for (int64_t t = eoff[e] + lane; t < eoff[e + 1]; t += kWave) {
      const uint32_t p = pins[t];
      keys[t] = (((uint64_t)e * (uint64_t)k + (uint64_t)part[p & kIdMask]) << 1) |
                (uint64_t)(p >> 31);
      vals[t] = 0;
    }
}

__global__ void run_head_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                int32_t* __restrict__ head) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) head[t] = (t == 0 || (keys[t] >> 1) != (keys[t - 1] >> 1)) ? 1 : 0;
}

// Runs of equal (e, part): the pair list with pin and flagged-pin counts,
// and the number of pairs per hyperedge.
__global__ void run_fill_kernel(const uint64_t* __restrict__ keys, int64_t n, int64_t k,
                                const int32_t* __restrict__ head, const int64_t* __restrict__ pos,
                                uint64_t* __restrict__ pair_key, int32_t* __restrict__ pair_cnt,
                                int32_t* __restrict__ pair_dcnt, int32_t* __restrict__ pcount) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) {
    const int64_t j = pos[t] + head[t] - 1;
    const uint64_t key = keys[t];
    if (head[t]) {
      pair_key[j] = key >> 1;
      atomicAdd(&pcount[(key >> 1) / (uint64_t)k], 1);
    }
    atomicAdd(&pair_cnt[j], 1);
    if (key & 1) atomicAdd(&pair_dcnt[j], 1);
  }
}

// internal(v) = axons of v that no flagged pin of v stands for any more.
// A wave per vertex.
__global__ void internal_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ voff,
                                const uint32_t* __restrict__ vinc, const int32_t* __restrict__ mult,
                                const int32_t* __restrict__ ax, int64_t* __restrict__ internal) {
  const int64_t V = d->V;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t v = wave; v < V; v += nw) {
    int64_t f = 0;
    for (int64_t j = voff[v] + lane; j < voff[v + 1]; j += kWave) {
      const uint32_t x = vinc[j];
      if (x & kDst) f += mult[x & kIdMask];
    }
#pragma unroll
    for (int s = kWave / 2; s > 0; s >>= 1) f += __shfl_xor(f, s, kWave);
    if (lane == 0) internal[v] = (int64_t)ax[v] - f;
  }
}

__global__ void part_state_vertex_kernel(const Dims* __restrict__ d,
                                         const int32_t* __restrict__ part,
                                         const int32_t* __restrict__ size,
                                         const int32_t* __restrict__ syn,
                                         const int64_t* __restrict__ internal,
                                         int64_t* __restrict__ psize, int64_t* __restrict__ psyn,
                                         int64_t* __restrict__ pax) {
  const int64_t V = d->V;
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; v < V; v += stride) {
    const int32_t p = part[v];
    atomicAdd((unsigned long long*)&psize[p], (unsigned long long)(int64_t)size[v]);
    atomicAdd((unsigned long long*)&psyn[p], (unsigned long long)(int64_t)syn[v]);
    atomicAdd((unsigned long long*)&pax[p], (unsigned long long)internal[v]);
  }
}

__global__ void part_state_pair_kernel(const uint64_t* __restrict__ pair_key,
                                       const int32_t* __restrict__ pair_dcnt,
                                       const int64_t* __restrict__ np, int64_t k,
                                       const int32_t* __restrict__ mult,
                                       int64_t* __restrict__ pax) {
  const int64_t n = *np;
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; j < n; j += stride)
    if (pair_dcnt[j] > 0) {
      const uint64_t key = pair_key[j];
      atomicAdd((unsigned long long*)&pax[key % (uint64_t)k],
                (unsigned long long)(int64_t)mult[key / (uint64_t)k]);
    }
}

struct ProposeArgs {
  const Dims* dims;
  const int64_t* voff;
  const uint32_t* vinc;
  const int32_t* w;
  const int32_t* mult;
  const int32_t* size;
  const int32_t* syn;
  const int32_t* ax;
  const int32_t* part;
  const uint64_t* pair_key;
  const int32_t* pair_cnt;
  const int32_t* pair_dcnt;
  const int64_t* pair_off;
  const int64_t* psize;
  const int64_t* psyn;
  const int64_t* pax;
  int64_t k;
  hg_limits lim;
  uint64_t* prop_key;  // [V]: sort key of the move, or ~0 for none
  int32_t* prop_to;    // [V]
  int32_t* has;        // [V]
  int32_t* work;
};

// A work-group per vertex: save and the incident weight, then conn and hit
// per part in LDS arrays over ranges of kRange part ids; best feasible move.
__global__ __launch_bounds__(kPropThreads) void propose_kernel(ProposeArgs a) {
  constexpr int NW = kPropThreads / kWave;
  __shared__ int32_t conn[kRange];
  __shared__ int32_t hit[kRange];
  __shared__ int64_t red[2 * NW];
  __shared__ uint64_t bred[NW];
  __shared__ int32_t s_item;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int64_t V = a.dims->V;
  for (int i = tid; i < kRange; i += kPropThreads) {
    conn[i] = 0;
    hit[i] = 0;
  }
  while (true) {
    __syncthreads();
    if (tid == 0) s_item = atomicAdd(a.work, 1);
    __syncthreads();
    const int64_t n = s_item;
    if (n >= V) break;
    const int32_t A = a.part[n];
    const int64_t beg = a.voff[n], deg = a.voff[n + 1] - beg;
    // save(n) and the incident weight
    int64_t save = 0, whole = 0;
    for (int64_t j = wid; j < deg; j += NW) {
      const uint32_t e = a.vinc[beg + j] & kIdMask;
      const int64_t w = a.w[e];
      if (lane == 0) whole += w;
      const uint64_t want = (uint64_t)e * (uint64_t)a.k + (uint64_t)A;
      for (int64_t q = a.pair_off[e] + lane; q < a.pair_off[e + 1]; q += kWave)
        if (a.pair_key[q] == want && a.pair_cnt[q] == 1) save += w;
    }
#pragma unroll
    for (int s = kWave / 2; s > 0; s >>= 1) {
      save += __shfl_xor(save, s, kWave);
      whole += __shfl_xor(whole, s, kWave);
    }
    if (lane == 0) {
      red[wid] = save;
      red[NW + wid] = whole;
    }
    __syncthreads();
    save = 0;
    whole = 0;
    for (int x = 0; x < NW; ++x) {
      save += red[x];
      whole += red[NW + x];
    }
    const int64_t size_n = a.size[n], syn_n = a.syn[n], ax_n = a.ax[n];
    uint64_t best = 0;
    for (int64_t r0 = 0; r0 < a.k; r0 += kRange) {  // block-uniform
      const int64_t r1 = r0 + kRange < a.k ? r0 + kRange : a.k;
      __syncthreads();  // arrays clear
      for (int64_t j = wid; j < deg; j += NW) {
        const uint32_t ent = a.vinc[beg + j];
        const uint32_t e = ent & kIdMask;
        const int32_t w = a.w[e];
        const int32_t m = (ent & kDst) ? a.mult[e] : 0;
        for (int64_t q = a.pair_off[e] + lane; q < a.pair_off[e + 1]; q += kWave) {
          const int64_t p = (int64_t)(a.pair_key[q] % (uint64_t)a.k);
          if (p != A && p >= r0 && p < r1) {
            atomicAdd(&conn[p - r0], w);
            if (m && a.pair_dcnt[q] > 0) atomicAdd(&hit[p - r0], m);
          }
        }
      }
      __syncthreads();
      for (int64_t i = tid; i < r1 - r0; i += kPropThreads) {
        const int32_t c = conn[i];
        if (c > 0) {
          const int64_t p = r0 + i;
          const int64_t gain = save - (whole - c);
          const bool ok = a.psize[p] + size_n <= a.lim.max_neurons &&
                          a.psyn[p] + syn_n <= a.lim.max_synapses &&
                          a.pax[p] + ax_n - hit[i] <= a.lim.max_axons;
          if (ok) {
            // gain in (-2^31, 2^31): biased into 32 bits; lowest part on ties
            const uint64_t key = ((uint64_t)(gain + 0x80000000ll) << 32) |
                                 (uint64_t)(0xFFFFFFFFu - (uint32_t)p);
            best = key > best ? key : best;
          }
        }
        conn[i] = 0;
        hit[i] = 0;
      }
    }
#pragma unroll
    for (int s = kWave / 2; s > 0; s >>= 1) {
      const uint64_t o = __shfl_xor(best, s, kWave);
      best = o > best ? o : best;
    }
    if (lane == 0) bred[wid] = best;
    __syncthreads();
    if (tid == 0) {
      uint64_t b = 0;
      for (int x = 0; x < NW; ++x) b = bred[x] > b ? bred[x] : b;
      if (b == 0) {
        a.has[n] = 0;
        a.prop_to[n] = -1;
        a.prop_key[n] = ~0ull;
      } else {
        const uint32_t gb = (uint32_t)(b >> 32);  // gain + 2^31
        a.has[n] = 1;
        a.prop_to[n] = (int32_t)(0xFFFFFFFFu - (uint32_t)(b & 0xFFFFFFFFull));
        // ascending order = gain descending, then vertex ascending
        a.prop_key[n] = ((uint64_t)(0xFFFFFFFFu - gb) << 32) | (uint64_t)n;
      }
    }
  }
}

__global__ void compact_moves_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ has,
                                     const int64_t* __restrict__ pos,
                                     const uint64_t* __restrict__ prop_key,
                                     uint64_t* __restrict__ mkeys, uint64_t* __restrict__ mvals) {
  const int64_t V = d->V;
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; v < V; v += stride)
    if (has[v]) {
      mkeys[pos[v]] = prop_key[v];
      mvals[pos[v]] = (uint64_t)v;
    }
}

__global__ void move_arrays_kernel(const int64_t* __restrict__ nmoves,
                                   const uint64_t* __restrict__ mvals,
                                   const int32_t* __restrict__ part,
                                   const int32_t* __restrict__ prop_to,
                                   const int64_t* __restrict__ voff, int32_t* __restrict__ m_n,
                                   int32_t* __restrict__ m_a, int32_t* __restrict__ m_b,
                                   int64_t* __restrict__ m_deg) {
  const int64_t K = *nmoves;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < K; i += stride) {
    const int32_t n = (int32_t)mvals[i];
    m_n[i] = n;
    m_a[i] = part[n];
    m_b[i] = prop_to[n];
    m_deg[i] = voff[n + 1] - voff[n];
  }
}

// Events of the recomputed gains: for move i and every hyperedge e of its
// vertex, (e, from) -1 and (e, to) +1, written in move order.
// value = i << 2 | plus << 1 | flag.
__global__ void gain_events_kernel(const int64_t* __restrict__ nmoves,
                                   const int32_t* __restrict__ m_n, const int32_t* __restrict__ m_a,
                                   const int32_t* __restrict__ m_b, const int64_t* __restrict__ moff,
                                   const int64_t* __restrict__ voff,
                                   const uint32_t* __restrict__ vinc, int64_t k,
                                   uint64_t* __restrict__ ekeys, uint64_t* __restrict__ evals) {
  const int64_t K = *nmoves;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t i = wave; i < K; i += nw) {
    const int32_t n = m_n[i];
    const uint64_t A = (uint64_t)m_a[i], B = (uint64_t)m_b[i];
    const int64_t beg = voff[n], deg = voff[n + 1] - beg;
    for (int64_t j = lane; j < deg; j += kWave) {
      const uint32_t ent = vinc[beg + j];
      const uint64_t e = ent & kIdMask, fl = ent >> 31;
      const int64_t at = 2 * (moff[i] + j);
      ekeys[at] = e * (uint64_t)k + A;
      evals[at] = ((uint64_t)i << 2) | fl;
      ekeys[at + 1] = e * (uint64_t)k + B;
      evals[at + 1] = ((uint64_t)i << 2) | 2ull | fl;
    }
  }
}

__global__ void event_delta_kernel(const uint64_t* __restrict__ evals, int64_t ne,
                                   int64_t* __restrict__ d1, int64_t* __restrict__ d2) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < ne; t += stride) {
    const uint64_t v = evals[t];
    const int64_t dl = (v & 2) ? 1 : -1;
    d1[t] = dl;
    d2[t] = (v & 1) ? dl : 0;
  }
}

// Count before each event = initial count + earlier events of its
// (hyperedge, part) segment.  Adds the event's share of its move's
// recomputed gain, and writes the event's part event: a change of the
// part's distinct axons when the hyperedge starts or stops being inbound.
__global__ void gain_scan_kernel(const uint64_t* __restrict__ ekeys,
                                 const uint64_t* __restrict__ evals, int64_t ne,
                                 const int64_t* __restrict__ s1, const int64_t* __restrict__ s2,
                                 const uint64_t* __restrict__ pair_key,
                                 const int32_t* __restrict__ pair_cnt,
                                 const int32_t* __restrict__ pair_dcnt,
                                 const int64_t* __restrict__ pair_off, int64_t k,
                                 const int32_t* __restrict__ w, const int32_t* __restrict__ mult,
                                 int64_t nmoves_cap, int64_t* __restrict__ gainp,
                                 uint64_t* __restrict__ qkey, int64_t* __restrict__ qax,
                                 int64_t q0) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < ne; t += stride) {
    const uint64_t key = ekeys[t], v = evals[t];
    const int64_t h = lower_bound_u64(ekeys, ne, key);
    const uint64_t e = key / (uint64_t)k, p = key % (uint64_t)k;
    // initial counts of (e, p)
    int64_t c0 = 0, d0 = 0;
    {
      int64_t lo = pair_off[e], hi = pair_off[e + 1];
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (pair_key[mid] < key) lo = mid + 1;
        else hi = mid;
      }
      if (lo < pair_off[e + 1] && pair_key[lo] == key) {
        c0 = pair_cnt[lo];
        d0 = pair_dcnt[lo];
      }
    }
    const int64_t before = c0 + (s1[t] - s1[h]);
    const int64_t dbefore = d0 + (s2[t] - s2[h]);
    const int64_t i = (int64_t)(v >> 2);
    const bool plus = (v & 2) != 0, fl = (v & 1) != 0;
    int64_t g = 0;
    if (!plus && before == 1) g = w[e];
    if (plus && before == 0) g = -(int64_t)w[e];
    if (g) atomicAdd((unsigned long long*)&gainp[i], (unsigned long long)g);
    int64_t dax = 0;
    if (fl && !plus && dbefore == 1) dax = -(int64_t)mult[e];
    if (fl && plus && dbefore == 0) dax = mult[e];
    qkey[q0 + t] = p * (uint64_t)nmoves_cap + (uint64_t)i;
    qax[q0 + t] = dax;
  }
}

// The moves' own part events: (from, i) less the vertex, (to, i) plus it.
__global__ void move_part_events_kernel(const int64_t* __restrict__ nmoves,
                                        const int32_t* __restrict__ m_n,
                                        const int32_t* __restrict__ m_a,
                                        const int32_t* __restrict__ m_b,
                                        const int32_t* __restrict__ size,
                                        const int32_t* __restrict__ syn,
                                        const int64_t* __restrict__ internal, int64_t nmoves_cap,
                                        uint64_t* __restrict__ qkey, int64_t* __restrict__ qsize,
                                        int64_t* __restrict__ qsyn, int64_t* __restrict__ qax) {
  const int64_t K = *nmoves;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < K; i += stride) {
    const int32_t n = m_n[i];
    const int64_t s = size[n], y = syn[n], x = internal[n];
    qkey[2 * i] = (uint64_t)m_a[i] * (uint64_t)nmoves_cap + (uint64_t)i;
    qsize[2 * i] = -s;
    qsyn[2 * i] = -y;
    qax[2 * i] = -x;
    qkey[2 * i + 1] = (uint64_t)m_b[i] * (uint64_t)nmoves_cap + (uint64_t)i;
    qsize[2 * i + 1] = s;
    qsyn[2 * i + 1] = y;
    qax[2 * i + 1] = x;
  }
}

__global__ void iota_u64_kernel(uint64_t* __restrict__ a, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) a[t] = (uint64_t)t;
}

__global__ void gather3_kernel(const uint64_t* __restrict__ idx, int64_t n,
                               const int64_t* __restrict__ a, const int64_t* __restrict__ b,
                               const int64_t* __restrict__ c, int64_t* __restrict__ oa,
                               int64_t* __restrict__ ob, int64_t* __restrict__ oc) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) {
    const uint64_t j = idx[t];
    oa[t] = a[j];
    ob[t] = b[j];
    oc[t] = c[j];
  }
}

__device__ inline int crossing(int64_t init, int64_t before, int64_t after, int64_t lim) {
  if (init > lim) return 0;  // only limits the part met before the round
  if (before <= lim && after > lim) return 1;
  if (before > lim && after <= lim) return -1;
  return 0;
}

// Per part, its totals in move order: violations added or removed per move.
__global__ void violation_kernel(const uint64_t* __restrict__ qkey, int64_t nq,
                                 const int64_t* __restrict__ ds, const int64_t* __restrict__ dy,
                                 const int64_t* __restrict__ dx, const int64_t* __restrict__ ss,
                                 const int64_t* __restrict__ sy, const int64_t* __restrict__ sx,
                                 const int64_t* __restrict__ psize,
                                 const int64_t* __restrict__ psyn,
                                 const int64_t* __restrict__ pax, int64_t nmoves_cap,
                                 hg_limits lim, int32_t* __restrict__ viol) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; t < nq; t += stride) {
    const uint64_t key = qkey[t];
    const uint64_t p = key / (uint64_t)nmoves_cap, i = key % (uint64_t)nmoves_cap;
    const int64_t h = lower_bound_u64(qkey, nq, p * (uint64_t)nmoves_cap);
    const int64_t bs = psize[p] + (ss[t] - ss[h]), by = psyn[p] + (sy[t] - sy[h]),
                  bx = pax[p] + (sx[t] - sx[h]);
    const int c = crossing(psize[p], bs, bs + ds[t], lim.max_neurons) +
                  crossing(psyn[p], by, by + dy[t], lim.max_synapses) +
                  crossing(pax[p], bx, bx + dx[t], lim.max_axons);
    if (c) atomicAdd(&viol[i], c);
  }
}

// Cumulative recomputed gain and violations per prefix; the best prefix.
__global__ void best_prefix_kernel(const int64_t* __restrict__ nmoves,
                                   const int64_t* __restrict__ gscan,
                                   const int64_t* __restrict__ vscan,
                                   unsigned long long* __restrict__ best_gain) {
  const int64_t K = *nmoves;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < K; i += stride) {
    const int64_t g = gscan[i + 1], v = vscan[i + 1];
    if (v == 0 && g > 0) atomicMax(best_gain, (unsigned long long)g);
  }
}

__global__ void best_len_kernel(const int64_t* __restrict__ nmoves,
                                const int64_t* __restrict__ gscan,
                                const int64_t* __restrict__ vscan,
                                const unsigned long long* __restrict__ best_gain,
                                unsigned long long* __restrict__ best_len) {
  const int64_t K = *nmoves;
  const int64_t bg = (int64_t)*best_gain;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < K; i += stride)
    if (bg > 0 && vscan[i + 1] == 0 && gscan[i + 1] == bg)
      atomicMin(best_len, (unsigned long long)(i + 1));
}

__global__ void apply_kernel(const int32_t* __restrict__ m_n, const int32_t* __restrict__ m_b,
                             int64_t len, int32_t* __restrict__ part) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < len; i += stride) part[m_n[i]] = m_b[i];
}

__global__ void set_i64_kernel(int64_t* p, int64_t v) { *p = v; }
__global__ void copy_i64_kernel(const int64_t* __restrict__ src, int64_t* __restrict__ dst) {
  *dst = *src;
}

int bits_for(uint64_t x) {
  int b = 0;
  while (b < 64 && (x >> b) != 0) ++b;
  return b;
}

}  // namespace
}  // namespace hg

using namespace hg;

namespace {

struct RefineScratch {
  Dims* dims;
  int32_t* vcount;
  int64_t* voff;
  uint32_t* vinc;
  int64_t* partials;
  int32_t* map;      // checked copy of the partition (the one refined)
  int32_t* nparts;   // device scalar
  uint64_t *k1, *v1, *k2, *v2;  // sort buffers, nmax entries each
  int32_t* counts;
  int64_t* offsets;
  int64_t* dn;
  int32_t* head;     // [nmax]
  int64_t* pos;      // [nmax + 1]
  uint64_t* pair_key;
  int32_t *pair_cnt, *pair_dcnt, *pcount;
  int64_t* pair_off;
  int64_t* np;
  int64_t* internal;
  int64_t *psize, *psyn, *pax;
  uint64_t* prop_key;
  int32_t *prop_to, *has, *work;
  int64_t* hpos;
  int32_t *m_n, *m_a, *m_b;
  int64_t *m_deg, *moff;
  int64_t *d1, *d2, *s1, *s2;  // [nmax (+1)]
  int64_t* gainp;
  int64_t *qsize, *qsyn, *qax;   // part events by slot
  int64_t *gs, *gy, *gx;         // gathered in sorted order
  int64_t *ss, *sy, *sx;         // their scans
  int32_t* viol;
  int64_t *gscan, *vscan;
  int64_t* nmoves;
  unsigned long long *best_gain, *best_len;
  int64_t* host_block;

  template <typename A>
  void carve(A& a, int64_t V, int64_t E, int64_t P, int64_t k) {
    // events: 2 per incidence entry of the moving vertices (<= 2P), part
    // events 2 per move plus one per event (<= 2V + 2P)
    const int64_t ne = 2 * P, nq = 2 * V + 2 * P;
    const int64_t nmax = (ne > nq ? ne : nq) > P ? (ne > nq ? ne : nq) : P;
    const int64_t nm = nmax > V ? nmax : V;
    dims = a.template take<Dims>(1);
    vcount = a.template take<int32_t>(V);
    voff = a.template take<int64_t>(V + 1);
    vinc = a.template take<uint32_t>(P);
    partials = a.template take<int64_t>(scan_partials_size());
    map = a.template take<int32_t>(V);
    nparts = a.template take<int32_t>(1);
    k1 = a.template take<uint64_t>(nm);
    v1 = a.template take<uint64_t>(nm);
    k2 = a.template take<uint64_t>(nm);
    v2 = a.template take<uint64_t>(nm);
    counts = a.template take<int32_t>(radix_sort_scratch(nm));
    offsets = a.template take<int64_t>(radix_sort_scratch(nm) + 1);
    dn = a.template take<int64_t>(1);
    head = a.template take<int32_t>(nm);
    pos = a.template take<int64_t>(nm + 1);
    pair_key = a.template take<uint64_t>(P);
    pair_cnt = a.template take<int32_t>(P);
    pair_dcnt = a.template take<int32_t>(P);
    pcount = a.template take<int32_t>(E);
    pair_off = a.template take<int64_t>(E + 1);
    np = a.template take<int64_t>(1);
    internal = a.template take<int64_t>(V);
    psize = a.template take<int64_t>(k);
    psyn = a.template take<int64_t>(k);
    pax = a.template take<int64_t>(k);
    prop_key = a.template take<uint64_t>(V);
    prop_to = a.template take<int32_t>(V);
    has = a.template take<int32_t>(V);
    work = a.template take<int32_t>(1);
    hpos = a.template take<int64_t>(V + 1);
    m_n = a.template take<int32_t>(V);
    m_a = a.template take<int32_t>(V);
    m_b = a.template take<int32_t>(V);
    m_deg = a.template take<int64_t>(V);
    moff = a.template take<int64_t>(V + 1);
    d1 = a.template take<int64_t>(nm);
    d2 = a.template take<int64_t>(nm);
    s1 = a.template take<int64_t>(nm + 1);
    s2 = a.template take<int64_t>(nm + 1);
    gainp = a.template take<int64_t>(V);
    qsize = a.template take<int64_t>(nm);
    qsyn = a.template take<int64_t>(nm);
    qax = a.template take<int64_t>(nm);
    gs = a.template take<int64_t>(nm);
    gy = a.template take<int64_t>(nm);
    gx = a.template take<int64_t>(nm);
    ss = a.template take<int64_t>(nm + 1);
    sy = a.template take<int64_t>(nm + 1);
    sx = a.template take<int64_t>(nm + 1);
    viol = a.template take<int32_t>(V);
    gscan = a.template take<int64_t>(V + 1);
    vscan = a.template take<int64_t>(V + 1);
    nmoves = a.template take<int64_t>(1);
    best_gain = a.template take<unsigned long long>(1);
    best_len = a.template take<unsigned long long>(1);
  }
};

int read_i64(hg_ctx* c, const int64_t* d, int64_t* h) {
  hipError_t e = hipMemcpyAsync(h, d, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "refinement read-back");
  return HG_OK;
}

}  // namespace

extern "C" {

int hg_refine(hg_ctx* c, const hg_level* lvl, int32_t* part, int32_t n_parts,
              const hg_limits* lim, int32_t max_rounds, int64_t* info) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_level(c, lvl, true);
  if (rc) return rc;
  if ((lvl->n_vertices > 0 && !part) || !lim || !info)
    return fail(c, HG_ERR_INVALID_ARG, "null argument");
  if (n_parts < 1 || n_parts > (lvl->n_vertices > 0 ? lvl->n_vertices : 1) || max_rounds < 0)
    return fail(c, HG_ERR_INVALID_ARG, "n_parts %d outside [1, V] or negative max_rounds",
                n_parts);
  if (c->validate && (rc = hg_validate_level(c, lvl)) != HG_OK) return rc;
  for (int i = 0; i < 4; ++i) info[i] = 0;
  const int64_t V = lvl->n_vertices, E = lvl->n_edges, P = lvl->n_pins, k = n_parts;
  if (V == 0 || max_rounds == 0) return HG_OK;
  Sizer sz;
  {
    RefineScratch S;
    S.carve(sz, V, E, P, k);
  }
  rc = ensure_arena(c, sz.off);
  if (rc) return rc;
  Carver cv{c->arena};
  RefineScratch S;
  S.carve(cv, V, E, P, k);
  hipStream_t s = c->stream;
  set_dims(S.dims, V, E, P, s);
  LevelView L = view_of(lvl, S.dims);
  const int gV = grid_for(V, 256, 16384), gP = grid_for(P, 256, 16384);
  const int gEw = grid_for(E, 4, 16384), gVw = grid_for(V, 4, 16384);
  // the partition, checked (values in [0, n_parts)), refined in S.map
  fill_i32(S.nparts, n_parts, 1, s);
  check_map_kernel_launch(part, V, S.nparts, S.map, nullptr, c->dev_err, s);
  build_incidence(L, V, E, P, S.vcount, S.voff, S.vinc, S.partials, s);
  internal_kernel<<<gVw, 256, 0, s>>>(S.dims, S.voff, S.vinc, lvl->edge_mult, lvl->v_axons,
                                      S.internal);
  const int dev_cus = device_cu_count();
  for (int32_t round = 0; round < max_rounds; ++round) {
    // ---- pins(p, e): pin keys sorted, runs ---------------------------------
    pin_keys_kernel<<<gEw, 256, 0, s>>>(S.dims, L.eoff, L.pins, S.map, k, S.k1, S.v1);
    radix_sort_pairs(S.k1, S.v1, S.k2, S.v2, P, 1 + bits_for((uint64_t)E * (uint64_t)k),
                     S.counts, S.offsets, S.dn, S.partials, s);
    run_head_kernel<<<gP, 256, 0, s>>>(S.k1, P, S.head);
    set_i64_kernel<<<1, 1, 0, s>>>(S.dn, P);
    exclusive_scan_i32(S.head, S.pos, S.dn, P, S.partials, s);
    copy_i64_kernel<<<1, 1, 0, s>>>(S.pos + P, S.np);
    fill_i32(S.pair_cnt, 0, P, s);
    fill_i32(S.pair_dcnt, 0, P, s);
    fill_i32(S.pcount, 0, E, s);
    run_fill_kernel<<<gP, 256, 0, s>>>(S.k1, P, k, S.head, S.pos, S.pair_key, S.pair_cnt,
                                       S.pair_dcnt, S.pcount);
    exclusive_scan_i32(S.pcount, S.pair_off, &S.dims->E, E, S.partials, s);
    // ---- part state --------------------------------------------------------
    fill_i64(S.psize, 0, k, s);
    fill_i64(S.psyn, 0, k, s);
    fill_i64(S.pax, 0, k, s);
    part_state_vertex_kernel<<<gV, 256, 0, s>>>(S.dims, S.map, lvl->v_size, lvl->v_syn,
                                                 S.internal, S.psize, S.psyn, S.pax);
    part_state_pair_kernel<<<gP, 256, 0, s>>>(S.pair_key, S.pair_dcnt, S.np, k, lvl->edge_mult,
                                               S.pax);
    // ---- proposals ---------------------------------------------------------
    fill_i32(S.work, 0, 1, s);
    ProposeArgs pa{S.dims,       S.voff,   S.vinc,      lvl->edge_weight, lvl->edge_mult,
                   lvl->v_size,  lvl->v_syn, lvl->v_axons, S.map,          S.pair_key,
                   S.pair_cnt,   S.pair_dcnt, S.pair_off, S.psize,          S.psyn,
                   S.pax,        k,          *lim,       S.prop_key,       S.prop_to,
                   S.has,        S.work};
    propose_kernel<<<dev_cus * 2, kPropThreads, 0, s>>>(pa);
    exclusive_scan_i32(S.has, S.hpos, &S.dims->V, V, S.partials, s);
    copy_i64_kernel<<<1, 1, 0, s>>>(S.hpos + V, S.nmoves);
    compact_moves_kernel<<<gV, 256, 0, s>>>(S.dims, S.has, S.hpos, S.prop_key, S.k1, S.v1);
    int64_t K = 0;
    if ((rc = read_i64(c, S.nmoves, &K)) != HG_OK) return rc;
    info[3] = K;
    if (K == 0) {
      info[0] = round + 1;
      break;
    }
    // ---- order ---------------------------------------------------------------
    radix_sort_pairs(S.k1, S.v1, S.k2, S.v2, K, 64, S.counts, S.offsets, S.dn, S.partials, s);
    move_arrays_kernel<<<gV, 256, 0, s>>>(S.nmoves, S.v1, S.map, S.prop_to, S.voff, S.m_n,
                                          S.m_a, S.m_b, S.m_deg);
    set_i64_kernel<<<1, 1, 0, s>>>(S.dn, K);
    exclusive_scan_i64(S.m_deg, S.moff, S.dn, V, S.partials, s);
    int64_t D = 0;
    if ((rc = read_i64(c, S.moff + K, &D)) != HG_OK) return rc;
    const int64_t NE = 2 * D, NQ = 2 * K + NE;
    const int gNE = grid_for(NE, 256, 16384), gNQ = grid_for(NQ, 256, 16384);
    // ---- recomputed gains -----------------------------------------------------
    gain_events_kernel<<<grid_for(K, 4, 16384), 256, 0, s>>>(
        S.nmoves, S.m_n, S.m_a, S.m_b, S.moff, S.voff, S.vinc, k, S.k1, S.v1);
    radix_sort_pairs(S.k1, S.v1, S.k2, S.v2, NE, bits_for((uint64_t)E * (uint64_t)k),
                     S.counts, S.offsets, S.dn, S.partials, s);
    event_delta_kernel<<<gNE, 256, 0, s>>>(S.v1, NE, S.d1, S.d2);
    set_i64_kernel<<<1, 1, 0, s>>>(S.dn, NE);
    exclusive_scan_i64(S.d1, S.s1, S.dn, NE, S.partials, s);
    exclusive_scan_i64(S.d2, S.s2, S.dn, NE, S.partials, s);
    fill_i64(S.gainp, 0, K, s);
    move_part_events_kernel<<<gV, 256, 0, s>>>(S.nmoves, S.m_n, S.m_a, S.m_b, lvl->v_size,
                                               lvl->v_syn, S.internal, K, S.k2, S.qsize,
                                               S.qsyn, S.qax);
    fill_i64(S.qsize + 2 * K, 0, NE, s);
    fill_i64(S.qsyn + 2 * K, 0, NE, s);
    gain_scan_kernel<<<gNE, 256, 0, s>>>(S.k1, S.v1, NE, S.s1, S.s2, S.pair_key, S.pair_cnt,
                                         S.pair_dcnt, S.pair_off, k, lvl->edge_weight,
                                         lvl->edge_mult, K, S.gainp, S.k2, S.qax, 2 * K);
    // ---- validity ---------------------------------------------------------------
    iota_u64_kernel<<<gNQ, 256, 0, s>>>(S.v2, NQ);
    // the part events move to (k1, v1) sorted; (k2, v2) are free afterwards
    (void)hipMemcpyAsync(S.k1, S.k2, NQ * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(S.v1, S.v2, NQ * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    radix_sort_pairs(S.k1, S.v1, S.k2, S.v2, NQ, bits_for((uint64_t)k * (uint64_t)K), S.counts,
                     S.offsets, S.dn, S.partials, s);
    gather3_kernel<<<gNQ, 256, 0, s>>>(S.v1, NQ, S.qsize, S.qsyn, S.qax, S.gs, S.gy, S.gx);
    set_i64_kernel<<<1, 1, 0, s>>>(S.dn, NQ);
    exclusive_scan_i64(S.gs, S.ss, S.dn, NQ, S.partials, s);
    exclusive_scan_i64(S.gy, S.sy, S.dn, NQ, S.partials, s);
    exclusive_scan_i64(S.gx, S.sx, S.dn, NQ, S.partials, s);
    fill_i32(S.viol, 0, K, s);
    violation_kernel<<<gNQ, 256, 0, s>>>(S.k1, NQ, S.gs, S.gy, S.gx, S.ss, S.sy, S.sx, S.psize,
                                         S.psyn, S.pax, K, *lim, S.viol);
    // ---- selection --------------------------------------------------------------
    set_i64_kernel<<<1, 1, 0, s>>>(S.dn, K);
    exclusive_scan_i64(S.gainp, S.gscan, S.dn, K, S.partials, s);
    exclusive_scan_i32(S.viol, S.vscan, S.dn, K, S.partials, s);
    fill_u64((uint64_t*)S.best_gain, 0, 1, s);
    fill_u64((uint64_t*)S.best_len, ~0ull, 1, s);
    best_prefix_kernel<<<gV, 256, 0, s>>>(S.nmoves, S.gscan, S.vscan, S.best_gain);
    best_len_kernel<<<gV, 256, 0, s>>>(S.nmoves, S.gscan, S.vscan, S.best_gain, S.best_len);
    int64_t bg = 0, bl = 0;
    if ((rc = read_i64(c, (const int64_t*)S.best_gain, &bg)) != HG_OK) return rc;
    if ((rc = read_i64(c, (const int64_t*)S.best_len, &bl)) != HG_OK) return rc;
    info[0] = round + 1;
    if (bg <= 0) break;
    apply_kernel<<<grid_for(bl, 256, 16384), 256, 0, s>>>(S.m_n, S.m_b, bl, S.map);
    info[1] += bl;
    info[2] += bg;
  }
  // the refined partition back to the caller's array
  (void)hipMemcpyAsync(part, S.map, V * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
  return launch_status(c);
}

}  // extern "C"
