// S2: neighbour scores and candidate selection (paper, Section 4.1,
// "Coarsening", Eq. 12).
//
// For a vertex n the score of a neighbour m is the summed weight of the
// hyperedges holding both.  A work-group owns one vertex at a time and
// accumulates its histogram in an LDS hash table of packed 64-bit slots
// (key = neighbour id in the high half, score in the low half; scores never
// carry into the key because the total weight of a level is < 2^31).
//
// Neighbourhoods larger than the table are processed in passes over
// contiguous ranges of neighbour ids.  Pins are ascending inside every
// hyperedge, so one cursor per incident hyperedge walks it across the passes
// and every pin is read once per pass that contains it.  A pass that would
// overfill the table is abandoned and retried with half the id range; a
// nearly empty pass doubles the range.
//
// Candidate = valid neighbour with the largest (score, -id), i.e. lowest id
// on ties.  Validity (Section 3 limits on the merged super-node) is tested
// only for table entries that beat the current best, and skipped entirely
// when the level maxima show that every neighbour of n is valid.  The
// distinct-axon overlap of n and m is needed only when ax_n + ax_m exceeds
// Delta; it is then the summed multiplicity of hyperedges in which both n and
// m carry the destination flag, found by binary search of m in n's inbound
// hyperedges.
#include "hg_internal.h"

namespace hg {

namespace {

constexpr uint64_t kEmpty = 0xFFFFFFFF00000000ull;

__device__ inline uint32_t slot_hash(uint32_t id, int shift) {
  return (id * 0x9E3779B1u) >> shift;
}

constexpr uint32_t kNoSlot = 0x40000000u;
constexpr int kMaxPasses = 1 << 16;

// Adds `wt` to the score of `id`; returns the slot, with bit 31 set when the
// entry is new.  The callers keep the table at most about half full, so the
// probe bound (the table size) is never reached by a correct run; if it is,
// the error word says so and kNoSlot is returned.  The probe loop has a
// single exit test (bitwise, not short-circuit), which keeps the mask
// bookkeeping of the divergent loop to a few scalar instructions a round.
__device__ inline uint32_t table_add(uint64_t* table, uint32_t mask, int shift, uint32_t id,
                                     uint32_t wt, int32_t* err) {
  uint32_t h = slot_hash(id, shift) & mask;
  const uint64_t mine = ((uint64_t)id << 32) | wt;
  uint64_t old;
  uint32_t probe = 0;
  while (true) {
    old = atomicCAS((unsigned long long*)&table[h], (unsigned long long)kEmpty,
                    (unsigned long long)mine);
    ++probe;
    const bool stop = (old == kEmpty) | ((uint32_t)(old >> 32) == id) | (probe > mask);
    if (stop) break;
    h = (h + 1) & mask;
  }
  if (old == kEmpty) return h | 0x80000000u;
  if ((uint32_t)(old >> 32) == id) {
    atomicAdd((unsigned long long*)&table[h], (unsigned long long)wt);
    return h;
  }
  atomicOr(err, kErrTableFull);
  return kNoSlot;
}

__device__ inline int log2_pow2(uint32_t c) { return 31 - __clz(c); }

// A value that is the same in every lane (e.g. read from LDS at a
// wave-uniform address), moved to a scalar register so that the control flow
// depending on it stays scalar.
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

// Scans the first `cap` slots: folds entries into `best`, empties them.
template <bool OV>
__device__ inline void drain_table(uint64_t* table, uint32_t* ovtab, int cap,
                                   const ScoreArgs& a, const VertexCtx& v, uint64_t& best,
                                   int tid, int nthreads) {
  for (int i = tid; i < cap; i += nthreads) {
    uint64_t s = table[i];
    if (s != kEmpty) {
      uint32_t id = (uint32_t)(s >> 32);
      uint64_t key = ((s & 0xFFFFFFFFull) << 32) | (uint64_t)(0x7FFFFFFFu - id);
      int64_t ov = 0;
      if (OV) {
        ov = ovtab[i];
        ovtab[i] = 0;
      }
      if (key > best && (v.all_valid || merge_valid(a, v, id, ov))) best = key;
      table[i] = kEmpty;
    }
  }
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

template <int THREADS>
__device__ inline void block_min_max_i64(int64_t& mn, int64_t& mx, int64_t* red) {
  constexpr int NW = THREADS / kWave;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    int64_t a = __shfl_xor(mn, d, kWave), b = __shfl_xor(mx, d, kWave);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) {
    red[wid] = mn;
    red[NW + wid] = mx;
  }
  __syncthreads();
  mn = red[0];
  mx = red[NW];
#pragma unroll
  for (int k = 1; k < NW; ++k) {
    mn = red[k] < mn ? red[k] : mn;
    mx = red[NW + k] > mx ? red[NW + k] : mx;
  }
  __syncthreads();
}

// One work-group per vertex, persistent over the bucket's work list.
// MULTI = false: the whole neighbourhood fits (X_n <= SLOTS / 2).
// OV = true: the distinct-axon bound can bind for these vertices, so the
// table also accumulates, per neighbour m, the multiplicity of hyperedges in
// which both n and m carry the destination flag (the shared inbound count).
template <int THREADS, int SLOTS, bool MULTI, bool OV>
__global__ __launch_bounds__(THREADS) void score_block_kernel(ScoreArgs a, int bucket,
                                                             int64_t maxV, int64_t maxP) {
  // Work inside a wave never depends on lane-specific control flow around a
  // cross-lane operation: hyperedges are dealt to waves statically (no
  // shuffled work counter), and per-wave bookkeeping in LDS is written by all
  // lanes of the wave with the same value.  A cursor is only ever written and
  // read by the wave that owns its hyperedge.
  constexpr int NW = THREADS / kWave;
  constexpr int MAXFILL = SLOTS / 2;
  static_assert(MAXFILL + NW * kWave < SLOTS, "table must never fill up");
  __shared__ uint64_t table[SLOTS];
  __shared__ uint32_t ovtab[OV ? SLOTS : 1];
  __shared__ uint64_t red[2 * NW];
  __shared__ int32_t s_item;
  __shared__ int32_t s_fill;       // fresh entries in this pass
  __shared__ int32_t s_wover[NW];  // wave saw the pass overflow

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  int32_t count = a.b.count[bucket];
  if (count > maxV) {
    if (tid == 0) atomicOr(a.err, kErrWorkCount);
    count = (int32_t)maxV;
  }
  const int32_t* list = a.b.list + (int64_t)bucket * maxV;

  for (int i = tid; i < SLOTS; i += THREADS) {
    table[i] = kEmpty;
    if (OV) ovtab[i] = 0;
  }

  while (true) {
    __syncthreads();
    if (tid == 0) s_item = atomicAdd(&a.work[bucket], 1);
    __syncthreads();
    const int32_t item = s_item;
    if (item >= count) break;

    VertexCtx v;
    v.n = list[item];
    v.beg = a.voff[v.n];
    v.deg = a.voff[v.n + 1] - v.beg;
    v.size_n = a.L.size[v.n];
    v.syn_n = a.L.syn[v.n];
    v.ax_n = a.L.ax[v.n];
    v.G = a.gc[a.L.gid ? a.L.gid[v.n] : 0];
    v.all_valid = (int64_t)v.size_n + v.G.max_size <= v.G.omega &&
                  (int64_t)v.syn_n + v.G.max_syn <= v.G.phi &&
                  (int64_t)v.ax_n + v.G.max_ax <= v.G.delta;
    const int64_t x = a.xn[v.n];
    const uint32_t n = (uint32_t)v.n;
    uint64_t best = 0;

    if (!MULTI) {
      // distinct neighbours are at most the visits and at most the other
      // vertices of the graph
      const int64_t dist = x < (int64_t)v.G.nverts - 1 ? x : (int64_t)v.G.nverts - 1;
      uint32_t cap = 64;
      while (cap < 2 * (uint64_t)dist && cap < (uint32_t)SLOTS) cap <<= 1;
      const int shift = 32 - log2_pow2(cap);
      // A wave takes 64 incidence entries at a time and sweeps the
      // concatenation of their pins 64 at a time (coarse hyperedges are
      // short, so a hyperedge per wave would leave most lanes idle).  Lane
      // l holds entry l's offset, length and prefix; a pin finds its entry
      // by a binary search over the lanes' prefixes.
      for (int64_t j0 = (int64_t)wid * kWave; j0 < v.deg; j0 += (int64_t)NW * kWave) {
        const int64_t j = j0 + lane;
        int64_t s0 = 0;
        int32_t len = 0, mu = 0;
        uint32_t wt = 0;
        if (j < v.deg) {
          const uint32_t ent = a.vinc[v.beg + j];
          const uint32_t e = ent & kIdMask;
          s0 = a.L.eoff[e];
          len = (int32_t)(a.L.eoff[e + 1] - s0);
          wt = (uint32_t)a.L.w[e];
          mu = (OV && (ent & kDst)) ? a.L.mult[e] : 0;
        }
        int32_t inc = len;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
          const int32_t o = __shfl_up(inc, d, kWave);
          inc += lane >= d ? o : 0;
        }
        const int32_t excl = inc - len;
        const int32_t total = __builtin_amdgcn_readlane(inc, kWave - 1);
        for (int32_t c = 0; c < total; c += kWave) {  // wave-uniform
          const int32_t q = c + lane;
          // last lane whose prefix is <= q (lanes past the list hold the
          // total, which no q reaches; no incident hyperedge is empty)
          int l = 0;
#pragma unroll
          for (int step = kWave / 2; step > 0; step >>= 1) {
            const int32_t ex = __shfl(excl, l + step, kWave);
            l = ex <= q ? l + step : l;
          }
          const int64_t base = __shfl(s0, l, kWave);
          const int32_t off = q - __shfl(excl, l, kWave);
          const uint32_t wl = (uint32_t)__shfl((int32_t)wt, l, kWave);
          const int32_t ml = OV ? __shfl(mu, l, kWave) : 0;
          if (q < total) {
            const uint32_t pin = a.L.pins[base + off];
            const uint32_t id = pin & kIdMask;
            if (id != n) {
              const uint32_t h = table_add(table, cap - 1, shift, id, wl, a.err);
              if (OV && ml && (pin & kDst) && h != kNoSlot)
                atomicAdd(&ovtab[h & kIdMask], (uint32_t)ml);
            }
          }
        }
      }
      __syncthreads();
      drain_table<OV>(table, ovtab, (int)cap, a, v, best, tid, THREADS);
    } else {
      constexpr uint32_t cap = SLOTS;
      const int shift = 32 - log2_pow2(cap);
      int32_t* cur = a.cursor + v.beg;          // committed cursors
      int32_t* tent = a.cursor + maxP + v.beg;  // cursors reached in this pass
      // Hyperedge j belongs to wave j % NW; within the wave, bookkeeping
      // loops spread a wave's hyperedges over its lanes.
      const int64_t own_step = (int64_t)NW * kWave;
      int64_t mn = INT64_MAX, mx = -1;
      for (int64_t j = wid + (int64_t)NW * lane; j < v.deg; j += own_step) {
        uint32_t e = a.vinc[v.beg + j] & kIdMask;
        int64_t s0 = a.L.eoff[e], e0 = a.L.eoff[e + 1];
        int64_t f = a.L.pins[s0] & kIdMask, l = a.L.pins[e0 - 1] & kIdMask;
        mn = f < mn ? f : mn;
        mx = l > mx ? l : mx;
        cur[j] = 0;
      }
      block_min_max_i64<THREADS>(mn, mx, (int64_t*)red);
      const int64_t hi_all = mx + 1;
      int64_t lo = mn;
      constexpr int64_t target = MAXFILL / 2;
      int64_t width = (hi_all - lo) * target / (x > 0 ? x : 1);
      if (width < 1) width = 1;
      int passes = 0;
      while (lo < hi_all) {
        const int64_t hi = lo + width < hi_all ? lo + width : hi_all;
        __syncthreads();  // previous pass fully drained / cleared and flags read
        if (++passes > kMaxPasses) {
          if (tid == 0) atomicOr(a.err, kErrPassLimit);
          break;
        }
        if (tid == 0) s_fill = 0;
        __syncthreads();
        bool wover = false;
        for (int64_t j = wid; j < v.deg && !wover; j += NW) {
          const uint32_t ent = a.vinc[v.beg + j];
          const uint32_t e = ent & kIdMask;
          const int64_t s0 = a.L.eoff[e], e0 = a.L.eoff[e + 1];
          const uint32_t wt = (uint32_t)a.L.w[e];
          const bool dn = OV && (ent & kDst);
          const int32_t mu = dn ? a.L.mult[e] : 0;
          int64_t c = s0 + cur[j];
          while (true) {
            const int64_t p = c + lane;
            const uint32_t pin = p < e0 ? a.L.pins[p] : 0x7FFFFFFFu;
            const uint32_t id = pin & kIdMask;
            const bool in = p < e0 && (int64_t)id < hi;
            bool fresh = false;
            if (in && id != n) {
              uint32_t h = table_add(table, cap - 1, shift, id, wt, a.err);
              fresh = (h & 0x80000000u) != 0;
              if (dn && (pin & kDst) && h != kNoSlot) atomicAdd(&ovtab[h & kIdMask], (uint32_t)mu);
            }
            const int cnt = __popcll(__ballot(in));
            const int nnew = __popcll(__ballot(fresh));
            if (nnew > 0) {  // wave-uniform
              // one lane adds the wave's new entries (a lane-varying operand
              // would make the compiler scan over all lanes)
              int32_t old = 0;
              if (lane == 0) old = atomicAdd(&s_fill, nnew);
              wover = __builtin_amdgcn_readlane(old, 0) + nnew > MAXFILL;
            }
            c += cnt;
            if (cnt < kWave || wover) break;
          }
          tent[j] = (int32_t)(c - s0);  // every lane stores the same value
        }
        s_wover[wid] = wover ? 1 : 0;  // every lane stores the same value
        __syncthreads();
        bool over = false;
        const int32_t fill = s_fill;
#pragma unroll
        for (int w = 0; w < NW; ++w) over |= s_wover[w] != 0;
        if (over) {
          for (int i = tid; i < (int)cap; i += THREADS) {
            table[i] = kEmpty;
            if (OV) ovtab[i] = 0;
          }
          width = width / 2 > 0 ? width / 2 : 1;
          continue;  // the loop head synchronises before the next pass
        }
        drain_table<OV>(table, ovtab, (int)cap, a, v, best, tid, THREADS);
        for (int64_t j = wid + (int64_t)NW * lane; j < v.deg; j += own_step) cur[j] = tent[j];
        lo = hi;
        // aim the next range at the pass target
        if (width < hi_all) {
          if (fill < target / 4) width *= 4;
          else if (fill < target) width = width * target / (fill > 0 ? fill : 1);
          if (width > hi_all) width = hi_all;
        }
      }
    }
    best = block_max_u64<THREADS>(best, red);
    if (tid == 0) {
      if (best == 0) {
        a.cand[v.n] = -1;
        a.cscore[v.n] = 0;
      } else {
        a.cand[v.n] = (int32_t)(0x7FFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull));
        a.cscore[v.n] = (int32_t)(best >> 32);
      }
    }
  }
}

// Multipass over neighbour-id ranges for vertices whose incident hyperedges
// fit in LDS.  Offsets, lengths, weights and cursors of the incident
// hyperedges are staged in LDS once per vertex; hyperedge j belongs to wave
// j % NW.  Every pass revisits all incident hyperedges, most of them for a
// few pins only, so a pass is bound by the latency of the dependent pin
// loads rather than by their bytes.  A wave therefore loads the first chunk
// of up to kBatch of its segments before it inserts any of them, and while
// it inserts a chunk whose last pin still lies in the range it already
// loads the next one.  Per chunk of 64 pins the work is a divergent probe
// loop with one exit test and two ballots; after every SLOTS/128 new entries
// of a wave, one single-lane LDS atomic both publishes them and returns the
// table fill.
template <int THREADS, int SLOTS, bool OV>
__global__ __launch_bounds__(THREADS) void score_stream_kernel(ScoreArgs a, int bucket,
                                                              int64_t maxV) {
  constexpr int NW = THREADS / kWave;
  constexpr int kBatch = 8;
  constexpr int MAXFILL = SLOTS * 5 / 8;
  constexpr uint32_t kSent = 0x7FFFFFFFu;  // id above every range end, flag clear
  // a wave publishes its new entries to the fill count every kPublish of
  // them, so the table holds at most MAXFILL + NW * (kPublish + 64) entries
  constexpr int kPublish = SLOTS / 128;
  static_assert(MAXFILL + NW * (kPublish + kWave) < SLOTS, "table must never fill up");
  __shared__ uint64_t table[SLOTS];
  __shared__ uint32_t ovtab[OV ? SLOTS : 1];
  __shared__ int64_t m_start[kMetaDeg];
  __shared__ int32_t m_len[kMetaDeg];
  __shared__ int32_t m_w[kMetaDeg];
  __shared__ int32_t m_cur[kMetaDeg];   // committed cursors
  __shared__ int32_t m_tent[kMetaDeg];  // cursors reached in the current pass
  __shared__ int32_t m_mult[OV ? kMetaDeg : 1];
  __shared__ uint64_t red[2 * NW];
  __shared__ int32_t s_item;
  __shared__ int32_t s_fill;
  __shared__ int32_t s_wover[NW];

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  int32_t count = a.b.count[bucket];
  if (count > maxV) {
    if (tid == 0) atomicOr(a.err, kErrWorkCount);
    count = (int32_t)maxV;
  }
  const int32_t* list = a.b.list + (int64_t)bucket * maxV;
  for (int i = tid; i < SLOTS; i += THREADS) {
    table[i] = kEmpty;
    if (OV) ovtab[i] = 0;
  }

  while (true) {
    __syncthreads();
    if (tid == 0) s_item = atomicAdd(&a.work[bucket], 1);
    __syncthreads();
    const int32_t item = s_item;
    if (item >= count) break;

    VertexCtx v;
    v.n = list[item];
    v.beg = a.voff[v.n];
    v.deg = a.voff[v.n + 1] - v.beg;
    v.size_n = a.L.size[v.n];
    v.syn_n = a.L.syn[v.n];
    v.ax_n = a.L.ax[v.n];
    v.G = a.gc[a.L.gid ? a.L.gid[v.n] : 0];
    v.all_valid = (int64_t)v.size_n + v.G.max_size <= v.G.omega &&
                  (int64_t)v.syn_n + v.G.max_syn <= v.G.phi &&
                  (int64_t)v.ax_n + v.G.max_ax <= v.G.delta;
    const int64_t x = a.xn[v.n];
    // pass target: fill16/16 of the slots, never above the fill bound
    const int64_t target = (int64_t)SLOTS * (a.fill16 > 0 ? a.fill16 : 1) / 16 < MAXFILL
                               ? (int64_t)SLOTS * (a.fill16 > 0 ? a.fill16 : 1) / 16
                               : MAXFILL;
    const uint32_t n = (uint32_t)v.n;
    const int32_t deg = (int32_t)v.deg;  // <= kMetaDeg by the bucket rule
    uint64_t best = 0;
    constexpr uint32_t cap = SLOTS;
    const int shift = 32 - log2_pow2(cap);

    int64_t mn = INT64_MAX, mx = -1;
    for (int j = tid; j < deg; j += THREADS) {
      const uint32_t ent = a.vinc[v.beg + j];
      const uint32_t e = ent & kIdMask;
      const int64_t s0 = a.L.eoff[e], e0 = a.L.eoff[e + 1];
      m_start[j] = s0;
      m_len[j] = (int32_t)(e0 - s0);
      m_w[j] = a.L.w[e];
      m_cur[j] = 0;
      if (OV) m_mult[j] = (ent & kDst) ? a.L.mult[e] : 0;
      const int64_t f = a.L.pins[s0] & kIdMask, l = a.L.pins[e0 - 1] & kIdMask;
      mn = f < mn ? f : mn;
      mx = l > mx ? l : mx;
    }
    block_min_max_i64<THREADS>(mn, mx, (int64_t*)red);  // also orders the staging
    const int64_t hi_all = mx + 1;
    int64_t lo = mn;
    int64_t width = x <= 8 * (int64_t)MAXFILL
                        ? hi_all - lo
                        : (hi_all - lo) * target / (x > 0 ? x : 1);
    if (width < 1) width = 1;
    int passes = 0;
    while (lo < hi_all) {
      const int64_t hi = lo + width < hi_all ? lo + width : hi_all;
      const uint32_t hi32 = (uint32_t)hi;  // ids are below 2^31
      __syncthreads();  // previous pass drained / cleared, flags read, cursors committed
      if (++passes > kMaxPasses) {
        if (tid == 0) atomicOr(a.err, kErrPassLimit);
        break;
      }
      if (tid == 0) s_fill = 0;
      __syncthreads();
      bool over = false;
      bool lost = false;    // a probe sequence reached its bound (never, if correct)
      int32_t pending = 0;  // new entries of this wave not yet published
      for (int32_t j0 = wid; j0 < deg && !over; j0 += kBatch * NW) {
        // straight-line code, so that all kBatch loads are in flight at once;
        // positions are 32-bit offsets from each hyperedge's first pin
        uint32_t pin[kBatch];
        bool ok[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int32_t j = j0 + b * NW;
          const int32_t js = j < deg ? j : j0;
          const uint32_t* seg = a.L.pins + m_start[js];
          const int32_t len = m_len[js];
          const int32_t p = m_cur[js] + lane;
          ok[b] = j < deg && p < len;
          pin[b] = seg[p < len ? p : len - 1];  // an incident hyperedge is never empty
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) pin[b] = ok[b] ? pin[b] : kSent;
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int32_t j = j0 + b * NW;
          if (j >= deg || over) break;  // wave-uniform
          const uint32_t* seg = a.L.pins + m_start[j];
          const int32_t len = m_len[j];
          const uint32_t wt = (uint32_t)m_w[j];
          const int32_t mu = OV ? m_mult[j] : 0;
          int32_t c = m_cur[j];
          uint32_t cur = pin[b];
          while (true) {
            // the segment goes on past this chunk iff its last lane holds a
            // pin below the range end (pins ascend; a lane past the
            // hyperedge holds the sentinel)
            const uint32_t last = __builtin_amdgcn_readlane(cur, kWave - 1);
            const bool cont = (last & kIdMask) < hi32 && c + kWave < len;
            // issued before the inserts so that its latency hides behind them
            const int32_t pn = c + kWave + lane;
            uint32_t nxt = kSent;
            if (cont) nxt = seg[pn < len ? pn : len - 1];  // wave-uniform
            const uint32_t id = cur & kIdMask;
            const bool in = id < hi32;
            bool fresh = false;
            if (in && id != n) {
              // plain divergent probe loop with a single exit: a lane leaves
              // as soon as its slot is found, and the loop ends when no lane
              // is left (nothing in it crosses lanes).  The table is never
              // full, so every probe sequence ends within `cap` rounds; the
              // bound only guards against a broken invariant.
              uint32_t h = slot_hash(id, shift);
              const uint64_t mine = ((uint64_t)id << 32) | wt;
              uint64_t old;
              uint32_t probe = 0;
              while (true) {
                old = atomicCAS((unsigned long long*)&table[h], (unsigned long long)kEmpty,
                                (unsigned long long)mine);
                ++probe;
                // bitwise, not short-circuit: one exit test, no branches
                const bool stop = (old == kEmpty) | ((uint32_t)(old >> 32) == id) | (probe >= cap);
                if (stop) break;
                h = (h + 1) & (cap - 1);
              }
              fresh = old == kEmpty;
              const bool hit = !fresh && (uint32_t)(old >> 32) == id;
              lost |= !fresh && !hit;
              // unconditional: a lane that did not hit adds 0 to its own new
              // entry (cheaper than another divergent region)
              atomicAdd((unsigned long long*)&table[h], (unsigned long long)(hit ? wt : 0u));
              if (OV && mu && (cur & kDst) && (fresh || hit)) atomicAdd(&ovtab[h], (uint32_t)mu);
            }
            const int cnt = __popcll(__ballot(in));
            pending += __popcll(__ballot(fresh));
            if (pending >= kPublish) {  // wave-uniform
              // one lane publishes the wave's new entries (a lane-varying
              // operand would make the compiler scan over all lanes)
              int32_t old = 0;
              if (lane == 0) old = atomicAdd(&s_fill, pending);
              over = __builtin_amdgcn_readlane(old, 0) + pending > MAXFILL;
              pending = 0;
            }
            c += cnt;
            if (!cont || over) break;
            cur = pn < len ? nxt : kSent;
          }
          m_tent[j] = c;  // every lane stores the same value
        }
      }
      if (__ballot(lost) != 0 && lane == 0) atomicOr(a.err, kErrTableFull);
      if (pending > 0) {  // wave-uniform
        int32_t old = 0;
        if (lane == 0) old = atomicAdd(&s_fill, pending);
        over = over || __builtin_amdgcn_readlane(old, 0) + pending > MAXFILL;
      }
      s_wover[wid] = over ? 1 : 0;  // every lane stores the same value
      __syncthreads();
      bool any_over = false;
#pragma unroll
      for (int w = 0; w < NW; ++w) any_over |= s_wover[w] != 0;
      const int32_t fill = s_fill;
      if (any_over) {
        for (int i = tid; i < (int)cap; i += THREADS) {
          table[i] = kEmpty;
          if (OV) ovtab[i] = 0;
        }
        width = width / 2 > 0 ? width / 2 : 1;
        continue;  // the loop head synchronises before the next pass
      }
      drain_table<OV>(table, ovtab, (int)cap, a, v, best, tid, THREADS);
      for (int jj = tid; jj < deg; jj += THREADS) m_cur[jj] = m_tent[jj];
      lo = hi;
      // aim the next range at the pass target
      if (width < hi_all) {
        if (fill < target / 4) width *= 4;
        else if (fill < target) width = width * target / (fill > 0 ? fill : 1);
        if (width > hi_all) width = hi_all;
      }
    }
    best = block_max_u64<THREADS>(best, red);
    if (tid == 0) {
      if (best == 0) {
        a.cand[v.n] = -1;
        a.cscore[v.n] = 0;
      } else {
        a.cand[v.n] = (int32_t)(0x7FFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull));
        a.cscore[v.n] = (int32_t)(best >> 32);
      }
    }
  }
}

// Multipass over windows of neighbour ids for vertices whose incident
// hyperedges fit in LDS (no distinct-axon overlap needed).  In a large
// neighbourhood most neighbours share a single hyperedge with n: the score
// of such a neighbour is that hyperedge's weight, known from the visit
// itself, and needs no table.  Per window [lo, lo + width) of ids, width at
// most kWinIds:
//   sweep 1 walks each incident hyperedge from its cursor to the window end,
//     setting one LDS bit per visited id; a visit that finds its bit already
//     set enters the id, as repeated, in a small LDS hash table (key only);
//   the bitmap is then rebuilt to hold just the repeated ids;
//   sweep 2 visits the same pins again, flattened over the known slices: a
//     repeated id adds the hyperedge weight to its table entry, any other id
//     has its complete score and is compared with the lane's best;
//   the table is folded into the best (validity tested only for entries that
//     beat it) and emptied.
// A window whose repeated ids would overfill the table is abandoned and
// retried at half the width.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void score_window_kernel(ScoreArgs a, int bucket,
                                                              int64_t maxV) {
  constexpr int NW = THREADS / kWave;
  constexpr int kBatch = 8;
  constexpr uint32_t kWinIds = 1u << 19;
  constexpr int kWords = (int)(kWinIds / 32);
  constexpr int HSLOTS = 8192;
  constexpr int HMAX = HSLOTS / 2;
  constexpr int kPublish = 32;
  constexpr uint32_t kSent = 0x7FFFFFFFu;
  static_assert(HMAX + NW * (kPublish + kWave) < HSLOTS, "table must never fill up");
  __shared__ uint32_t seen[kWords];
  __shared__ uint64_t rtab[HSLOTS];
  __shared__ uint32_t m_start[kMetaDeg];  // pin offsets are below 2^31
  __shared__ int32_t m_len[kMetaDeg];
  __shared__ int32_t m_w[kMetaDeg];
  __shared__ int32_t m_cur[kMetaDeg];   // committed cursors
  __shared__ int32_t m_tent[kMetaDeg];  // cursors reached in the current window
  __shared__ uint64_t red[2 * NW];
  __shared__ int32_t s_item;
  __shared__ int32_t s_fill;
  __shared__ int32_t s_wover[NW];

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  int32_t count = a.b.count[bucket];
  if (count > maxV) {
    if (tid == 0) atomicOr(a.err, kErrWorkCount);
    count = (int32_t)maxV;
  }
  const int32_t* list = a.b.list + (int64_t)bucket * maxV;
  for (int i = tid; i < kWords; i += THREADS) seen[i] = 0;
  for (int i = tid; i < HSLOTS; i += THREADS) rtab[i] = kEmpty;
  const int hshift = 32 - log2_pow2(HSLOTS);

  while (true) {
    __syncthreads();
    if (tid == 0) s_item = atomicAdd(&a.work[bucket], 1);
    __syncthreads();
    const int32_t item = s_item;
    if (item >= count) break;

    VertexCtx v;
    v.n = list[item];
    v.beg = a.voff[v.n];
    v.deg = a.voff[v.n + 1] - v.beg;
    v.size_n = a.L.size[v.n];
    v.syn_n = a.L.syn[v.n];
    v.ax_n = a.L.ax[v.n];
    v.G = a.gc[a.L.gid ? a.L.gid[v.n] : 0];
    v.all_valid = (int64_t)v.size_n + v.G.max_size <= v.G.omega &&
                  (int64_t)v.syn_n + v.G.max_syn <= v.G.phi &&
                  (int64_t)v.ax_n + v.G.max_ax <= v.G.delta;
    const uint32_t n = (uint32_t)v.n;
    const int32_t deg = (int32_t)v.deg;  // <= kMetaDeg by the bucket rule
    uint64_t best = 0;

    int64_t mn = INT64_MAX, mx = -1;
    for (int j = tid; j < deg; j += THREADS) {
      const uint32_t e = a.vinc[v.beg + j] & kIdMask;
      const int64_t s0 = a.L.eoff[e], e0 = a.L.eoff[e + 1];
      m_start[j] = (uint32_t)s0;
      m_len[j] = (int32_t)(e0 - s0);
      m_w[j] = a.L.w[e];
      m_cur[j] = 0;
      const int64_t f = a.L.pins[s0] & kIdMask, l = a.L.pins[e0 - 1] & kIdMask;
      mn = f < mn ? f : mn;
      mx = l > mx ? l : mx;
    }
    block_min_max_i64<THREADS>(mn, mx, (int64_t*)red);  // also orders the staging
    const int64_t hi_all = mx + 1;
    int64_t lo = mn;
    int64_t width = hi_all - lo < (int64_t)kWinIds ? hi_all - lo : (int64_t)kWinIds;
    int passes = 0;
    while (lo < hi_all) {
      const int64_t hi = lo + width < hi_all ? lo + width : hi_all;
      const uint32_t lo32 = (uint32_t)lo, hi32 = (uint32_t)hi;  // ids are below 2^31
      __syncthreads();  // previous window drained / cleared, flags read, cursors committed
      if (++passes > kMaxPasses) {
        if (tid == 0) atomicOr(a.err, kErrPassLimit);
        break;
      }
      if (tid == 0) s_fill = 0;
      __syncthreads();

      // ---- sweep 1: seen bits, repeated ids into the table, slice ends ----
      // Per-hyperedge values read from LDS are the same for the whole wave;
      // reading them into scalar registers keeps the loop control scalar.
      bool over = false;
      int32_t pending = 0;  // repeated ids entered by this wave, not yet published
      for (int32_t j0 = wid; j0 < deg && !over; j0 += kBatch * NW) {
        uint32_t pin[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int32_t j = j0 + b * NW;
          const int32_t js = j < deg ? j : j0;
          const uint32_t st = rfl_u32(m_start[js]);
          const int32_t len = rfl_i32(m_len[js]);
          const int32_t p = rfl_i32(m_cur[js]) + lane;
          const bool ok = j < deg && p < len;
          pin[b] = a.L.pins[st + (uint32_t)(p < len ? p : len - 1)];  // never empty
          pin[b] = ok ? pin[b] : kSent;
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int32_t j = j0 + b * NW;
          if (j >= deg || over) break;  // wave-uniform
          const uint32_t* seg = a.L.pins + rfl_u32(m_start[j]);
          const int32_t len = rfl_i32(m_len[j]);
          int32_t c = rfl_i32(m_cur[j]);
          uint32_t cur = pin[b];
          while (true) {
            // the slice goes on past this chunk iff its last lane holds a pin
            // below the window end (pins ascend; lanes past the hyperedge
            // hold the sentinel)
            const uint32_t last = __builtin_amdgcn_readlane(cur, kWave - 1);
            const bool cont = (last & kIdMask) < hi32 && c + kWave < len;
            const int32_t pn = c + kWave + lane;
            uint32_t nxt = kSent;
            if (cont) nxt = seg[pn < len ? pn : len - 1];  // wave-uniform
            const uint32_t id = cur & kIdMask;
            const bool in = id < hi32;  // and >= lo: the cursor starts at the window
            const bool act = in & (id != n);
            // branch-free: an idle lane ors 0 into a word of its own
            const uint32_t rel = id - lo32;
            const uint32_t word = act ? rel >> 5 : (uint32_t)lane;
            const uint32_t bit = act ? 1u << (rel & 31) : 0u;
            const bool rep = (atomicOr(&seen[word], bit) & bit) != 0;
            if (__ballot(rep) != 0) {  // wave-uniform; rare in sparse neighbourhoods
              bool fresh = false;
              if (rep) {
                uint32_t h = slot_hash(id, hshift);
                const uint64_t mine = (uint64_t)id << 32;
                uint64_t old;
                uint32_t probe = 0;
                while (true) {
                  old = atomicCAS((unsigned long long*)&rtab[h], (unsigned long long)kEmpty,
                                  (unsigned long long)mine);
                  ++probe;
                  const bool stop = (old == kEmpty) | ((uint32_t)(old >> 32) == id) |
                                    (probe >= (uint32_t)HSLOTS);
                  if (stop) break;
                  h = (h + 1) & (HSLOTS - 1);
                }
                fresh = old == kEmpty;
                // the probe bound is never reached while the fill bound holds
                if (!fresh && (uint32_t)(old >> 32) != id) atomicOr(a.err, kErrTableFull);
              }
              pending = rfl_i32(pending + __popcll(__ballot(fresh)));
              if (pending >= kPublish) {  // wave-uniform
                // one lane publishes (a lane-varying operand would make the
                // compiler scan over all lanes)
                int32_t old = 0;
                if (lane == 0) old = atomicAdd(&s_fill, pending);
                over = __builtin_amdgcn_readlane(old, 0) + pending > HMAX;
                pending = 0;
              }
            }
            c += __popcll(__ballot(in));
            if (!cont || over) break;
            cur = pn < len ? nxt : kSent;
          }
          m_tent[j] = c;  // every lane stores the same value
        }
      }
      if (pending > 0) {  // wave-uniform
        int32_t old = 0;
        if (lane == 0) old = atomicAdd(&s_fill, pending);
        over = over || __builtin_amdgcn_readlane(old, 0) + pending > HMAX;
      }
      s_wover[wid] = over ? 1 : 0;  // every lane stores the same value
      __syncthreads();
      bool any_over = false;
#pragma unroll
      for (int w = 0; w < NW; ++w) any_over |= s_wover[w] != 0;
      const int32_t fill = s_fill;
      for (int i = tid; i < kWords; i += THREADS) seen[i] = 0;
      if (any_over) {
        for (int i = tid; i < HSLOTS; i += THREADS) rtab[i] = kEmpty;
        width = width / 2 > 0 ? width / 2 : 1;
        continue;  // the loop head synchronises before the next window
      }
      __syncthreads();  // bitmap cleared
      if (fill > 0) {
        for (int i = tid; i < HSLOTS; i += THREADS) {
          const uint64_t s = rtab[i];
          if (s != kEmpty) {
            const uint32_t rel = (uint32_t)(s >> 32) - lo32;
            atomicOr(&seen[rel >> 5], 1u << (rel & 31));
          }
        }
        __syncthreads();  // bitmap holds the repeated ids
      }

      // ---- sweep 2: the slices [m_cur, m_tent) again ----
      for (int32_t j0 = wid; j0 < deg; j0 += kBatch * NW) {
        uint32_t pin[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int32_t j = j0 + b * NW;
          const int32_t js = j < deg ? j : j0;
          const int32_t c0 = rfl_i32(m_cur[js]);
          const int32_t sl = rfl_i32(m_tent[js]) - c0;
          // a lane past the slice re-reads the slice's last pin, and an
          // empty slice (possibly at the hyperedge's end) its first pin; such
          // lanes are masked below
          const int32_t p = sl > 0 ? c0 + (lane < sl ? lane : sl - 1) : 0;
          pin[b] = a.L.pins[rfl_u32(m_start[js]) + (uint32_t)p];
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int32_t j = j0 + b * NW;
          if (j >= deg) break;  // wave-uniform
          const int32_t c0 = rfl_i32(m_cur[j]);
          const int32_t sl = rfl_i32(m_tent[j]) - c0;
          const uint32_t* seg = a.L.pins + rfl_u32(m_start[j]) + (uint32_t)c0;
          const uint32_t wt = rfl_u32(m_w[j]);
          uint32_t cur = pin[b];
          for (int32_t c = 0; c < sl; c += kWave) {  // wave-uniform
            const int32_t pn = c + kWave + lane;
            uint32_t nxt = 0;
            if (c + kWave < sl) nxt = seg[pn < sl ? pn : sl - 1];  // wave-uniform
            const uint32_t id = cur & kIdMask;
            const bool act = (c + lane < sl) & (id != n);
            const uint32_t rel = id - lo32;  // in the window for every lane
            const bool isrep = fill > 0 && ((seen[rel >> 5] >> (rel & 31)) & 1u);
            const uint64_t key = ((uint64_t)wt << 32) | (uint64_t)(kSent - id);
            if (act & !isrep & (key > best)) {
              if (v.all_valid || merge_valid(a, v, id, 0)) best = key;
            }
            const bool add = act & isrep;
            if (__ballot(add) != 0) {  // wave-uniform
              if (add) {
                uint32_t h = slot_hash(id, hshift);
                uint64_t s;
                uint32_t probe = 0;
                while (true) {
                  s = rtab[h];
                  ++probe;
                  const bool stop = ((uint32_t)(s >> 32) == id) | (s == kEmpty) |
                                    (probe >= (uint32_t)HSLOTS);
                  if (stop) break;
                  h = (h + 1) & (HSLOTS - 1);
                }
                if ((uint32_t)(s >> 32) == id)
                  atomicAdd((unsigned long long*)&rtab[h], (unsigned long long)wt);
                else  // every repeated id was entered in sweep 1
                  atomicOr(a.err, kErrTableFull);
              }
            }
            cur = nxt;
          }
        }
      }
      __syncthreads();  // sweep 2 done: table complete
      if (fill > 0) {
        for (int i = tid; i < HSLOTS; i += THREADS) {
          const uint64_t s = rtab[i];
          if (s != kEmpty) {
            const uint32_t id = (uint32_t)(s >> 32);
            const uint64_t key = ((s & 0xFFFFFFFFull) << 32) | (uint64_t)(kSent - id);
            if (key > best && (v.all_valid || merge_valid(a, v, id, 0))) best = key;
            rtab[i] = kEmpty;
            seen[(id - lo32) >> 5] = 0;
          }
        }
      }
      for (int jj = tid; jj < deg; jj += THREADS) m_cur[jj] = m_tent[jj];
      lo = hi;
      if (fill < HMAX / 4 && width < (int64_t)kWinIds) {
        width *= 2;
        if (width > (int64_t)kWinIds) width = kWinIds;
      }
    }
    best = block_max_u64<THREADS>(best, red);
    if (tid == 0) {
      if (best == 0) {
        a.cand[v.n] = -1;
        a.cscore[v.n] = 0;
      } else {
        a.cand[v.n] = (int32_t)(kSent - (uint32_t)(best & 0xFFFFFFFFull));
        a.cscore[v.n] = (int32_t)(best >> 32);
      }
    }
  }
}

__global__ void no_candidate_kernel(const Dims* __restrict__ d, int32_t* __restrict__ cand,
                                    int32_t* __restrict__ cscore, int32_t* __restrict__ work) {
  int64_t V = d->V;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (i < kNumBuckets) work[i] = 0;
  for (; i < V; i += stride) {
    cand[i] = -1;
    cscore[i] = 0;
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

void score_candidates(const ScoreArgs& a, int64_t maxV, int64_t maxP, hipStream_t s) {
  no_candidate_kernel<<<grid_for(maxV, 256, 8192), 256, 0, s>>>(a.L.dims, a.cand, a.cscore,
                                                               a.work);
  static int g[kNumBuckets] = {0};
  auto k0 = score_block_kernel<256, kSmallSlots, false, false>;
  auto k1 = score_block_kernel<512, kBigSlots, false, false>;
  auto k2 = score_window_kernel<1024>;
  auto k3 = score_block_kernel<512, kBigSlots, true, false>;
  auto k4 = score_block_kernel<256, kSmallSlots, false, true>;
  auto k5 = score_block_kernel<512, kBigSlotsOv, false, true>;
  auto k6 = score_stream_kernel<1024, kBigSlotsOv, true>;
  auto k7 = score_block_kernel<512, kBigSlotsOv, true, true>;
  if (!g[0]) {
    g[0] = persistent_grid(k0, 256);
    g[1] = persistent_grid(k1, 512);
    g[2] = persistent_grid(k2, 1024);
    g[3] = persistent_grid(k3, 512);
    g[4] = persistent_grid(k4, 256);
    g[5] = persistent_grid(k5, 512);
    g[6] = persistent_grid(k6, 1024);
    g[7] = persistent_grid(k7, 512);
  }
  k0<<<g[0], 256, 0, s>>>(a, 0, maxV, maxP);
  k1<<<g[1], 512, 0, s>>>(a, 1, maxV, maxP);
  k2<<<g[2], 1024, 0, s>>>(a, 2, maxV);
  k3<<<g[3], 512, 0, s>>>(a, 3, maxV, maxP);
  k4<<<g[4], 256, 0, s>>>(a, 4, maxV, maxP);
  k5<<<g[5], 512, 0, s>>>(a, 5, maxV, maxP);
  k6<<<g[6], 1024, 0, s>>>(a, 6, maxV);
  k7<<<g[7], 512, 0, s>>>(a, 7, maxV, maxP);
}

}  // namespace hg
