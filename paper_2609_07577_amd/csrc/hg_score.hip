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
#include <type_traits>
#include "hg_internal.h"
#include "hg_score_common.h"

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
// most kWinMax, the bitmap starts at the word holding lo (bit i of word k
// stands for id 32 (lo / 32 + k) + i), so that an id's word and bit come
// from the id alone:
//   sweep 1 visits the pins of every incident hyperedge from its cursor up
//     to the window end, setting one LDS bit per id; a visit that finds its
//     bit already set appends the id to the wave's part of a list of repeat
//     visits, and the pins below the window end are counted;
//   the bitmap is then rebuilt to hold just the repeated ids (n, visited
//     like any id, counts as repeated), and a prefix count per bitmap word
//     gives every repeated id a dense rank (the number of repeated ids below
//     it in the window);
//   sweep 2 visits the same pins again: a repeated id adds the hyperedge
//     weight to the score at its rank, any other id has its complete score
//     and is compared with the lane's best (when no merge of n can break a
//     limit, a batch lighter than one in which the wave already scored such
//     an id is not compared: it cannot hold the vertex's best);
//   the fold: each repeat visit names a repeated id, whose score (at its
//     rank) is compared with the lane's best (validity tested only for
//     those that beat it; n is left out), and the cursors move past the
//     counted pins.
// No step probes a table: each visit is one LDS bit operation, and a
// repeated one one more LDS add.  A window whose repeat visits overflow a
// wave's part of the list, or whose repeated ids could outnumber the
// scores, is abandoned and retried at half the width.
//
// Work balance: hyperedge sizes follow a heavy-tailed law, so each sweep cuts
// the vertex's slices into batches of B chunks (64 pins each) and numbers
// the batches of all hyperedges in a row; each wave starts on the batch of
// its own number and claims its next one from a counter in LDS, a fetch
// ahead (waves of one CU do not progress at one rate, and a fixed deal
// left the faster ones idle at the sweep's end).  A 16-byte list entry per hyperedge with batches holds its first
// batch number, the hyperedge, a virtual base and the end of the pins its
// batches cover, so a wave finds its next batch with one 16-byte LDS read
// per lane, a ballot and a few readlanes, and the batch's start and pin
// count with two scalar operations each.  A wave issues the B loads of its next batch before it
// processes the current one.  In sweep 1 the slice end is not known in
// advance: the batches cover an estimate of it (from the pins' id density,
// plus two standard deviations and a chunk), every pin is tested against
// the window end, and when a slice runs on past its batches the wave holding
// the last of them continues with further batches until the end.  The count
// of pins below the window end is exact whatever the estimate; a poor one
// only costs loads.  Since a hyperedge's pins ascend, that count is a batch's
// ballot of ids below the window end (lanes past the batch hold its last
// pin), capped at the batch's size.
//
// The sweeps are bound by each wave's instruction stream (a batch holds
// 150-250 useful pins), so the per-batch bookkeeping is kept scalar and
// short: lanes are tested against the batch's pin count with one compare
// per chunk, loads take a scalar base and a lane offset clamped to the
// batch's last live pin, and an id's bitmap word and bit come from the id
// (a bit-field extract and the id's low five bits) without the window
// origin subtracted first.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void score_window_kernel(ScoreArgs a, int bucket,
                                                              int64_t maxV) {
  constexpr int NW = THREADS / kWave;
  constexpr int B = 4;  // chunks per batch
  constexpr int kBatchPins = B * kWave;
  constexpr uint32_t kWinIds = 1u << 19;       // ids the bitmap holds
  constexpr int kWords = (int)(kWinIds / 32);
  // the widest window: from any lo, its ids fall in kWords words
  constexpr int64_t kWinMax = (int64_t)kWinIds - 32;
  constexpr int kList = 4096;         // repeat visits of a window
  constexpr int kSeg = kList / NW;    // a wave's part of them
  constexpr int kScores = 4096;       // repeated ids of a window
  constexpr uint32_t kSent = 0x7FFFFFFFu;
  // thread t ranks the bitmap words [16 t, 16 t + 16)
  static_assert(kWords == 16 * THREADS, "a thread owns 16 consecutive bitmap words");
  static_assert(kWinDeg <= THREADS, "thread j lists hyperedge j");
  static_assert(kWinDeg <= 1024, "a list entry holds the hyperedge in 10 bits");
  static_assert(B == 4, "the register uses name B registers");
  // One LDS block laid out by hand: the descriptors of the listed
  // hyperedges and the bitmap come first, so that their offsets fit the
  // immediate field of the LDS instructions of the sweeps.
  struct Lds {
    // The hyperedges that have batches in the current sweep, one 16-byte
    // entry each, read by a lane in one LDS access (one extra entry: its x
    // holds the number of batches):
    //   x  batches before the hyperedge
    //   y  the hyperedge j (bits 0-9) and, in sweep 1, whether its slice may
    //      run on past its batches (bit 31)
    //   z  the first pin of its slice less x * kBatchPins (modulo 2^32), so
    //      that batch b starts at pin z + b * kBatchPins
    //   w  the pin after the last its batches cover
    uint4 c_ent[kWinDeg + 1];
    alignas(16) uint32_t seen[kWords];
    // the ids of sweep 1's repeat visits, wave w's from w * kSeg on (plus a
    // slot per lane that takes no visit); they stay for the final fold
    uint32_t lst[kList + kWave];
    uint32_t sc[kScores];          // sweep 2 on: the score of each rank
    alignas(16) uint16_t wpre[kWords];  // repeated ids in the words before each word
    // the incident hyperedges
    uint32_t m_base[kWinDeg];      // first pin not yet below a window (offsets < 2^31)
    int32_t m_rem[kWinDeg];        // pins from there to the hyperedge's end
    int32_t m_w[kWinDeg];
    uint32_t m_last[kWinDeg];      // largest id of the hyperedge
    int32_t m_cnt[kWinDeg];        // pins of the slice (below the window end)
    int32_t s_wcnt[NW];            // repeat visits of each wave (-1: its part overflowed)
    int32_t ws[3 * NW];
    uint64_t red[2 * NW];
    int32_t s_item;
    int32_t s_next;                // the next batch of the sweep no wave holds
  };
  __shared__ Lds S;

  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wid = rfl_i32(tid / kWave);  // the same in every lane: keep it scalar
  int32_t count = a.b.count[bucket];
  if (count > maxV) {
    if (tid == 0) atomicOr(a.err, kErrWorkCount);
    count = (int32_t)maxV;
  }
  const int32_t* list = a.b.list + (int64_t)bucket * maxV;
  uint4* const seen4 = reinterpret_cast<uint4*>(S.seen);
  uint4* const wpre4 = reinterpret_cast<uint4*>(S.wpre);
#pragma unroll
  for (int i = 0; i < 4; ++i) seen4[4 * tid + i] = make_uint4(0u, 0u, 0u, 0u);
  // What the last completed window left in the bitmap: the words of the
  // wave's repeat visits (the bitmap starting at word prev_lw of the ids)
  // and of n (prev_nword, -1 for none).  They are cleared at the next
  // window's start.
  int32_t prev_wcnt = 0, prev_nword = -1;
  uint32_t prev_lw = 0;
  // byte offset of the lane's pin in each chunk of a batch
  uint32_t lofs[B];
#pragma unroll
  for (int u = 0; u < B; ++u) lofs[u] = (uint32_t)(u * kWave + lane) * 4u;

  while (true) {
    __syncthreads();
    if (tid == 0) S.s_item = atomicAdd(&a.work[bucket], 1);
    __syncthreads();
    const int32_t item = S.s_item;
    if (item >= count) break;

    VertexCtx v;
    v.n = list[item];
    v.beg = a.voff[v.n];
    v.deg = a.voff[v.n + 1] - v.beg;
    if (v.deg > kWinDeg) {  // block-uniform; the bucket rule excludes it
      if (tid == 0) atomicOr(a.err, kErrWorkCount);
      continue;
    }
    v.size_n = a.L.size[v.n];
    v.syn_n = a.L.syn[v.n];
    v.ax_n = a.L.ax[v.n];
    v.G = a.gc[a.L.gid ? a.L.gid[v.n] : 0];
    v.all_valid = (int64_t)v.size_n + v.G.max_size <= v.G.omega &&
                  (int64_t)v.syn_n + v.G.max_syn <= v.G.phi &&
                  (int64_t)v.ax_n + v.G.max_ax <= v.G.delta;
    const uint32_t n = (uint32_t)v.n;
    const int32_t deg = (int32_t)v.deg;  // 1 .. kWinDeg
    uint64_t best = 0;
    // the heaviest batch in which the wave has scored a single (sweep 2,
    // no merge of n invalid): the block's best key is at least sw << 32,
    // so a lighter batch holds no single that could win
    uint32_t sw = 0;

    int64_t mn = INT64_MAX, mx = -1;
    for (int j = tid; j < deg; j += THREADS) {
      const uint32_t e = a.vinc[v.beg + j] & kIdMask;
      const int64_t s0 = a.L.eoff[e], e0 = a.L.eoff[e + 1];
      S.m_base[j] = (uint32_t)s0;
      S.m_rem[j] = (int32_t)(e0 - s0);
      S.m_w[j] = a.L.w[e];
      const uint32_t f = a.L.pins[s0] & kIdMask, l = a.L.pins[e0 - 1] & kIdMask;
      S.m_last[j] = l;
      mn = (int64_t)f < mn ? (int64_t)f : mn;
      mx = (int64_t)l > mx ? (int64_t)l : mx;
    }
    block_min_max_i64<THREADS>(mn, mx, (int64_t*)S.red);  // also orders the staging
    const int64_t hi_all = mx + 1;
    int64_t lo = mn;
    int64_t width = hi_all - lo < kWinMax ? hi_all - lo : kWinMax;
    int passes = 0;

    // Lists the hyperedges with batches: thread j looks at hyperedge j and
    // passes in its chunk count nb, run-on flag, slice start and pin count,
    // and the place of its entry and first batch (from a block scan of the
    // batch counts; a hyperedge with batches takes one entry).
    auto list_write = [&](int32_t nb, bool ro, uint32_t base, int32_t r, int32_t pc,
                          int32_t pb) {
      if (nb > 0) {
        const int64_t cover = (int64_t)nb * kWave;
        S.c_ent[pc] = make_uint4((uint32_t)pb, (uint32_t)tid | (ro ? 0x80000000u : 0u),
                                 base - (uint32_t)pb * (uint32_t)kBatchPins,
                                 base + (uint32_t)(r < cover ? r : cover));
      }
    };

    // A batch: pins [base, base + lim) of hyperedge j's slice (lim = 0: no
    // batch), weight wt (sweep 2); rem (sweep 1) > 0 when the slice may run
    // on past the batch, with rem pins left in the hyperedge after it.
    struct Batch {
      uint32_t base;
      int32_t lim, j, rem;
      uint32_t wt;
    };
    int32_t nc = 0, tb = 0;  // listed hyperedges, batches of the current sweep
    int32_t bnext = 0, ci = 0;
    // The waves take batches as they go: each claims its next batch from
    // s_next one fetch ahead (the claim in lane 0 of bclaim), so that a wave
    // held up on one batch leaves the rest to the others.
    int32_t bclaim = 0;
    bool has_cont = false;
    int32_t cont_j = 0, cont_rem = 0;  // a continuation: hyperedge, pins left
    uint32_t cont_base = 0;            // and its first pin
    // The wave's next batch; its loads are issued at once (for no batch, at
    // pin 0, so that every path issues B loads).
    auto fetch = [&](Batch& t, uint32_t (&pin)[B], bool sweep1) {
      uint32_t base = 0, wt = 0;
      int32_t lim = 0, j = deg, rem = 0;
      bool took = false;  // a claimed batch taken: claim the next
      if (sweep1 && has_cont) {  // wave-uniform
        has_cont = false;
        j = cont_j;
        base = cont_base;
        lim = cont_rem < kBatchPins ? cont_rem : kBatchPins;
        rem = cont_rem - lim;
      } else if ((bnext = __builtin_amdgcn_readlane(bclaim, 0)) < tb) {  // wave-uniform
        // The last listed hyperedge (from ci on) whose first batch is at most
        // bnext: the entries are strictly increasing, so the lanes that pass
        // form a prefix, the lane at ci always among them.  Every lane reads
        // its entry, and the chosen one is taken with readlane; when all 64
        // pass, the search moves on by 63 entries (the extra entry at nc
        // holds tb, which no batch reaches, so it ends).
        // (the whole entry is read at once: left to itself the compiler
        // reads the other fields only after the search, a second round trip)
        int32_t idx = ci + lane < nc ? ci + lane : nc;
        uint4 ent = S.c_ent[idx];
        asm volatile("" : "+v"(ent.x), "+v"(ent.y), "+v"(ent.z), "+v"(ent.w));
        uint64_t m = ballot((int32_t)ent.x <= bnext);
        while (m == ~0ull) {
          ci += kWave - 1;
          idx = ci + lane < nc ? ci + lane : nc;
          ent = S.c_ent[idx];
          asm volatile("" : "+v"(ent.x), "+v"(ent.y), "+v"(ent.z), "+v"(ent.w));
          m = ballot((int32_t)ent.x <= bnext);
        }
        const int32_t e_l = (int32_t)ent.y;
        const uint32_t base_l = ent.z, end_l = ent.w;
        const int32_t sel = (int32_t)__popcll(m) - 1;
        ci += sel;
        const int32_t e = __builtin_amdgcn_readlane(e_l, sel);
        const uint32_t end = (uint32_t)__builtin_amdgcn_readlane((int32_t)end_l, sel);
        j = e & 0x3FF;
        base = (uint32_t)__builtin_amdgcn_readlane((int32_t)base_l, sel) +
               (uint32_t)bnext * (uint32_t)kBatchPins;
        const uint32_t left = end - base;  // at least 1
        lim = (int32_t)(left < (uint32_t)kBatchPins ? left : (uint32_t)kBatchPins);
        // only the batch that reaches the end of the hyperedge's listed pins
        // may find that the slice runs on (its chunks are then full); the
        // pins left are those up to the hyperedge's end
        if (sweep1 && e < 0 && left <= (uint32_t)kBatchPins)
          rem = (int32_t)(S.m_base[j] + (uint32_t)S.m_rem[j] - end);
        if (!sweep1) wt = (uint32_t)S.m_w[j];
        took = true;
      }
      t.base = rfl_u32(base);
      t.lim = rfl_i32(lim);
      t.j = rfl_i32(j);
      t.rem = rfl_i32(rem);
      t.wt = rfl_u32(wt);
      // lanes past the batch load its last live pin (a scalar bound: the
      // readfirstlane keeps the compiler from turning it into a per-lane
      // select after the clamp)
      const uint32_t last4 = rfl_u32(t.lim > 0 ? (uint32_t)(t.lim - 1) * 4u : 0u);
      const char* p = reinterpret_cast<const char*>(a.L.pins + t.base);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const uint32_t off = lofs[u] < last4 ? lofs[u] : last4;
        pin[u] = *reinterpret_cast<const uint32_t*>(p + off);
      }
      if (took) {  // wave-uniform; after the loads, so that they leave first
        int32_t c = 0;
        if (lane == 0) c = atomicAdd(&S.s_next, 1);
        bclaim = c;
      }
      // the batch's loads leave before any work on the previous batch
      __builtin_amdgcn_sched_barrier(0);
    };

    while (lo < hi_all) {
      const int64_t hi = lo + width < hi_all ? lo + width : hi_all;
      const uint32_t lo32 = (uint32_t)lo, hi32 = (uint32_t)hi;  // ids are below 2^31
      const uint32_t lw = lo32 >> 5;  // the ids' word at the bitmap's start
      // the bitmap indexed by an id's word (id / 32) itself, and the lane's
      // own word in that indexing
      uint32_t* const seenw = S.seen - lw;
      const uint32_t lane_w = (uint32_t)lane + lw;
      __syncthreads();  // previous window folded, flags read, cursors committed
      if (++passes > kMaxPasses) {
        if (tid == 0) atomicOr(a.err, kErrPassLimit);
        break;
      }
      // ---- sweep 1 batches: all remaining chunks when the hyperedge ends in
      // the window (or has at most two left), else a generous estimate of the
      // slice, flagged as possibly running on
      {
        int32_t nb = 0, r = 0, full = 0;
        uint32_t base = 0;
        if (tid < deg) {
          r = S.m_rem[tid];
          full = (r + kWave - 1) / kWave;
          nb = full;
          const uint32_t last = S.m_last[tid];
          if (last >= hi32 && full > 2) {
            // (the hardware reciprocal and square root: an estimate only,
            // and the same on every run)
            const uint32_t span = last - lo32 + 1u;
            const float est =
                (float)r * (float)(hi32 - lo32) * __builtin_amdgcn_rcpf((float)span);
            const float body = est + 2.0f * __builtin_amdgcn_sqrtf(est) + (float)kWave;
            nb = (int32_t)(body * (1.0f / (float)kWave)) + 1;
            nb = nb < full ? nb : full;
          }
          base = S.m_base[tid];
          S.m_cnt[tid] = 0;
        }
        const int32_t nbat = (nb + B - 1) / B;
        int32_t x3[3] = {nbat > 0, nbat, 0}, p3[3], t3[3];
        block_scan3<THREADS>(x3, p3, t3, S.ws);
        nc = t3[0];
        tb = t3[1];
        list_write(nb, nb < full, base, r, p3[0], p3[1]);
        if (tid == 0) {
          S.c_ent[nc].x = (uint32_t)tb;
          S.s_next = NW;  // batches 0 .. NW - 1: one for each wave to start
        }
      }
      // the bitmap starts empty: the last window left only its repeated ids
      for (int o = lane; o < prev_wcnt; o += kWave)
        S.seen[(S.lst[wid * kSeg + o] >> 5) - prev_lw] = 0;
      if (tid == 0 && prev_nword >= 0) S.seen[prev_nword] = 0;
      prev_wcnt = 0;
      prev_nword = -1;
      __syncthreads();
      bclaim = wid;
      ci = 0;
      has_cont = false;

      // ---- sweep 1 ----
      bool over = false;
      int32_t wcnt = 0;  // repeat visits in the wave's part of the list
      // A batch of sweep 1: the B chunks' bitmap updates are issued back to
      // back (one wait for all of them); lanes past the batch and pins at or
      // above the window end update a word of their own with 0.  n itself is
      // visited like any id (once per incident hyperedge): it ends up
      // repeated, and is left out when the scores are folded.
      auto process1 = [&](const Batch& t, const uint32_t (&pin)[B]) {
        const uint32_t lim4 = (uint32_t)t.lim * 4u;
        uint32_t id[B], bit[B], old[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          id[u] = pin[u] & kIdMask;
          const bool in = (lofs[u] < lim4) & (id[u] < hi32);  // ids >= lo: cursor order
          const uint32_t word = in ? id[u] >> 5 : lane_w;
          bit[u] = in ? 1u << (id[u] & 31) : 0u;
          old[u] = atomicOr(&seenw[word], bit[u]);
        }
        // the pins below the window end: the batch's pins ascend and the
        // lanes past it hold its last live pin, so the lanes below the end
        // are its first cnt pins, or all lanes when cnt is the batch's size;
        // and the repeat visits
        bool rep[B];
        uint64_t rb[B];
        int32_t nr = 0, cnt = 0;
#pragma unroll
        for (int u = 0; u < B; ++u) {
          cnt += (int32_t)__popcll(ballot(id[u] < hi32));
          rep[u] = (old[u] & bit[u]) != 0;
          rb[u] = ballot(rep[u]);
          nr += (int32_t)__popcll(rb[u]);
        }
        cnt = cnt < t.lim ? cnt : t.lim;
        if (nr > 0 && !over) {  // wave-uniform (most batches hold a few)
          if (wcnt + nr > kSeg) {
            over = true;
          } else {
            // every lane writes: a repeat visit to its place in the wave's
            // part of the list, any other lane to a slot of its own
            uint32_t at = (uint32_t)(wid * kSeg + wcnt);
            wcnt += nr;
#pragma unroll
            for (int u = 0; u < B; ++u) {
              uint32_t below = __builtin_amdgcn_mbcnt_hi(
                  (uint32_t)(rb[u] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)rb[u], 0u));
              // in every lane (left to itself the compiler computes it under
              // an exec mask of the repeat lanes, at more scalar cost)
              asm volatile("" : "+v"(below));
              S.lst[rep[u] ? at + below : (uint32_t)(kList + lane)] = id[u];
              at += (uint32_t)__popcll(rb[u]);
            }
          }
        }
        if (cnt > 0 && lane == 0) atomicAdd(&S.m_cnt[t.j], cnt);
        // the slice runs on past this batch iff the batch ends the
        // hyperedge's listed chunks (or is a continuation), pins are left
        // after it, and its last pin (lane 63 of its last chunk, which is
        // full) lies below the window end
        if (t.rem > 0 && !over) {  // wave-uniform
          const int32_t c = (t.lim >> 6) - 1;
          const uint32_t lp = c == 0 ? pin[0] : c == 1 ? pin[1] : c == 2 ? pin[2] : pin[3];
          const uint32_t last = (uint32_t)__builtin_amdgcn_readlane((int32_t)lp, kWave - 1);
          if ((last & kIdMask) < hi32) {
            has_cont = true;
            cont_j = t.j;
            cont_base = t.base + (uint32_t)t.lim;
            cont_rem = t.rem;
          }
        }
        // every batch's loads are complete here, on every path, which keeps
        // the compiler's count of loads in flight exact across the loop
        asm volatile("" ::"v"(pin[0]), "v"(pin[1]), "v"(pin[2]), "v"(pin[3]));
      };
      // One exit, at the top: an exit between the two halves would give the
      // loop a second path into its head, along which the other buffer's
      // loads are still in flight, and the compiler would then wait for them
      // at the head.
      {
        Batch ta, tb2;
        uint32_t pa[B], pb[B];
        fetch(ta, pa, true);
        while ((ta.lim > 0 || has_cont) && !over) {
          fetch(tb2, pb, true);
          process1(ta, pa);
          fetch(ta, pa, true);
          process1(tb2, pb);
        }
      }
      S.s_wcnt[wid] = over ? -1 : wcnt;  // every lane stores the same value
      __syncthreads();
      // the waves' counts, one per lane
      const int32_t wc = lane < NW ? S.s_wcnt[lane] : 0;
      bool any_over = ballot(wc < 0) != 0;
      const int32_t nrep =  // repeat visits of the window
          __builtin_amdgcn_readlane(wave_incl_scan(wc > 0 ? wc : 0), kWave - 1);
      // more repeated ids than scores (at most nrep, and n)
      any_over |= nrep >= kScores;  // more repeated ids than scores (at most nrep)
#pragma unroll
      for (int i = 0; i < 4; ++i) seen4[4 * tid + i] = make_uint4(0u, 0u, 0u, 0u);
      if (any_over) {
        width = width / 2 > 0 ? width / 2 : 1;
        continue;  // the loop head synchronises before the next window
      }
      // ---- sweep 2 batches (the exact slices), the bitmap of repeated ids
      // and their ranks.  The bitmap was cleared above; each wave sets the
      // ids of its own part of the list, and n counts as repeated, so that
      // sweep 2 never takes it for a single.  Thread t then ranks its 16
      // words: one block scan gives the list places and the ranks, stored
      // per word two to a 32-bit store; the scores start at 0.
      int32_t nb2 = 0, r2 = 0;
      uint32_t base2 = 0;
      if (tid < deg) {
        r2 = S.m_cnt[tid];
        nb2 = (r2 + kWave - 1) / kWave;
        base2 = S.m_base[tid];
      }
      __syncthreads();  // bitmap cleared
      for (int o = lane; o < wcnt; o += kWave) {
        const uint32_t id = S.lst[wid * kSeg + o];
        atomicOr(&S.seen[(id >> 5) - lw], 1u << (id & 31));
      }
      const bool n_in = n >= lo32 && n < hi32;  // block-uniform
      if (tid == 0 && n_in) atomicOr(&S.seen[(n >> 5) - lw], 1u << (n & 31));
      __syncthreads();  // repeated ids marked
      int32_t nrank = 0;  // repeated ids of the window
      {
        uint4 q[4];
        const int32_t nbat = (nb2 + B - 1) / B;
        int32_t x3[3] = {nbat > 0, nbat, 0}, p3[3], t3[3];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          q[i] = seen4[4 * tid + i];
          x3[2] += __popc(q[i].x) + __popc(q[i].y) + __popc(q[i].z) + __popc(q[i].w);
        }
        block_scan3<THREADS>(x3, p3, t3, S.ws);
        nc = t3[0];
        tb = t3[1];
        nrank = t3[2];
        list_write(nb2, false, base2, r2, p3[0], p3[1]);
        if (tid == 0) {
          S.c_ent[nc].x = (uint32_t)tb;
          S.s_next = NW;  // batches 0 .. NW - 1: one for each wave to start
        }
        uint32_t run = (uint32_t)p3[2], pk[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t r0 = run;
          run += __popc(q[i].x);
          const uint32_t r1 = run;
          run += __popc(q[i].y);
          const uint32_t r2 = run;
          run += __popc(q[i].z);
          const uint32_t r3 = run;
          run += __popc(q[i].w);
          pk[2 * i] = r0 | (r1 << 16);
          pk[2 * i + 1] = r2 | (r3 << 16);
        }
        if (nrank > 0) {  // block-uniform
          wpre4[2 * tid] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
          wpre4[2 * tid + 1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
          for (int i = tid; i < nrank; i += THREADS) S.sc[i] = 0;
        }
      }
      bclaim = wid;
      ci = 0;
      __syncthreads();  // list of batches, bitmap, ranks and scores ready

      // ---- sweep 2 ----
      // (allv: std::true_type when no merge of n can break a limit, so that
      // the loop for that case carries no validity test)
      auto process2 = [&](const Batch& t, const uint32_t (&pin)[B], auto allv) {
        if (t.lim == 0) {  // wave-uniform: no batch (its pins may lie outside
                           // the window; they are not looked at)
          asm volatile("" ::"v"(pin[0]), "v"(pin[1]), "v"(pin[2]), "v"(pin[3]));
          return;
        }
        // the B chunks' bitmap reads are issued back to back; lanes past the
        // batch hold its last live pin (inside the window)
        const uint32_t lim4 = (uint32_t)t.lim * 4u;
        uint32_t id[B], w[B];
        bool act[B], rep[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          id[u] = pin[u] & kIdMask;
          act[u] = lofs[u] < lim4;  // n is marked repeated: never a single
          w[u] = seenw[id[u] >> 5];
        }
        bool anyadd = false;
        if (decltype(allv)::value) {
#pragma unroll
          for (int u = 0; u < B; ++u) {
            rep[u] = __builtin_amdgcn_ubfe(w[u], id[u], 1u) != 0;  // (bit id % 32)
            anyadd |= act[u] & rep[u];
          }
          if (t.wt >= sw) {  // wave-uniform
            // every single scores the batch's weight: the best of them is
            // the smallest id
            uint32_t mid = kSent;
#pragma unroll
            for (int u = 0; u < B; ++u) {
              const bool single = act[u] & !rep[u];
              mid = single && id[u] < mid ? id[u] : mid;
            }
            const uint64_t key = ((uint64_t)t.wt << 32) | (uint64_t)(kSent - mid);
            best = mid != kSent && key > best ? key : best;
            if (ballot(mid != kSent) != 0) sw = t.wt;
          }
        } else {
#pragma unroll
          for (int u = 0; u < B; ++u) {
            rep[u] = __builtin_amdgcn_ubfe(w[u], id[u], 1u) != 0;  // (bit id % 32)
            const uint64_t key = ((uint64_t)t.wt << 32) | (uint64_t)(kSent - id[u]);
            bool better = act[u] & !rep[u] & (key > best);
            if (ballot(better) != 0) {  // wave-uniform
              if (better) better = merge_valid(a, v, id[u], 0);
            }
            best = better ? key : best;
            anyadd |= act[u] & rep[u];
          }
        }
        if (ballot(anyadd) != 0) {  // wave-uniform
#pragma unroll
          for (int u = 0; u < B; ++u) {
            if (act[u] & rep[u]) {
              const uint32_t rank = (uint32_t)S.wpre[(id[u] >> 5) - lw] +
                                    (uint32_t)__popc(w[u] & ((1u << (id[u] & 31)) - 1u));
              atomicAdd(&S.sc[rank], t.wt);
            }
          }
        }
        // as in sweep 1: every batch's loads are complete here
        asm volatile("" ::"v"(pin[0]), "v"(pin[1]), "v"(pin[2]), "v"(pin[3]));
      };
      auto sweep2 = [&](auto allv) {
        Batch ta, tb2;
        uint32_t pa[B], pb[B];
        fetch(ta, pa, false);
        while (ta.lim > 0) {
          fetch(tb2, pb, false);
          process2(ta, pa, allv);
          fetch(ta, pa, false);
          process2(tb2, pb, allv);
        }
      };
      if (v.all_valid)  // block-uniform: one sweep-2 loop per case
        sweep2(std::true_type{});
      else
        sweep2(std::false_type{});
      __syncthreads();  // sweep 2 done: scores complete
      // The fold: every repeat visit of the wave's part names a repeated id
      // (an id visited k times has k - 1 of them); its score is at its rank.
      // Ids named twice are compared twice, to the same effect; n is no
      // candidate of its own.
      for (int o = lane; o < wcnt; o += kWave) {
        const uint32_t id = S.lst[wid * kSeg + o];
        const uint32_t word = (id >> 5) - lw;
        const uint32_t w = S.seen[word];
        const uint32_t rank =
            (uint32_t)S.wpre[word] + (uint32_t)__popc(w & ((1u << (id & 31)) - 1u));
        const uint64_t key = ((uint64_t)S.sc[rank] << 32) | (uint64_t)(kSent - id);
        if (id != n && key > best && (v.all_valid || merge_valid(a, v, id, 0))) best = key;
      }
      if (tid < deg) {
        const int32_t c = S.m_cnt[tid];
        S.m_base[tid] += (uint32_t)c;
        S.m_rem[tid] -= c;
      }
      prev_wcnt = wcnt;
      prev_lw = lw;
      prev_nword = n_in ? (int32_t)((n >> 5) - lw) : -1;
      lo = hi;
      if (nrep < kList / 4 && width < kWinMax) {
        width *= 2;
        if (width > kWinMax) width = kWinMax;
      }
    }
    best = block_max_u64<THREADS>(best, S.red);
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

// Slices of every hyperedge at the aligned id windows: splits[e (W + 1) + w]
// = the number of pins of e with id below w << kWinAlignBits (a thread per
// hyperedge, binary searches over its ascending pins).
__global__ void window_splits_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
                                     const uint32_t* __restrict__ pins, int32_t W,
                                     uint32_t* __restrict__ splits) {
  const int64_t E = d->E;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; e < E; e += stride) {
    const int64_t s0 = eoff[e];
    const uint32_t len = (uint32_t)(eoff[e + 1] - s0);
    uint32_t* out = splits + e * (int64_t)(W + 1);
    out[0] = 0;
    uint32_t lo = 0;
    for (int32_t w = 1; w < W; ++w) {
      const uint32_t bound = (uint32_t)w << kWinAlignBits;
      uint32_t hi = len;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((pins[s0 + mid] & kIdMask) < bound) lo = mid + 1;
        else hi = mid;
      }
      out[w] = lo;
    }
    out[W] = len;
  }
}

// Windows with exact slices (large neighbourhoods, at most kWinDeg incident
// hyperedges).  OV: the distinct-axon bound of Section 3 can bind for the
// vertex, so the overlap of n and m (the multiplicity of the hyperedges in
// which both carry the destination flag) enters the validity test: for a
// single it is the visiting hyperedge's multiplicity when both flags are set;
// for a repeated id it is summed in sweep 2 next to the score.  The id space
// is cut into aligned windows of 2^kWinAlignBits ids, and every hyperedge's
// pins at those boundaries are known from `splits`, so a window's slice of
// each incident hyperedge is exact and no pin is tested against the window.
// Per window, the slices are cut into chunks of 64 pins listed back to back
// (a chunk descriptor holds its first pin, its hyperedge and its pin count),
// so that a batch of B chunks is full whatever the slices' lengths; waves
// claim batches from an LDS counter a fetch ahead.
//   sweep 1 sets one bitmap bit per visit; a visit finding its bit set puts
//     the id on its wave's list of repeat visits;
//   the bitmap is rebuilt with just the repeated ids (n among them), and
//     each repeated id gets a dense rank from per-word prefix counts;
//   singles: an id visited once has the visiting hyperedge's weight as its
//     score, so the best single of a window is, over the hyperedges, the
//     first pin of the slice (pins ascend) that is not repeated (and, where
//     a merge of n may break a limit, is valid): one thread per hyperedge
//     walks its slice from the start;
//   sweep 2 visits the chunks again and adds each repeat's weight to the
//     score at its id's rank; the fold compares the repeated ids' scores.
// A window whose chunks, repeat visits or repeated ids exceed the LDS room
// is retried at half the width (slices cut again by binary search), and the
// width grows back once windows fit.
template <int THREADS, bool OV>
__global__ __launch_bounds__(THREADS) void score_window2_kernel(ScoreArgs a, int bucket,
                                                               int64_t maxV) {
  constexpr int NW = THREADS / kWave;
  constexpr int B = 4;  // chunks per batch
  constexpr uint32_t kWinIds = 1u << kWinAlignBits;
  constexpr int kWords = (int)(kWinIds / 32);
  constexpr int kList = 4096;
  constexpr int kSeg = kList / NW;
  constexpr int kScores = 4096;
  constexpr int kMaxChunks = OV ? 1024 : 1536;
  constexpr uint32_t kSent = 0x7FFFFFFFu;
  static_assert(kWords == 16 * THREADS, "a thread owns 16 consecutive bitmap words");
  static_assert(kWinDeg <= THREADS, "thread j owns hyperedge j");
  static_assert(kWinDeg <= 1024, "a chunk descriptor holds the hyperedge in 10 bits");
  struct Lds {
    alignas(16) uint32_t seen[kWords];
    alignas(16) uint16_t wpre[kWords];   // repeated ids in the words before each word
    uint32_t lst[kList + kWave];         // repeat visits, wave w's from w * kSeg on
    uint32_t sc[kScores];                // score of each rank
    uint32_t ovsc[OV ? kScores : 1];     // overlap of each rank (OV)
    uint2 desc[kMaxChunks + B];          // x: first pin; y: hyperedge | pin count << 10
    int32_t m_w[kWinDeg];
    int32_t m_mu[OV ? kWinDeg : 1];      // mult of hyperedge j if n has its flag, else 0
    int32_t s_wcnt[NW];
    int32_t ws[3 * NW];
    uint64_t red[2 * NW];
    int32_t s_item;
    int32_t s_next;
  };
  __shared__ Lds S;

  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wid = rfl_i32(tid / kWave);
  int32_t count = a.b.count[bucket];
  if (count > maxV) {
    if (tid == 0) atomicOr(a.err, kErrWorkCount);
    count = (int32_t)maxV;
  }
  const int32_t* list = a.b.list + (int64_t)bucket * maxV;
  const int32_t W = a.n_win;
  uint4* const seen4 = reinterpret_cast<uint4*>(S.seen);
  uint4* const wpre4 = reinterpret_cast<uint4*>(S.wpre);
#pragma unroll
  for (int i = 0; i < 4; ++i) seen4[4 * tid + i] = make_uint4(0u, 0u, 0u, 0u);
  int32_t prev_wcnt = 0, prev_nword = -1;
  uint32_t prev_lw = 0;
  uint32_t lofs[B];
#pragma unroll
  for (int u = 0; u < B; ++u) lofs[u] = (uint32_t)lane * 4u;

  while (true) {
    __syncthreads();
    if (tid == 0) S.s_item = atomicAdd(&a.work[bucket], 1);
    __syncthreads();
    const int32_t item = S.s_item;
    if (item >= count) break;

    VertexCtx v;
    v.n = list[item];
    v.beg = a.voff[v.n];
    v.deg = a.voff[v.n + 1] - v.beg;
    if (v.deg > kWinDeg) {  // block-uniform; the bucket rule excludes it
      if (tid == 0) atomicOr(a.err, kErrWorkCount);
      continue;
    }
    v.size_n = a.L.size[v.n];
    v.syn_n = a.L.syn[v.n];
    v.ax_n = a.L.ax[v.n];
    v.G = a.gc[a.L.gid ? a.L.gid[v.n] : 0];
    v.all_valid = (int64_t)v.size_n + v.G.max_size <= v.G.omega &&
                  (int64_t)v.syn_n + v.G.max_syn <= v.G.phi &&
                  (int64_t)v.ax_n + v.G.max_ax <= v.G.delta;
    const uint32_t n = (uint32_t)v.n;
    const int32_t deg = (int32_t)v.deg;
    uint64_t best = 0;
    // thread j owns incident hyperedge j: its pins' base, weight, and the
    // cursor of the unprocessed part of its slice
    const bool owner = tid < deg;
    uint32_t e_j = 0, cur = 0;
    int32_t w_j = 0, mu_j = 0;
    const uint32_t* srow = nullptr;
    if (owner) {
      const uint32_t ent = a.vinc[v.beg + tid];
      e_j = ent & kIdMask;
      cur = (uint32_t)a.L.eoff[e_j];
      w_j = a.L.w[e_j];
      S.m_w[tid] = w_j;
      if (OV) {
        mu_j = (ent & kDst) ? a.L.mult[e_j] : 0;
        S.m_mu[tid] = mu_j;
      }
      srow = a.splits + (int64_t)e_j * (W + 1);
    }
    int passes = 0;
    bool stop = false;  // a bound was reached: the vertex keeps no candidate
    for (int32_t wi = 0; wi < W && !stop; ++wi) {  // block-uniform
      const uint32_t W0 = (uint32_t)wi << kWinAlignBits;
      uint32_t W1 = W0 + kWinIds;
      // the slice's end at the aligned window's end
      uint32_t wend = 0;
      if (owner) wend = (uint32_t)a.L.eoff[e_j] + srow[wi + 1];
      uint32_t lo = W0;
      uint32_t width = kWinIds;
      while (lo < W1) {  // block-uniform
        const uint32_t hi = W1 - lo <= width ? W1 : lo + width;
        const uint32_t lw = lo >> 5;
        uint32_t* const seenw = S.seen - lw;
        const uint32_t lane_w = (uint32_t)lane + lw;
        __syncthreads();  // previous window folded, lists read, descriptors free
        if (++passes > kMaxPasses) {
          if (tid == 0) atomicOr(a.err, kErrPassLimit);
          stop = true;
          break;
        }
        // ---- exact slices and their chunk list
        uint32_t end = cur;
        if (owner) {
          if (hi == W1) {
            end = wend;
          } else {
            uint32_t l = cur, h = wend;
            while (l < h) {
              const uint32_t mid = (l + h) >> 1;
              if ((a.L.pins[mid] & kIdMask) < hi) l = mid + 1;
              else h = mid;
            }
            end = l;
          }
        }
        const int32_t nch = (int32_t)((end - cur + kWave - 1) / kWave);
        int32_t x3[3] = {nch, 0, 0}, p3[3], t3[3];
        block_scan3<THREADS>(x3, p3, t3, S.ws);
        const int32_t T = t3[0];
        if (T > kMaxChunks) {  // block-uniform
          width >>= 1;
          continue;
        }
        if (T == 0) {  // no pin of n's hyperedges in this range
          lo = hi;
          continue;
        }
        for (int32_t c = 0; c < nch; ++c) {
          const uint32_t first = cur + (uint32_t)c * kWave;
          const uint32_t left = end - first;
          S.desc[p3[0] + c] =
              make_uint2(first, (uint32_t)tid | ((left < (uint32_t)kWave ? left : kWave) << 10));
        }
        if (tid < B) S.desc[T + tid] = make_uint2(0u, 0u);
        if (tid == 0) S.s_next = NW;
        // the bitmap starts empty: the last window left only its repeated ids
        for (int o = lane; o < prev_wcnt; o += kWave)
          S.seen[(S.lst[wid * kSeg + o] >> 5) - prev_lw] = 0;
        if (tid == 0 && prev_nword >= 0) S.seen[prev_nword] = 0;
        prev_wcnt = 0;
        prev_nword = -1;
        __syncthreads();
        const int32_t tb = (T + B - 1) / B;  // batches

        // A batch's chunks: descriptors read at a wave-uniform address,
        // made scalar; lanes past a chunk's pins load its last pin.
        struct Batch {
          uint32_t x[B];
          int32_t cnt[B];
          int32_t j[B];
        };
        int32_t bclaim = wid;
        auto fetch = [&](Batch& t, uint32_t (&pin)[B], int32_t bno) {
#pragma unroll
          for (int u = 0; u < B; ++u) {
            uint2 d = make_uint2(0u, 0u);
            if (bno < tb) d = S.desc[bno * B + u];
            t.x[u] = rfl_u32(d.x);
            const uint32_t y = rfl_u32(d.y);
            t.cnt[u] = (int32_t)(y >> 10);
            t.j[u] = (int32_t)(y & 0x3FFu);
          }
#pragma unroll
          for (int u = 0; u < B; ++u) {
            const uint32_t last4 = t.cnt[u] > 0 ? (uint32_t)(t.cnt[u] - 1) * 4u : 0u;
            const char* p = reinterpret_cast<const char*>(a.L.pins + t.x[u]);
            const uint32_t off = lofs[u] < last4 ? lofs[u] : last4;
            pin[u] = *reinterpret_cast<const uint32_t*>(p + off);
          }
          if (bno < tb) {  // wave-uniform: claim the next batch
            int32_t c = 0;
            if (lane == 0) c = atomicAdd(&S.s_next, 1);
            bclaim = c;
          }
          __builtin_amdgcn_sched_barrier(0);
        };

        // ---- sweep 1
        bool over = false;
        int32_t wcnt = 0;
        auto process1 = [&](const Batch& t, const uint32_t (&pin)[B]) {
          uint32_t id[B], bit[B], old[B];
#pragma unroll
          for (int u = 0; u < B; ++u) {
            id[u] = pin[u] & kIdMask;
            const bool act = lofs[u] < (uint32_t)t.cnt[u] * 4u;
            const uint32_t word = act ? id[u] >> 5 : lane_w;
            bit[u] = act ? 1u << (id[u] & 31) : 0u;
            old[u] = atomicOr(&seenw[word], bit[u]);
          }
          bool rep[B];
          uint64_t rb[B];
          int32_t nr = 0;
#pragma unroll
          for (int u = 0; u < B; ++u) {
            rep[u] = (old[u] & bit[u]) != 0;
            rb[u] = ballot(rep[u]);
            nr += (int32_t)__popcll(rb[u]);
          }
          if (nr > 0 && !over) {  // wave-uniform
            if (wcnt + nr > kSeg) {
              over = true;
            } else {
              uint32_t at = (uint32_t)(wid * kSeg + wcnt);
              wcnt += nr;
#pragma unroll
              for (int u = 0; u < B; ++u) {
                uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(rb[u] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)rb[u], 0u));
                asm volatile("" : "+v"(below));
                S.lst[rep[u] ? at + below : (uint32_t)(kList + lane)] = id[u];
                at += (uint32_t)__popcll(rb[u]);
              }
            }
          }
          asm volatile("" ::"v"(pin[0]), "v"(pin[1]), "v"(pin[2]), "v"(pin[3]));
        };
        {
          Batch ta, tb2;
          uint32_t pa[B], pb[B];
          int32_t cur_b = wid;
          fetch(ta, pa, cur_b);
          while (cur_b < tb && !over) {
            const int32_t nb = __builtin_amdgcn_readlane(bclaim, 0);
            fetch(tb2, pb, nb);
            process1(ta, pa);
            cur_b = nb;
            if (cur_b >= tb || over) break;
            const int32_t nb2 = __builtin_amdgcn_readlane(bclaim, 0);
            fetch(ta, pa, nb2);
            process1(tb2, pb);
            cur_b = nb2;
          }
        }
        S.s_wcnt[wid] = over ? -1 : wcnt;
        __syncthreads();
        const int32_t wc = lane < NW ? S.s_wcnt[lane] : 0;
        bool any_over = ballot(wc < 0) != 0;
        const int32_t nrep =
            __builtin_amdgcn_readlane(wave_incl_scan(wc > 0 ? wc : 0), kWave - 1);
        any_over |= nrep >= kScores;
#pragma unroll
        for (int i = 0; i < 4; ++i) seen4[4 * tid + i] = make_uint4(0u, 0u, 0u, 0u);
        if (any_over) {  // block-uniform
          width = width / 2 > 0 ? width / 2 : 1;
          continue;
        }
        __syncthreads();  // bitmap cleared
        for (int o = lane; o < wcnt; o += kWave) {
          const uint32_t id = S.lst[wid * kSeg + o];
          atomicOr(&S.seen[(id >> 5) - lw], 1u << (id & 31));
        }
        const bool n_in = n >= lo && n < hi;  // block-uniform
        if (tid == 0 && n_in) atomicOr(&S.seen[(n >> 5) - lw], 1u << (n & 31));
        __syncthreads();  // repeated ids marked
        {
          uint4 q[4];
          int32_t x4[3] = {0, 0, 0}, p4[3], t4[3];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            q[i] = seen4[4 * tid + i];
            x4[0] += __popc(q[i].x) + __popc(q[i].y) + __popc(q[i].z) + __popc(q[i].w);
          }
          block_scan3<THREADS>(x4, p4, t4, S.ws);
          const int32_t nrank = t4[0];
          uint32_t run = (uint32_t)p4[0], pk[8];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t r0 = run;
            run += __popc(q[i].x);
            const uint32_t r1 = run;
            run += __popc(q[i].y);
            const uint32_t r2 = run;
            run += __popc(q[i].z);
            const uint32_t r3 = run;
            run += __popc(q[i].w);
            pk[2 * i] = r0 | (r1 << 16);
            pk[2 * i + 1] = r2 | (r3 << 16);
          }
          if (nrank > 0) {  // block-uniform
            wpre4[2 * tid] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
            wpre4[2 * tid + 1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
            for (int i = tid; i < nrank; i += THREADS) {
              S.sc[i] = 0;
              if (OV) S.ovsc[i] = 0;
            }
          }
        }
        if (tid == 0) S.s_next = NW;
        // ---- singles: the first pin of each slice that is not repeated (a
        // single shares one hyperedge with n: its overlap is that
        // hyperedge's multiplicity when both carry the flag)
        if (owner) {
          for (uint32_t pp = cur; pp < end; ++pp) {
            const uint32_t pin = a.L.pins[pp];
            const uint32_t id = pin & kIdMask;
            const bool rep = (seenw[id >> 5] >> (id & 31)) & 1u;
            const int64_t ov = (OV && (pin & kDst)) ? mu_j : 0;
            if (!rep && (v.all_valid || merge_valid(a, v, id, ov))) {
              const uint64_t key = ((uint64_t)(uint32_t)w_j << 32) | (uint64_t)(kSent - id);
              best = key > best ? key : best;
              break;
            }
          }
        }
        __syncthreads();  // ranks, scores and the claim counter ready

        // ---- sweep 2: weights of the repeat visits at their ranks
        auto process2 = [&](const Batch& t, const uint32_t (&pin)[B]) {
          uint32_t id[B], wv[B];
          (void)pin;
          bool rep[B];
          bool anyrep = false;
#pragma unroll
          for (int u = 0; u < B; ++u) {
            id[u] = pin[u] & kIdMask;
            const bool act = lofs[u] < (uint32_t)t.cnt[u] * 4u;
            wv[u] = seenw[id[u] >> 5];
            rep[u] = act & (__builtin_amdgcn_ubfe(wv[u], id[u], 1u) != 0);
            anyrep |= rep[u];
          }
          if (ballot(anyrep) != 0) {  // wave-uniform
#pragma unroll
            for (int u = 0; u < B; ++u) {
              if (rep[u]) {
                const uint32_t rank = (uint32_t)S.wpre[(id[u] >> 5) - lw] +
                                      (uint32_t)__popc(wv[u] & ((1u << (id[u] & 31)) - 1u));
                atomicAdd(&S.sc[rank], (uint32_t)S.m_w[t.j[u]]);
                if (OV) {
                  const int32_t mu = S.m_mu[t.j[u]];
                  if (mu && (pin[u] & kDst)) atomicAdd(&S.ovsc[rank], (uint32_t)mu);
                }
              }
            }
          }
          asm volatile("" ::"v"(pin[0]), "v"(pin[1]), "v"(pin[2]), "v"(pin[3]));
        };
        bclaim = wid;
        {
          Batch ta, tb2;
          uint32_t pa[B], pb[B];
          int32_t cur_b = wid;
          fetch(ta, pa, cur_b);
          while (cur_b < tb) {
            const int32_t nb = __builtin_amdgcn_readlane(bclaim, 0);
            fetch(tb2, pb, nb);
            process2(ta, pa);
            cur_b = nb;
            if (cur_b >= tb) break;
            const int32_t nb2 = __builtin_amdgcn_readlane(bclaim, 0);
            fetch(ta, pa, nb2);
            process2(tb2, pb);
            cur_b = nb2;
          }
        }
        __syncthreads();  // scores complete
        // ---- fold: the repeated ids of the wave's list
        for (int o = lane; o < wcnt; o += kWave) {
          const uint32_t id = S.lst[wid * kSeg + o];
          const uint32_t word = (id >> 5) - lw;
          const uint32_t w = S.seen[word];
          const uint32_t rank =
              (uint32_t)S.wpre[word] + (uint32_t)__popc(w & ((1u << (id & 31)) - 1u));
          const uint64_t key = ((uint64_t)S.sc[rank] << 32) | (uint64_t)(kSent - id);
          const int64_t ov = OV ? (int64_t)S.ovsc[rank] : 0;
          if (id != n && key > best && (v.all_valid || merge_valid(a, v, id, ov))) best = key;
        }
        cur = end;
        prev_wcnt = wcnt;
        prev_lw = lw;
        prev_nword = n_in ? (int32_t)((n >> 5) - lw) : -1;
        lo = hi;
        if (nrep < kList / 4 && width < kWinIds) width *= 2;
      }
    }
    if (stop) best = 0;
    best = block_max_u64<THREADS>(best, S.red);
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


}  // namespace

void score_candidates(const ScoreArgs& a, int64_t maxV, int64_t maxP, hipStream_t s) {
  no_candidate_kernel<<<grid_for(maxV, 256, 8192), 256, 0, s>>>(a.L.dims, a.cand, a.cscore,
                                                               a.work);
  // persistent grids, per device (the CU count and the occupancy of each
  // kernel are fixed for a device)
  constexpr int kMaxDevices = 64;
  static int grids[kMaxDevices][kNumBuckets] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
  int* g = grids[dev];
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
  const bool aligned = a.n_win > 0 && a.splits;
  static int g2[kMaxDevices][2] = {};
  auto k2w = score_window2_kernel<1024, false>;
  auto k6w = score_window2_kernel<1024, true>;
  if (aligned) {
    if (!g2[dev][0]) {
      g2[dev][0] = persistent_grid(k2w, 1024);
      g2[dev][1] = persistent_grid(k6w, 1024);
    }
    window_splits_kernel<<<4096, 256, 0, s>>>(a.L.dims, a.L.eoff, a.L.pins, a.n_win,
                                              a.splits);
    if (!(a.wide && score_wide(a, 2, false, maxV, s))) k2w<<<g2[dev][0], 1024, 0, s>>>(a, 2, maxV);
  } else {
    k2<<<g[2], 1024, 0, s>>>(a, 2, maxV);
  }
  k3<<<g[3], 512, 0, s>>>(a, 3, maxV, maxP);
  k4<<<g[4], 256, 0, s>>>(a, 4, maxV, maxP);
  k5<<<g[5], 512, 0, s>>>(a, 5, maxV, maxP);
  if (aligned) {
    if (!(a.wide && score_wide(a, 6, true, maxV, s))) k6w<<<g2[dev][1], 1024, 0, s>>>(a, 6, maxV);
  }
  else
    k6<<<g[6], 1024, 0, s>>>(a, 6, maxV);
  score_dense(a, maxV, s);
  k7<<<g[7], 512, 0, s>>>(a, 7, maxV, maxP);
}

}  // namespace hg
