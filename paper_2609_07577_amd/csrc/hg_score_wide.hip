// S2 for large neighbourhoods on levels with aligned id windows (Section 4.1,
// "Coarsening", Eq. 12): the window scheme of the aligned-window kernel with
// the long slices read 16 bytes per lane.
//
// A vertex's window visits are dominated by long slices (at the 2M-neuron
// level a visit lies, on average, in a slice of about a thousand pins), so a
// slice is cut into a body of 256-pin chunks starting at a 16-byte boundary
// (each lane loads four consecutive pins with one instruction) and a tail of
// 64-pin chunks (one pin per lane).  The first body chunk may start up to
// three pins before the slice; those lanes' pins are masked.  Per 256 pins
// the body pays one descriptor and one load instead of four of each, and a
// wave keeps four times the bytes in flight.
//
// Per window (ids [lo, hi) of an aligned window of 2^kWinAlignBits ids):
//   sweep 1 sets one bitmap bit per visit; a visit that finds its bit set
//     puts the id on its wave's list of repeat visits;
//   the bitmap is rebuilt with just the repeated ids (n among them), each
//     repeated id gets a dense rank from per-word prefix counts;
//   singles: an id visited once has the visiting hyperedge's weight as its
//     score, so the best single of a slice is its first pin that is not
//     repeated (pins ascend); that pin was loaded before sweep 1;
//   sweep 2 visits the chunks again and adds each repeated id's weight (and,
//     with OV, the overlap) at its rank; the fold takes the best repeated id.
// A window whose chunks, repeat visits or repeated ids exceed the LDS room is
// retried at half the width; the width grows back once windows fit.
#include "hg_internal.h"
#include "hg_score_common.h"

namespace hg {

namespace {

constexpr int kWideMaxPasses = 1 << 16;

template <int THREADS, bool OV>
__global__ __launch_bounds__(THREADS) void score_wide_kernel(ScoreArgs a, int bucket,
                                                            int64_t maxV) {
  constexpr int NW = THREADS / kWave;
  constexpr int BB = 2;      // body chunks per batch
  constexpr int BS = 4;      // tail chunks per batch
  constexpr int kBody = 256; // pins per body chunk (four per lane)
  constexpr uint32_t kWinIds = 1u << kWinAlignBits;
  constexpr int kWords = (int)(kWinIds / 32);
  constexpr int kList = 4096;
  constexpr int kSeg = kList / NW;
  constexpr int kScores = 4096;
  constexpr int kMaxBody = OV ? 384 : 448;
  constexpr int kMaxTail = OV ? 784 : 1088;
  constexpr uint32_t kSent = 0x7FFFFFFFu;
  constexpr uint32_t kDead = (uint32_t)kBody;  // skip value of a padding chunk
  static_assert(kWords == 16 * THREADS, "a thread owns 16 consecutive bitmap words");
  static_assert(kWinDeg <= THREADS, "thread j owns hyperedge j");
  static_assert(kWinDeg <= 1024, "a chunk descriptor holds the hyperedge in 10 bits");
  // a window of one id has at most one chunk per incident hyperedge: halving
  // always ends with a window that fits
  static_assert(kMaxTail >= kWinDeg, "tail list holds one chunk per hyperedge");
  struct Lds {
    alignas(16) uint32_t seen[kWords];
    alignas(16) uint16_t wpre[kWords];   // repeated ids in the words before each word
    uint32_t lst[kList + kWave];         // repeat visits, wave w's from w * kSeg on
    uint32_t sc[kScores];                // score of each rank
    uint32_t ovsc[OV ? kScores : 1];     // overlap of each rank (OV)
    uint2 bdesc[kMaxBody + BB];          // x: first pin (16-byte aligned); y: j | skip << 10
    uint2 tdesc[kMaxTail + BS];          // x: first pin; y: j | pin count << 10
    int32_t m_w[kWinDeg];
    int32_t m_mu[OV ? kWinDeg : 1];      // mult of hyperedge j if n has its flag, else 0
    int32_t s_wcnt[NW];
    int32_t ws[3 * NW];
    uint64_t red[2 * NW];
    int32_t s_item;
    int32_t s_nb;                        // next body batch to claim
    int32_t s_nt;                        // next tail batch to claim
  };
  static_assert(sizeof(Lds) <= 160 * 1024, "LDS of one work-group per CU");
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
  const uint32_t lofs = (uint32_t)lane * 4u;   // byte offset of a tail lane's pin; the
                                               // position of a body lane's first pin
  const uint32_t bofs = (uint32_t)lane * 16u;  // byte offset of a body lane's pins
  const char* const pin_bytes = reinterpret_cast<const char*>(a.L.pins);

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
    // thread j owns incident hyperedge j: its weight, the cursor of the
    // unprocessed part of its slice and the slice's end at the next aligned
    // window boundary (loaded one window ahead)
    // (the split value is kept as loaded and added only where it is used, a
    // window later: an add right after the load would wait for it there)
    const bool owner = tid < deg;
    uint32_t e_j = 0, cur = 0, base_j = 0, split_next = 0;
    int32_t w_j = 0, mu_j = 0;
    const uint32_t* srow = nullptr;
    if (owner) {
      const uint32_t ent = a.vinc[v.beg + tid];
      e_j = ent & kIdMask;
      base_j = (uint32_t)a.L.eoff[e_j];
      cur = base_j;
      w_j = a.L.w[e_j];
      S.m_w[tid] = w_j;
      if (OV) {
        mu_j = (ent & kDst) ? a.L.mult[e_j] : 0;
        S.m_mu[tid] = mu_j;
      }
      srow = a.splits + (int64_t)e_j * (W + 1);
      split_next = srow[1];
    }
    int passes = 0;
    bool stop = false;  // a bound was reached: the vertex keeps no candidate
    for (int32_t wi = 0; wi < W && !stop; ++wi) {  // block-uniform
      const uint32_t W0 = (uint32_t)wi << kWinAlignBits;
      const uint32_t W1 = W0 + kWinIds;
      const uint32_t wend = base_j + split_next;
      if (owner && wi + 1 < W) split_next = srow[wi + 2];
      // the slice's first pin, tested for a single after sweep 1
      uint32_t first_pin = 0;
      if (owner && cur < wend) first_pin = a.L.pins[cur];
      uint32_t lo = W0;
      uint32_t width = kWinIds;
      while (lo < W1) {  // block-uniform
        const uint32_t hi = W1 - lo <= width ? W1 : lo + width;
        const uint32_t lw = lo >> 5;
        uint32_t* const seenw = S.seen - lw;
        const uint32_t lane_w = (uint32_t)lane + lw;
        __syncthreads();  // previous window folded, lists read, descriptors free
        if (++passes > kWideMaxPasses) {
          if (tid == 0) atomicOr(a.err, kErrPassLimit);
          stop = true;
          break;
        }
        // ---- exact slices: a body of 256-pin chunks from the 16-byte
        // boundary at or below the slice start, and a tail of 64-pin chunks
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
        const uint32_t a0 = cur & ~3u;
        const int32_t nbody = end - a0 >= (uint32_t)kBody ? (int32_t)((end - a0) / kBody) : 0;
        const uint32_t tail0 = nbody ? a0 + (uint32_t)nbody * kBody : cur;
        const int32_t ntail = (int32_t)((end - tail0 + kWave - 1) / kWave);
        int32_t x3[3] = {nbody, ntail, 0}, p3[3], t3[3];
        block_scan3<THREADS>(x3, p3, t3, S.ws);
        const int32_t TB = t3[0], TT = t3[1];
        if (TB > kMaxBody || TT > kMaxTail) {  // block-uniform
          width >>= 1;
          continue;
        }
        if (TB + TT == 0) {  // no pin of n's hyperedges in this range
          lo = hi;
          continue;
        }
        for (int32_t c = 0; c < nbody; ++c)
          S.bdesc[p3[0] + c] = make_uint2(
              a0 + (uint32_t)c * kBody, (uint32_t)tid | ((c == 0 ? cur - a0 : 0u) << 10));
        if (nbody > 0 && p3[0] + nbody == TB) {  // padding: dead copies of the last chunk
#pragma unroll
          for (int u = 0; u < BB; ++u)
            S.bdesc[TB + u] = make_uint2(a0 + (uint32_t)(nbody - 1) * kBody,
                                         (uint32_t)tid | (kDead << 10));
        }
        for (int32_t c = 0; c < ntail; ++c) {
          const uint32_t first = tail0 + (uint32_t)c * kWave;
          const uint32_t left = end - first;
          S.tdesc[p3[1] + c] =
              make_uint2(first, (uint32_t)tid | ((left < (uint32_t)kWave ? left : kWave) << 10));
        }
        if (tid < BS) S.tdesc[TT + tid] = make_uint2(0u, 0u);
        if (tid == 0) {
          S.s_nb = NW;
          S.s_nt = NW;
        }
        // the bitmap starts empty: the last window left only its repeated ids
        for (int o = lane; o < prev_wcnt; o += kWave)
          S.seen[(S.lst[wid * kSeg + o] >> 5) - prev_lw] = 0;
        if (tid == 0 && prev_nword >= 0) S.seen[prev_nword] = 0;
        prev_wcnt = 0;
        prev_nword = -1;
        __syncthreads();
        const int32_t tbb = (TB + BB - 1) / BB;  // body batches
        const int32_t tbt = (TT + BS - 1) / BS;  // tail batches

        // Body batch: BB chunks, descriptors read at a wave-uniform address
        // and made scalar.  A batch past the list loads nothing.
        struct Body {
          uint32_t x[BB];
          uint32_t skip[BB];
          int32_t j[BB];
        };
        int32_t bclaim = wid;
        auto fetch_body = [&](Body& t, uint4 (&q)[BB], int32_t bno) {
          const bool live = bno < tbb;
#pragma unroll
          for (int u = 0; u < BB; ++u) {
            uint2 d = make_uint2(0u, 0u);
            if (live) d = S.bdesc[bno * BB + u];
            t.x[u] = rfl_u32(d.x);
            const uint32_t y = rfl_u32(d.y);
            t.skip[u] = y >> 10;
            t.j[u] = (int32_t)(y & 0x3FFu);
          }
          if (live) {
#pragma unroll
            for (int u = 0; u < BB; ++u)
              q[u] = *reinterpret_cast<const uint4*>(pin_bytes + (size_t)t.x[u] * 4u + bofs);
            int32_t c = 0;
            if (lane == 0) c = atomicAdd(&S.s_nb, 1);
            bclaim = c;
          }
          __builtin_amdgcn_sched_barrier(0);
        };
        // Tail batch: BS chunks; lanes past a chunk's pins load its last pin.
        struct Tail {
          uint32_t x[BS];
          int32_t cnt[BS];
          int32_t j[BS];
        };
        int32_t tclaim = wid;
        auto fetch_tail = [&](Tail& t, uint32_t (&pin)[BS], int32_t bno) {
#pragma unroll
          for (int u = 0; u < BS; ++u) {
            uint2 d = make_uint2(0u, 0u);
            if (bno < tbt) d = S.tdesc[bno * BS + u];
            t.x[u] = rfl_u32(d.x);
            const uint32_t y = rfl_u32(d.y);
            t.cnt[u] = (int32_t)(y >> 10);
            t.j[u] = (int32_t)(y & 0x3FFu);
          }
#pragma unroll
          for (int u = 0; u < BS; ++u) {
            const uint32_t last4 = t.cnt[u] > 0 ? (uint32_t)(t.cnt[u] - 1) * 4u : 0u;
            const uint32_t off = lofs < last4 ? lofs : last4;
            pin[u] = *reinterpret_cast<const uint32_t*>(pin_bytes + (size_t)t.x[u] * 4u + off);
          }
          if (bno < tbt) {
            int32_t c = 0;
            if (lane == 0) c = atomicAdd(&S.s_nt, 1);
            tclaim = c;
          }
          __builtin_amdgcn_sched_barrier(0);
        };

        // ---- sweep 1
        bool over = false;
        int32_t wcnt = 0;
        // appends the repeat visits of NP pin slots to the wave's list
        auto append = [&](const uint32_t* id, const bool* rep, int np) {
          uint64_t rb[4 * BB > BS ? 4 * BB : BS];
          int32_t nr = 0;
          for (int u = 0; u < np; ++u) {
            rb[u] = ballot(rep[u]);
            nr += (int32_t)__popcll(rb[u]);
          }
          if (nr > 0 && !over) {  // wave-uniform
            if (wcnt + nr > kSeg) {
              over = true;
            } else {
              uint32_t at = (uint32_t)(wid * kSeg + wcnt);
              wcnt += nr;
              for (int u = 0; u < np; ++u) {
                uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(rb[u] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)rb[u], 0u));
                asm volatile("" : "+v"(below));
                S.lst[rep[u] ? at + below : (uint32_t)(kList + lane)] = id[u];
                at += (uint32_t)__popcll(rb[u]);
              }
            }
          }
        };
        auto body1 = [&](const Body& t, const uint4 (&q)[BB]) {
          uint32_t id[4 * BB], bit[4 * BB], word[4 * BB];
          bool rep[4 * BB];
#pragma unroll
          for (int u = 0; u < BB; ++u) {
            const uint32_t p[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              id[4 * u + k] = p[k] & kIdMask;
              word[4 * u + k] = id[4 * u + k] >> 5;
              bit[4 * u + k] = 1u << (p[k] & 31u);
            }
          }
#pragma unroll
          for (int u = 0; u < BB; ++u) {
            if (t.skip[u]) {  // wave-uniform: pins before the slice, or a padding chunk
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                const bool act = lofs + (uint32_t)k >= t.skip[u];
                word[4 * u + k] = act ? word[4 * u + k] : lane_w;
                bit[4 * u + k] = act ? bit[4 * u + k] : 0u;
              }
            }
          }
#pragma unroll
          for (int s = 0; s < 4 * BB; ++s) {
            const uint32_t old = atomicOr(&seenw[word[s]], bit[s]);
            rep[s] = (old & bit[s]) != 0;
          }
          append(id, rep, 4 * BB);
        };
        auto tail1 = [&](const Tail& t, const uint32_t (&pin)[BS]) {
          uint32_t id[BS];
          bool rep[BS];
#pragma unroll
          for (int u = 0; u < BS; ++u) {
            id[u] = pin[u] & kIdMask;
            const bool act = lofs < (uint32_t)t.cnt[u] * 4u;
            const uint32_t word = act ? id[u] >> 5 : lane_w;
            const uint32_t bit = act ? 1u << (id[u] & 31) : 0u;
            const uint32_t old = atomicOr(&seenw[word], bit);
            rep[u] = (old & bit) != 0;
          }
          append(id, rep, BS);
          asm volatile("" ::"v"(pin[0]), "v"(pin[1]), "v"(pin[2]), "v"(pin[3]));
        };
        // the two lists, each with one batch in flight while the other is
        // processed
        auto sweep = [&](auto&& body_fn, auto&& tail_fn, bool check_over) {
          {
            Body ta, tb;
            uint4 qa[BB], qb[BB];
            int32_t cur_b = wid;
            fetch_body(ta, qa, cur_b);
            while (cur_b < tbb && !(check_over && over)) {
              const int32_t nb = __builtin_amdgcn_readlane(bclaim, 0);
              fetch_body(tb, qb, nb);
              body_fn(ta, qa);
              cur_b = nb;
              if (cur_b >= tbb || (check_over && over)) break;
              const int32_t nb2 = __builtin_amdgcn_readlane(bclaim, 0);
              fetch_body(ta, qa, nb2);
              body_fn(tb, qb);
              cur_b = nb2;
            }
          }
          {
            Tail ta, tb;
            uint32_t pa[BS], pb[BS];
            int32_t cur_b = wid;
            fetch_tail(ta, pa, cur_b);
            while (cur_b < tbt && !(check_over && over)) {
              const int32_t nb = __builtin_amdgcn_readlane(tclaim, 0);
              fetch_tail(tb, pb, nb);
              tail_fn(ta, pa);
              cur_b = nb;
              if (cur_b >= tbt || (check_over && over)) break;
              const int32_t nb2 = __builtin_amdgcn_readlane(tclaim, 0);
              fetch_tail(ta, pa, nb2);
              tail_fn(tb, pb);
              cur_b = nb2;
            }
          }
        };
        sweep(body1, tail1, true);
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
        if (tid == 0) {
          S.s_nb = NW;
          S.s_nt = NW;
        }
        // ---- singles: the first pin of each slice that is not repeated (a
        // single shares one hyperedge with n: its overlap is that
        // hyperedge's multiplicity when both carry the flag)
        if (owner && cur < end) {
          uint32_t pin = first_pin;
          for (uint32_t pp = cur;;) {
            const uint32_t id = pin & kIdMask;
            const bool rep = (seenw[id >> 5] >> (id & 31)) & 1u;
            const int64_t ov = (OV && (pin & kDst)) ? mu_j : 0;
            if (!rep && (v.all_valid || merge_valid(a, v, id, ov))) {
              const uint64_t key = ((uint64_t)(uint32_t)w_j << 32) | (uint64_t)(kSent - id);
              best = key > best ? key : best;
              break;
            }
            if (++pp >= end) break;
            pin = a.L.pins[pp];
          }
        }
        __syncthreads();  // ranks, scores and the claim counters ready

        // ---- sweep 2: weights of the repeat visits at their ranks
        auto add_rep = [&](uint32_t id, uint32_t wv, uint32_t pin, int32_t j) {
          const uint32_t rank = (uint32_t)S.wpre[(id >> 5) - lw] +
                                (uint32_t)__popc(wv & ((1u << (id & 31)) - 1u));
          atomicAdd(&S.sc[rank], (uint32_t)S.m_w[j]);
          if (OV) {
            const int32_t mu = S.m_mu[j];
            if (mu && (pin & kDst)) atomicAdd(&S.ovsc[rank], (uint32_t)mu);
          }
        };
        auto body2 = [&](const Body& t, const uint4 (&q)[BB]) {
          uint32_t id[4 * BB], wv[4 * BB], pn[4 * BB];
          bool rep[4 * BB];
          bool anyrep = false;
#pragma unroll
          for (int u = 0; u < BB; ++u) {
            const uint32_t p[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              pn[4 * u + k] = p[k];
              id[4 * u + k] = p[k] & kIdMask;
            }
          }
#pragma unroll
          for (int u = 0; u < BB; ++u) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int s = 4 * u + k;
              uint32_t word = id[s] >> 5;
              if (t.skip[u]) word = lofs + (uint32_t)k >= t.skip[u] ? word : lane_w;
              wv[s] = seenw[word];
              rep[s] = __builtin_amdgcn_ubfe(wv[s], id[s], 1u) != 0;
              if (t.skip[u]) rep[s] = rep[s] && lofs + (uint32_t)k >= t.skip[u];
              anyrep |= rep[s];
            }
          }
          if (ballot(anyrep) != 0) {  // wave-uniform
#pragma unroll
            for (int u = 0; u < BB; ++u)
#pragma unroll
              for (int k = 0; k < 4; ++k)
                if (rep[4 * u + k]) add_rep(id[4 * u + k], wv[4 * u + k], pn[4 * u + k], t.j[u]);
          }
        };
        auto tail2 = [&](const Tail& t, const uint32_t (&pin)[BS]) {
          uint32_t id[BS], wv[BS];
          bool rep[BS];
          bool anyrep = false;
#pragma unroll
          for (int u = 0; u < BS; ++u) {
            id[u] = pin[u] & kIdMask;
            const bool act = lofs < (uint32_t)t.cnt[u] * 4u;
            wv[u] = seenw[id[u] >> 5];
            rep[u] = act & (__builtin_amdgcn_ubfe(wv[u], id[u], 1u) != 0);
            anyrep |= rep[u];
          }
          if (ballot(anyrep) != 0) {  // wave-uniform
#pragma unroll
            for (int u = 0; u < BS; ++u)
              if (rep[u]) add_rep(id[u], wv[u], pin[u], t.j[u]);
          }
          asm volatile("" ::"v"(pin[0]), "v"(pin[1]), "v"(pin[2]), "v"(pin[3]));
        };
        bclaim = wid;
        tclaim = wid;
        sweep(body2, tail2, false);
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
        if (owner && hi < W1 && cur < wend) first_pin = a.L.pins[cur];
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

}  // namespace

bool score_wide(const ScoreArgs& a, int bucket, bool ov, int64_t maxV, hipStream_t s) {
  // the body loads need 16-byte aligned pins
  if ((reinterpret_cast<uintptr_t>(a.L.pins) & 15u) != 0 || a.n_win <= 0 || !a.splits)
    return false;
  constexpr int kMaxDevices = 64;
  static int grids[kMaxDevices][2] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
  auto k0 = score_wide_kernel<1024, false>;
  auto k1 = score_wide_kernel<1024, true>;
  if (!grids[dev][0]) {
    grids[dev][0] = persistent_grid(k0, 1024);
    grids[dev][1] = persistent_grid(k1, 1024);
  }
  if (ov)
    k1<<<grids[dev][1], 1024, 0, s>>>(a, bucket, maxV);
  else
    k0<<<grids[dev][0], 1024, 0, s>>>(a, bucket, maxV);
  return true;
}

}  // namespace hg
