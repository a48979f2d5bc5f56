// S2 for dense neighbourhoods (paper, Section 4.1, "Coarsening", Eq. 12):
// vertices whose neighbour visits reach a large share of the level's ids
// (work lists 8 and 9 of the bucket rule), scored in windows of 2^14 ids
// with one packed LDS entry per id.
#include <type_traits>

#include "hg_internal.h"
#include "hg_score_common.h"

namespace hg {

namespace {

// Slices of every hyperedge at the dense windows of 2^kDenseBits ids: a wave
// per hyperedge walks its ascending pins 64 at a time; where the window of
// consecutive pins changes, the windows passed over get the pin's position.
__global__ void dense_splits_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
                                    const uint32_t* __restrict__ pins, int32_t W,
                                    uint32_t* __restrict__ splits) {
  const int64_t E = d->E;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t e = wave; e < E; e += nw) {
    const int64_t s0 = eoff[e];
    const int32_t len = (int32_t)(eoff[e + 1] - s0);
    uint32_t* out = splits + e * (int64_t)(W + 1);
    int32_t prev_w = -1;  // window of the pin before the chunk (-1: before the first)
    for (int32_t c = 0; c < len; c += kWave) {  // wave-uniform
      const int32_t i = c + lane;
      const int32_t w = i < len ? (int32_t)((pins[s0 + i] & kIdMask) >> kDenseBits) : W;
      int32_t before = __shfl_up(w, 1, kWave);
      if (lane == 0) before = prev_w;
      // windows (before, w] start at pin i (pins of window w begin here)
      if (i < len)
        for (int32_t x = before + 1; x <= w && x <= W; ++x) out[x] = (uint32_t)i;
      prev_w = __shfl(w, kWave - 1, kWave);
      if (prev_w >= W) break;
    }
    // windows after the last pin's window end at the hyperedge's end
    const int32_t last = len > 0 ? (int32_t)((pins[s0 + len - 1] & kIdMask) >> kDenseBits) : -1;
    for (int32_t x = last + 1 + lane; x <= W; x += kWave) out[x] = (uint32_t)len;
  }
}

// Dense windows (neighbourhoods that visit at least one id in dense_ratio
// of the level): per window of ids, one packed LDS entry per id, and one
// sweep over the window's slices adds each visit's (weight, overlap share)
// to its id's entry with a non-returning LDS atomic (nothing in the sweep
// waits for the LDS).  Then every thread reads the final (score, overlap)
// of its own entries, takes the best valid (score, -id) among them (n left
// out) and zeroes them for the next window: each id is tested for validity
// at most once, with its exact totals, and only when its key beats the
// thread's best and the vertex's threshold (a key some thread found valid).
// OV: the overlap share of a visit is the hyperedge's multiplicity when n
// and the visited id both carry its flag.
//
// Entry width per vertex: a score is at most S_n (the weight of n's
// incident hyperedges) and an overlap at most M_n (their multiplicity where
// n carries the flag).  When both fit in 32 bits together (always without
// OV), entries are 32-bit, score << b | overlap with b the bits of M_n, and a
// window spans 2^(kDenseBits + 1) ids (two windows of the split table);
// otherwise entries are 64-bit, score << 32 | overlap, over 2^kDenseBits
// ids.  The window's slices (from `splits14`) are cut into chunks of up to
// 64 pins listed in LDS and claimed by the waves in batches of B; a window
// of more than kMaxChunks chunks is swept in rounds.
template <int THREADS, bool OV>
__global__ __launch_bounds__(THREADS) void score_dense_kernel(ScoreArgs a, int bucket,
                                                             int64_t maxV) {
  constexpr int NW = THREADS / kWave;
  constexpr int B = 4;
  constexpr int kIds = 1 << kDenseBits;
  constexpr int kMaxChunks = 1024;
  constexpr uint32_t kSent = 0x7FFFFFFFu;
  static_assert(kIds * 8 == THREADS * 128, "a thread clears 128 bytes of the table");
  struct Lds {
    uint64_t tab[kIds];          // 2^14 64-bit entries or 2^15 32-bit ones
    uint4 desc[kMaxChunks + B];  // x first pin, y pin count, z weight, w overlap share
    int32_t ws[3 * NW];
    uint64_t red[2 * NW];
    uint64_t thr;                // largest key found valid so far for the vertex
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
  // splits14 rows hold n_win14 + 1 entries (the windows of the largest
  // level); the windows past this level's ids are empty and skipped
  const int32_t W = a.n_win14;
  const int64_t Vl = a.L.dims->V;
  const int32_t Wl = (int32_t)((Vl + kIds - 1) >> kDenseBits) < W
                         ? (int32_t)((Vl + kIds - 1) >> kDenseBits) : W;
  uint4* const tab4 = reinterpret_cast<uint4*>(S.tab);
  uint32_t* const tab32 = reinterpret_cast<uint32_t*>(S.tab);
  const uint32_t lofs = (uint32_t)lane * 4u;
  // the table starts zeroed; every window's scan zeroes the entries it read
#pragma unroll
  for (int i = 0; i < 8; ++i) tab4[8 * tid + i] = make_uint4(0u, 0u, 0u, 0u);

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
    v.size_n = a.L.size[v.n];
    v.syn_n = a.L.syn[v.n];
    v.ax_n = a.L.ax[v.n];
    v.G = a.gc[a.L.gid ? a.L.gid[v.n] : 0];
    v.all_valid = (int64_t)v.size_n + v.G.max_size <= v.G.omega &&
                  (int64_t)v.syn_n + v.G.max_syn <= v.G.phi &&
                  (int64_t)v.ax_n + v.G.max_ax <= v.G.delta;
    const uint32_t n = (uint32_t)v.n;
    const int64_t deg = v.deg;
    uint64_t best = 0;
    if (tid == 0) S.thr = 0;  // read after the barriers below
    // the id range of n's neighbourhood (first and last pins of its incident
    // hyperedges; pins ascend): windows outside it hold no visit (a graph of
    // a batch occupies one id range of the union)
    uint32_t idmin = 0xFFFFFFFFu, idmax = 0;
    for (int64_t j = tid; j < deg; j += THREADS) {
      const uint32_t e = a.vinc[v.beg + j] & kIdMask;
      const int64_t e0 = a.L.eoff[e], e1 = a.L.eoff[e + 1];
      const uint32_t f = a.L.pins[e0] & kIdMask, l = a.L.pins[e1 - 1] & kIdMask;
      idmin = f < idmin ? f : idmin;
      idmax = l > idmax ? l : idmax;
    }
    idmax = (uint32_t)block_max_u64<THREADS>(idmax, S.red);
    idmin = ~(uint32_t)block_max_u64<THREADS>((uint64_t)(~idmin), S.red);
    // bounds of a score (S_n) and of an overlap (M_n), for the entry width
    int32_t ob = 0;  // overlap bits of a compact entry
    bool compact = true;
    if (OV) {
      // both sums stay below 2^31: the weights of a level sum below 2^31 and
      // the multiplicities below the number of original axons
      int32_t sw = 0, sm = 0;
      for (int64_t j = tid; j < deg; j += THREADS) {
        const uint32_t ent = a.vinc[v.beg + j];
        const uint32_t e = ent & kIdMask;
        sw += a.L.w[e];
        if (ent & kDst) sm += a.L.mult[e];
      }
      int32_t x3[3] = {sw, sm, 0}, p3[3], t3[3];
      block_scan3<THREADS>(x3, p3, t3, S.ws);
      const uint32_t S_n = (uint32_t)t3[0], M_n = (uint32_t)t3[1];
      const int sb = S_n ? 32 - __clz(S_n) : 0;
      ob = M_n ? 32 - __clz(M_n) : 0;
      compact = sb + ob <= 32;
      __syncthreads();  // the scan words are read before the windows' scans
    }
    auto windows = [&](auto compact_tag) {
      constexpr bool C = decltype(compact_tag)::value;
      constexpr int kBits = C ? kDenseBits + 1 : kDenseBits;
      const int32_t nw = C ? (Wl + 1) / 2 : Wl;
      const int32_t w_lo = deg > 0 ? (int32_t)(idmin >> kBits) : 0;
      const int32_t w_hi = deg > 0 ? (int32_t)(idmax >> kBits) + 1 : 0;  // exclusive
      const uint32_t omask = C ? ((1u << ob) - 1u) : 0xFFFFFFFFu;
      // split-table bounds of window wi (two 2^14 windows when compact)
      auto bounds = [&](const uint32_t* sr, int32_t wi, uint32_t& b0, uint32_t& b1) {
        if (C) {
          b0 = sr[2 * wi];
          b1 = sr[2 * wi + 2 <= W ? 2 * wi + 2 : W];
        } else {
          b0 = sr[wi];
          b1 = sr[wi + 1];
        }
      };
      // with at most THREADS incident hyperedges (one segment) thread t keeps
      // hyperedge t's window-independent values in registers for all windows
      // and loads the next window's slice bounds while this one is swept
      const bool one_seg = deg <= THREADS;  // block-uniform
      const int32_t w_end = nw < w_hi ? nw : w_hi;
      uint32_t h_e0 = 0, h_wt = 0, h_mu = 0, nb0 = 0, nb1 = 0;
      const uint32_t* h_row = a.splits14;
      if (one_seg && tid < deg) {
        const uint32_t ent = a.vinc[v.beg + tid];
        const uint32_t e = ent & kIdMask;
        h_row = a.splits14 + (int64_t)e * (W + 1);
        if (w_lo < w_end) bounds(h_row, w_lo, nb0, nb1);
        h_e0 = (uint32_t)a.L.eoff[e];
        h_wt = (uint32_t)a.L.w[e];
        h_mu = (OV && (ent & kDst)) ? (uint32_t)a.L.mult[e] : 0u;
      }
      for (int32_t wi = w_lo; wi < w_end; ++wi) {  // block-uniform
        const uint32_t lo = (uint32_t)wi << kBits;
        bool cleared = false;  // block-uniform: the table is cleared before the first sweep
        // segments of THREADS incident hyperedges; thread t holds hyperedge
        // seg + t of the segment (its slice of the window) in registers
        for (int64_t seg = 0; seg < deg; seg += THREADS) {  // block-uniform
          const int64_t j = seg + tid;
          uint32_t first = 0, len = 0, wt = 0, mu = 0;
          if (one_seg) {
            if (j < deg) {
              len = nb1 - nb0;
              first = h_e0 + nb0;
              wt = h_wt;
              mu = h_mu;
              if (wi + 1 < w_end) bounds(h_row, wi + 1, nb0, nb1);
            }
          } else if (j < deg) {
            const uint32_t ent = a.vinc[v.beg + j];
            const uint32_t e = ent & kIdMask;
            uint32_t b0, b1;
            bounds(a.splits14 + (int64_t)e * (W + 1), wi, b0, b1);
            len = b1 - b0;
            if (len) {
              first = (uint32_t)a.L.eoff[e] + b0;
              wt = (uint32_t)a.L.w[e];
              mu = (OV && (ent & kDst)) ? (uint32_t)a.L.mult[e] : 0u;
            }
          }
          const int32_t nch = (int32_t)((len + kWave - 1) / kWave);
          int32_t x3[3] = {nch, 0, 0}, p3[3], t3[3];
          block_scan3<THREADS>(x3, p3, t3, S.ws);
          const int32_t T = t3[0];
          if (T == 0) {  // block-uniform; the scan's words are read before the next scan
            __syncthreads();
            continue;
          }
          cleared = true;
          for (int32_t r0 = 0; r0 < T; r0 += kMaxChunks) {  // block-uniform
            const int32_t Tr = T - r0 < kMaxChunks ? T - r0 : kMaxChunks;
            __syncthreads();  // table clear, previous round's chunks done
            const int32_t c = p3[0];  // this thread's first chunk in the segment's list
            if (c + nch > r0 && c < r0 + Tr) {
              for (int32_t q = 0; q < nch; ++q) {
                const int32_t at = c + q - r0;
                if (at < 0 || at >= Tr) continue;
                const uint32_t left = len - (uint32_t)q * kWave;
                S.desc[at] = make_uint4(first + (uint32_t)q * kWave,
                                        left < (uint32_t)kWave ? left : (uint32_t)kWave, wt, mu);
              }
            }
            if (tid < B) S.desc[Tr + tid] = make_uint4(0u, 0u, 0u, 0u);
            if (tid == 0) S.s_next = NW;
            __syncthreads();
            const int32_t tb = (Tr + B - 1) / B;
            // ---- the sweep
            struct Batch {
              uint32_t x[B];
              int32_t cnt[B];
              uint32_t wt[B], mu[B];
            };
            int32_t bclaim = wid;
            auto fetch = [&](Batch& t, uint32_t (&pin)[B], int32_t bno) {
#pragma unroll
              for (int u = 0; u < B; ++u) {
                uint4 d = make_uint4(0u, 0u, 0u, 0u);
                if (bno < tb) d = S.desc[bno * B + u];
                t.x[u] = rfl_u32(d.x);
                t.cnt[u] = (int32_t)rfl_u32(d.y);
                t.wt[u] = rfl_u32(d.z);
                t.mu[u] = rfl_u32(d.w);
              }
#pragma unroll
              for (int u = 0; u < B; ++u) {
                const uint32_t last4 = t.cnt[u] > 0 ? (uint32_t)(t.cnt[u] - 1) * 4u : 0u;
                const char* p = reinterpret_cast<const char*>(a.L.pins + t.x[u]);
                const uint32_t off = lofs < last4 ? lofs : last4;
                pin[u] = *reinterpret_cast<const uint32_t*>(p + off);
              }
              if (bno < tb) {  // wave-uniform: claim the next batch
                int32_t cc = 0;
                if (lane == 0) cc = atomicAdd(&S.s_next, 1);
                bclaim = cc;
              }
              __builtin_amdgcn_sched_barrier(0);
            };
            auto process = [&](const Batch& t, const uint32_t (&pin)[B]) {
#pragma unroll
              for (int u = 0; u < B; ++u) {
                const uint32_t id = pin[u] & kIdMask;
                const bool act = lofs < (uint32_t)t.cnt[u] * 4u;
                if (act) {  // no cross-lane operation inside
                  const uint32_t share = (OV && (pin[u] & kDst)) ? t.mu[u] : 0u;
                  if (C) {
                    atomicAdd(&tab32[id - lo], (t.wt[u] << ob) | share);
                  } else {
                    atomicAdd((unsigned long long*)&S.tab[id - lo],
                              (unsigned long long)(((uint64_t)t.wt[u] << 32) | (uint64_t)share));
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
              while (cur_b < tb) {
                const int32_t nb = __builtin_amdgcn_readlane(bclaim, 0);
                fetch(tb2, pb, nb);
                process(ta, pa);
                cur_b = nb;
                if (cur_b >= tb) break;
                const int32_t nb2 = __builtin_amdgcn_readlane(bclaim, 0);
                fetch(ta, pa, nb2);
                process(tb2, pb);
                cur_b = nb2;
              }
            }
          }
        }  // segments
        if (cleared) {  // block-uniform
          __syncthreads();  // the window's sweeps done
          // this thread's entries: their best valid key, then zeroed
          const uint64_t thr = S.thr;
          uint64_t lim = best > thr ? best : thr;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const uint4 q = tab4[8 * tid + i];
            tab4[8 * tid + i] = make_uint4(0u, 0u, 0u, 0u);
            const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < (C ? 4 : 2); ++k) {
              uint64_t sc;
              uint32_t ov, id;
              if (C) {
                sc = w4[k] >> ob;
                ov = w4[k] & omask;
                id = lo + (uint32_t)(32 * tid + 4 * i + k);
              } else {
                sc = w4[2 * k + 1];
                ov = w4[2 * k];
                id = lo + (uint32_t)(16 * tid + 2 * i + k);
              }
              const uint64_t key = (sc << 32) | (uint64_t)(kSent - id);
              if (sc > 0 && id != n && key > lim &&
                  (v.all_valid || merge_valid(a, v, id, OV ? (int64_t)ov : 0))) {
                best = key;
                lim = key;
              }
            }
          }
          uint64_t m = best;
#pragma unroll
          for (int d = kWave / 2; d > 0; d >>= 1) {
            const uint64_t o = __shfl_xor(m, d, kWave);
            m = o > m ? o : m;
          }
          if (lane == 0 && m > thr) atomicMax((unsigned long long*)&S.thr, (unsigned long long)m);
        }
      }
    };
    if (compact) windows(std::integral_constant<bool, true>{});
    else windows(std::integral_constant<bool, false>{});
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

void score_dense(const ScoreArgs& a, int64_t maxV, hipStream_t s) {
  if (a.n_win14 <= 0 || !a.splits14) return;
  constexpr int kMaxDevices = 64;
  static int grids[kMaxDevices][2] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
  auto k8 = score_dense_kernel<1024, false>;
  auto k9 = score_dense_kernel<1024, true>;
  if (!grids[dev][0]) {
    grids[dev][0] = persistent_grid(k8, 1024);
    grids[dev][1] = persistent_grid(k9, 1024);
  }
  dense_splits_kernel<<<4096, 256, 0, s>>>(a.L.dims, a.L.eoff, a.L.pins, a.n_win14, a.splits14);
  k8<<<grids[dev][0], 1024, 0, s>>>(a, 8, maxV);
  k9<<<grids[dev][1], 1024, 0, s>>>(a, 9, maxV);
}

}  // namespace hg
