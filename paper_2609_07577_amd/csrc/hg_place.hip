// Placement of the partitioned hypergraph G_P on the core lattice (paper,
// Section 4.2): initial placement by recursive bisection with label
// propagation and folding, laid along the Hilbert curve; swap refinement by
// forces (Eq. 14) and tensions (Eq. 15), matched over cores by the rule of
// Eq. 13, ordered by tension, with the best prefix of recomputed tensions
// applied; the residual distance (the objective the swaps descend).  Every
// call runs `n_starts` placements at once (the multi-start of Section 4.2);
// per-start arrays are start-major.
//
// Lattice: width x height cores, core c = (x, y) = (c / height, c % height),
// Manhattan distance; nodes are the parts (at most 4096, one per core).
//
// Work shapes.  Passes over hyperedges give a wave to a hyperedge and a
// block to one start and a share of the hyperedges; per-node sums are kept
// in LDS for the block's start and added to global memory once per block.
// The per-start steps on at most 4096 cores or nodes (sorts, matching,
// prefix sums) run in one block per start.
//
// Forces without pairs.  For a node p at h = (x, y) and a hyperedge a of n
// pins holding it, the inner sum of Eq. 14 towards the core k one step
// along +x is  #(pins with x' > x) - #(pins with x' <= x, p excluded)  minus
// one when the node at k is a pin of a: the distances change by one for
// every pin and max(., 1) differs from the distance only at k itself.  So
// a histogram of the hyperedge's x and y coordinates gives every pin's four
// forces, in O(n + width + height) per hyperedge.
//
// Recomputed tensions without replay.  Swaps of a round are disjoint and
// each moves nodes by one step; the tension of swap i (cores a < b, nodes p
// at a, q at b) changes with an earlier swap j only through co-members
// that j moves across the line between a and b, which happens exactly when
// j swaps across the same line (same pair of columns, or of rows).  Each
// such co-member r adds 2 eta(e) for every hyperedge e shared with p or q,
// signed +1 when r and the node it pairs with (p or q) moved the same way.
// A pass over hyperedges accumulates these corrections per swap.
#include "hg_host.h"

namespace hg {

namespace {

constexpr int kMaxNodes = 4096;  // nodes (parts) and cores per start
constexpr int kMaxSide = 64;     // lattice width and height
constexpr int kTreeIds = 2 * kMaxNodes;
constexpr int kPT = 1024;        // threads of the per-start kernels
constexpr int kHT = 1024;        // threads of the hyperedge passes
constexpr int kHW = kHT / kWave;

__device__ inline int32_t wave_scan_incl(int32_t x) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ inline int64_t wave_scan_incl64(int64_t x) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ inline int64_t wave_sum64(int64_t x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

__device__ inline int depth_of(uint32_t heap_id) { return 31 - __clz(heap_id); }

// Blocks of a hyperedge pass: `per_start` blocks for each start.
struct HPass {
  int32_t starts, per_start;
  __device__ int32_t start() const { return blockIdx.x / per_start; }
  __device__ int32_t part() const { return blockIdx.x % per_start; }
};

// ---- Hilbert order and the bisection tree ----------------------------------

// Position d on the Hilbert curve of an n x n square (n a power of two) to
// (x, y): quadrant by quadrant from the finest, each quadrant reflected and
// transposed as the curve's recursive definition orders it.
__device__ inline void hilbert_point(int32_t n, int32_t d, int32_t& x, int32_t& y) {
  x = 0;
  y = 0;
  for (int32_t s = 1; s < n; s <<= 1) {
    const int32_t rx = (d >> 1) & 1;
    const int32_t ry = (d ^ rx) & 1;
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - x;
        y = s - 1 - y;
      }
      const int32_t t = x;
      x = y;
      y = t;
    }
    x += s * rx;
    y += s * ry;
    d >>= 2;
  }
}

// The lattice's cores in the order of the Hilbert curve of the smallest
// power-of-two square holding it (cores outside the lattice skipped).
__global__ __launch_bounds__(kPT) void hilbert_kernel(int32_t width, int32_t height,
                                                      int32_t* __restrict__ hc) {
  __shared__ int32_t ws[kPT / kWave];
  __shared__ int32_t base;
  int32_t n = 1;
  while (n < width || n < height) n <<= 1;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int32_t d0 = 0; d0 < n * n; d0 += kPT) {  // block-uniform
    const int32_t d = d0 + threadIdx.x;
    int32_t x = 0, y = 0;
    bool in = false;
    if (d < n * n) {
      hilbert_point(n, d, x, y);
      in = x < width && y < height;
    }
    const int32_t inc = wave_scan_incl(in ? 1 : 0);
    if (lane == kWave - 1) ws[wid] = inc;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int w = 0; w < kPT / kWave; ++w) {
      if (w < wid) before += ws[w];
      total += ws[w];
    }
    if (in) hc[base + before + inc - 1] = x * height + y;
    __syncthreads();
    if (threadIdx.x == 0) base += total;
    __syncthreads();
  }
}

// The bisection tree of V positions in heap numbering (root 1 = [0, V);
// node i of length len >= 2 has children 2i = its first ceil(len/2)
// positions and 2i + 1 the rest); tlen = 0 for ids that are no section.
// leaf_of[x] is the heap id of the one-position section of x.
__global__ __launch_bounds__(kPT) void tree_kernel(int32_t V, int32_t n_ids,
                                                   int32_t* __restrict__ tstart,
                                                   int32_t* __restrict__ tlen,
                                                   int32_t* __restrict__ leaf_of) {
  for (int32_t i = threadIdx.x; i < n_ids; i += kPT) {
    tstart[i] = 0;
    tlen[i] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    tstart[1] = 0;
    tlen[1] = V;
  }
  __syncthreads();
  for (int32_t lo = 1; lo < n_ids; lo <<= 1) {  // depth by depth
    for (int32_t i = lo + threadIdx.x; i < 2 * lo && i < n_ids; i += kPT) {
      const int32_t len = tlen[i], st = tstart[i];
      if (len == 1) leaf_of[st] = i;
      if (len >= 2 && 2 * i + 1 < n_ids) {
        const int32_t nl = len - len / 2;
        tstart[2 * i] = st;
        tlen[2 * i] = nl;
        tstart[2 * i + 1] = st + nl;
        tlen[2 * i + 1] = len - nl;
      }
    }
    __syncthreads();
  }
}

// The starting orders: seq[s][i] = orders[s][i], pos the inverse; an order
// that is not a permutation of [0, V) sets kErrPlacement.
__global__ void orders_kernel(int32_t S, int32_t V, const int32_t* __restrict__ orders,
                              int32_t* __restrict__ seq, int32_t* __restrict__ pos,
                              int32_t* __restrict__ seen, int32_t* __restrict__ err) {
  const int64_t n = (int64_t)S * V;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / V;
    const int32_t u = orders[i];
    if (u < 0 || u >= V) {
      atomicOr(err, kErrPlacement);
      seq[i] = 0;
      continue;
    }
    seq[i] = u;
    if (atomicAdd(&seen[s * V + u], 1) == 0) pos[s * V + u] = (int32_t)(i - s * V);
    else atomicOr(err, kErrPlacement);
  }
}

// ---- per-wave position bitmaps ----------------------------------------------

// A hyperedge's pins marked by position (V <= 4096 positions: 64 words and
// a zero word), with per-word prefix counts, so that any range of positions
// counts its pins in O(1).
struct PosBits {
  unsigned long long* bm;  // [65]
  int32_t* wp;             // [65] pins in the words before
  __device__ int32_t rank(int32_t x) const {  // pins at positions < x
    const int32_t w = x >> 6, b = x & 63;
    return wp[w] + (b ? __popcll(bm[w] & ((1ull << b) - 1ull)) : 0);
  }
  __device__ int32_t count(int32_t lo, int32_t hi) const { return rank(hi) - rank(lo); }
};

// Marks the pins of hyperedge [beg, end) by the positions pos[] of their
// nodes, then the prefix counts.  Wave-cooperative; the words start zero.
__device__ inline void mark_positions(const uint32_t* __restrict__ pins, int64_t beg, int64_t end,
                                      int32_t V, const int32_t* __restrict__ pos, PosBits& B) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t k = beg + lane; k < end; k += kWave) {
    const uint32_t u = pins[k] & kIdMask;
    if (u >= (uint32_t)V) continue;  // not a node: ignored (hg_validate_level reports it)
    const int32_t x = pos[u];
    atomicOr(&B.bm[x >> 6], 1ull << (x & 63));
  }
  __builtin_amdgcn_wave_barrier();
  const int32_t c = __popcll(B.bm[lane]);
  const int32_t inc = wave_scan_incl(c);
  B.wp[lane] = inc - c;
  if (lane == kWave - 1) B.wp[kWave] = inc;
  __builtin_amdgcn_wave_barrier();
}

__device__ inline void clear_positions(PosBits& B) {
  const int lane = threadIdx.x & (kWave - 1);
  __builtin_amdgcn_wave_barrier();
  B.bm[lane] = 0ull;
  __builtin_amdgcn_wave_barrier();
}

// ---- bisection: label-propagation gains -------------------------------------

struct GainArgs {
  HPass hp;
  int32_t V, E, depth;
  const int64_t* eoff;
  const uint32_t* pins;
  const int32_t* eta;
  const int32_t* pos;      // [S][V]
  const int32_t* tstart;
  const int32_t* tlen;
  const int32_t* leaf_of;
  const int32_t* active;   // [S][kTreeIds]
  int64_t* gain;           // [S][V], zero on entry
};

// Gain of every node of an active section at `depth` for crossing to the
// other half: +eta for a hyperedge whose only pin on the node's side is the
// node while the other half holds some; -eta for one with other pins on the
// node's side and none on the other (counting the section's nodes only).
__global__ __launch_bounds__(kHT) void lp_gain_kernel(GainArgs a) {
  __shared__ int64_t g[kMaxNodes];
  __shared__ unsigned long long bm[kHW][kWave + 1];
  __shared__ int32_t wp[kHW][kWave + 1];
  const int32_t s = a.hp.start();
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int32_t i = threadIdx.x; i < a.V; i += kHT) g[i] = 0;
  if (threadIdx.x < kHW) bm[threadIdx.x][kWave] = 0ull;
  bm[wid][lane] = 0ull;
  __syncthreads();
  const int32_t* pos = a.pos + (int64_t)s * a.V;
  const int32_t* act = a.active + (int64_t)s * kTreeIds;
  PosBits B{bm[wid], wp[wid]};
  const int64_t step = (int64_t)a.hp.per_start * kHW;
  for (int64_t e = (int64_t)a.hp.part() * kHW + wid; e < a.E; e += step) {
    const int64_t beg = a.eoff[e], end = a.eoff[e + 1];
    if (end - beg < 2) continue;  // wave-uniform
    mark_positions(a.pins, beg, end, a.V, pos, B);
    const int64_t w = a.eta[e];
    for (int64_t k = beg + lane; k < end; k += kWave) {
      const int32_t u = (int32_t)(a.pins[k] & kIdMask);
      if (u >= a.V) continue;
      const int32_t x = pos[u];
      const uint32_t leaf = (uint32_t)a.leaf_of[x];
      const int ld = depth_of(leaf);
      if (ld < a.depth) continue;
      const uint32_t hid = leaf >> (ld - a.depth);
      const int32_t len = a.tlen[hid];
      if (len < 2 || !act[hid]) continue;
      const int32_t st = a.tstart[hid], nl = len - len / 2;
      const bool left = x < st + nl;
      const int32_t cl = B.count(st, st + nl), cr = B.count(st + nl, st + len);
      const int32_t mine = left ? cl : cr, other = left ? cr : cl;
      if (mine == 1 && other > 0) atomicAdd((unsigned long long*)&g[u], (unsigned long long)w);
      else if (other == 0 && mine > 1)
        atomicAdd((unsigned long long*)&g[u], (unsigned long long)(-w));
    }
    clear_positions(B);
  }
  __syncthreads();
  int64_t* out = a.gain + (int64_t)s * a.V;
  for (int32_t i = threadIdx.x; i < a.V; i += kHT)
    if (g[i] != 0) atomicAdd((unsigned long long*)&out[i], (unsigned long long)g[i]);
}

// Sort entry of the per-start kernels: ordered by grp ascending, then val
// descending, then id ascending.
struct SortEnt {
  int64_t val;
  int32_t grp, id;
};

__device__ inline bool ent_before(const SortEnt& p, const SortEnt& q) {
  if (p.grp != q.grp) return p.grp < q.grp;
  if (p.val != q.val) return p.val > q.val;
  return p.id < q.id;
}

// Bitonic sort of n (a power of two, <= 4096) entries in LDS by one block.
__device__ inline void block_bitonic(SortEnt* v, int32_t n) {
  for (int32_t k = 2; k <= n; k <<= 1) {
    for (int32_t j = k >> 1; j > 0; j >>= 1) {
      for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int32_t l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const SortEnt p = v[i], q = v[l];
          if (up ? ent_before(q, p) : ent_before(p, q)) {
            v[i] = q;
            v[l] = p;
          }
        }
      }
      __syncthreads();
    }
  }
}

// One label-propagation round of every active section at `depth`, for one
// start per block: both halves sorted by (gain desc, id asc) and the i-th
// pairs swapped while their gains sum above 0 (the sums only fall along i,
// so each pair decides alone); a section without a swap stops.
__global__ __launch_bounds__(kPT) void lp_swap_kernel(int32_t V, int32_t depth,
                                                      const int32_t* __restrict__ tstart,
                                                      const int32_t* __restrict__ tlen,
                                                      const int32_t* __restrict__ leaf_of,
                                                      int32_t* __restrict__ seq,
                                                      int32_t* __restrict__ pos,
                                                      const int64_t* __restrict__ gain,
                                                      int32_t* __restrict__ active) {
  __shared__ SortEnt ent[kMaxNodes];
  __shared__ int32_t swaps[kTreeIds];
  const int32_t s = blockIdx.x;
  int32_t* sq = seq + (int64_t)s * V;
  int32_t* ps = pos + (int64_t)s * V;
  const int64_t* gn = gain + (int64_t)s * V;
  int32_t* act = active + (int64_t)s * kTreeIds;
  int32_t n = 1;
  while (n < V) n <<= 1;
  constexpr int32_t kNoGroup = 0x7FFFFFFF;
  for (int32_t x = threadIdx.x; x < n; x += kPT) {
    SortEnt t{0, kNoGroup, x};
    if (x < V) {
      const uint32_t leaf = (uint32_t)leaf_of[x];
      const int ld = depth_of(leaf);
      if (ld >= depth) {
        const uint32_t hid = leaf >> (ld - depth);
        const int32_t len = tlen[hid];
        if (len >= 2 && act[hid]) {
          const int32_t u = sq[x];
          const bool right = x >= tstart[hid] + (len - len / 2);
          t = SortEnt{gn[u], (int32_t)(2 * hid + (right ? 1 : 0)), u};
        }
      }
    }
    ent[x] = t;
  }
  for (int32_t i = threadIdx.x; i < kTreeIds; i += kPT) swaps[i] = 0;
  __syncthreads();
  block_bitonic(ent, n);
  // lower bound of a group in the sorted entries
  auto first_of = [&](int32_t grp) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (ent[mid].grp < grp) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  for (int32_t j = threadIdx.x; j < n; j += kPT) {
    const SortEnt L = ent[j];
    if (L.grp == kNoGroup || (L.grp & 1)) continue;
    const int32_t hid = L.grp >> 1;
    const int32_t len = tlen[hid], nl = len - len / 2;
    const int32_t i = j - first_of(L.grp);
    if (i >= len - nl) continue;
    const SortEnt R = ent[first_of(L.grp + 1) + i];
    if (L.val + R.val <= 0) continue;
    const int32_t xu = ps[L.id], xv = ps[R.id];
    ps[L.id] = xv;
    ps[R.id] = xu;
    sq[xu] = R.id;
    sq[xv] = L.id;
    atomicAdd(&swaps[hid], 1);
  }
  __syncthreads();
  const int32_t lo = 1 << depth;
  for (int32_t h = lo + threadIdx.x; h < 2 * lo && h < kTreeIds; h += kPT)
    if (act[h] && tlen[h] >= 2 && swaps[h] == 0) act[h] = 0;
}

// ---- folding ------------------------------------------------------------------

struct ConnArgs2 {
  HPass hp;
  int32_t V, E;
  const int64_t* eoff;
  const uint32_t* pins;
  const int32_t* eta;
  const int32_t* pos;
  const int32_t* tstart;
  const int32_t* tlen;
  const int32_t* leaf_of;
  int64_t* conn;  // [S][kTreeIds], zero on entry
};

// conn[c] for every section c at depth >= 2: the weight of the hyperedges
// with pins both in c and in the sibling of c's parent.  Each hyperedge
// adds its weight once per such c, from its first pin inside c.
__global__ __launch_bounds__(kHT) void fold_conn_kernel(ConnArgs2 a) {
  __shared__ int64_t cn[kTreeIds];
  __shared__ unsigned long long bm[kHW][kWave + 1];
  __shared__ int32_t wp[kHW][kWave + 1];
  const int32_t s = a.hp.start();
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int32_t i = threadIdx.x; i < kTreeIds; i += kHT) cn[i] = 0;
  if (threadIdx.x < kHW) bm[threadIdx.x][kWave] = 0ull;
  bm[wid][lane] = 0ull;
  __syncthreads();
  const int32_t* pos = a.pos + (int64_t)s * a.V;
  PosBits B{bm[wid], wp[wid]};
  const int64_t step = (int64_t)a.hp.per_start * kHW;
  for (int64_t e = (int64_t)a.hp.part() * kHW + wid; e < a.E; e += step) {
    const int64_t beg = a.eoff[e], end = a.eoff[e + 1];
    if (end - beg < 2) continue;  // wave-uniform
    mark_positions(a.pins, beg, end, a.V, pos, B);
    const int64_t w = a.eta[e];
    for (int64_t k = beg + lane; k < end; k += kWave) {
      const uint32_t u = a.pins[k] & kIdMask;
      if (u >= (uint32_t)a.V) continue;
      const int32_t x = pos[u];
      const uint32_t leaf = (uint32_t)a.leaf_of[x];
      const int ld = depth_of(leaf);
      for (int d = 2; d <= ld; ++d) {
        const uint32_t c = leaf >> (ld - d);
        if (B.count(a.tstart[c], x) != 0) continue;  // not the first pin in c
        const uint32_t u = (c >> 1) ^ 1u;
        if (B.count(a.tstart[u], a.tstart[u] + a.tlen[u]) > 0)
          atomicAdd((unsigned long long*)&cn[c], (unsigned long long)w);
      }
    }
    clear_positions(B);
  }
  __syncthreads();
  int64_t* out = a.conn + (int64_t)s * kTreeIds;
  for (int32_t i = threadIdx.x; i < kTreeIds; i += kHT)
    if (cn[i] != 0) atomicAdd((unsigned long long*)&out[i], (unsigned long long)cn[i]);
}

// Final order and cores: going up from a node's leaf, its offset inside
// each section is placed after the first child's length when it sits in
// the second child, and mirrored when the section flips (a non-root
// section flips when its child facing away from the section's sibling is
// the more connected one to that sibling).
__global__ void fold_place_kernel(int32_t S, int32_t V, const int32_t* __restrict__ seq,
                                  const int32_t* __restrict__ tlen,
                                  const int32_t* __restrict__ leaf_of,
                                  const int64_t* __restrict__ conn, const int32_t* __restrict__ hc,
                                  int32_t* __restrict__ core_of) {
  const int64_t n = (int64_t)S * V;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / V;
    const int32_t x = (int32_t)(i - s * V);
    const int64_t* cn = conn + s * kTreeIds;
    uint32_t c = (uint32_t)leaf_of[x];
    int32_t off = 0;
    while (c > 1) {
      const uint32_t sec = c >> 1;
      const int32_t len = tlen[sec], nl = len - len / 2;
      if (c & 1u) off += nl;
      if (sec > 1) {
        const int64_t k0 = cn[2 * sec], k1 = cn[2 * sec + 1];
        const bool flip = (sec & 1u) == 0 ? k0 > k1 : k1 > k0;
        if (flip) off = len - 1 - off;
      }
      c = sec;
    }
    core_of[s * V + seq[i]] = hc[off];
  }
}

// ---- swap refinement ----------------------------------------------------------

// occ[s][c] = node on core c or -1; a core outside the lattice or held
// twice sets kErrPlacement.  occ must be -1 everywhere on entry.
__global__ void occ_kernel(int32_t S, int32_t V, int32_t C, const int32_t* __restrict__ core_of,
                           const int32_t* __restrict__ done, int32_t* __restrict__ occ,
                           int32_t* __restrict__ err) {
  const int64_t n = (int64_t)S * V;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / V;
    if (done && done[s]) continue;
    const int32_t c = core_of[i];
    if (c < 0 || c >= C) {
      atomicOr(err, kErrPlacement);
      continue;
    }
    if (atomicCAS(&occ[s * C + c], -1, (int32_t)(i - s * V)) != -1) atomicOr(err, kErrPlacement);
  }
}

struct ForceArgs {
  HPass hp;
  int32_t V, E, C, width, height;
  const int64_t* eoff;
  const uint32_t* pins;
  const int32_t* eta;
  const int32_t* core_of;  // [S][V]
  const int32_t* occ;      // [S][C]
  const int32_t* done;     // [S]
  int64_t* force;          // [S][V][4], zero on entry
};

// Eq. 14 for every node towards its four neighbour cores, in ascending
// core order: d = 0 (x - 1), 1 (y - 1), 2 (y + 1), 3 (x + 1).
__global__ __launch_bounds__(kHT) void force_kernel(ForceArgs a) {
  __shared__ int64_t F[kMaxNodes * 4];
  __shared__ int32_t hx[kHW][kWave], hy[kHW][kWave], px[kHW][kWave], py[kHW][kWave];
  __shared__ unsigned long long nb[kHW][kWave];
  const int32_t s = a.hp.start();
  if (a.done[s]) return;  // block-uniform
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int32_t i = threadIdx.x; i < a.V * 4; i += kHT) F[i] = 0;
  hx[wid][lane] = 0;
  hy[wid][lane] = 0;
  nb[wid][lane] = 0ull;
  __syncthreads();
  const int32_t* core = a.core_of + (int64_t)s * a.V;
  const int32_t* oc = a.occ + (int64_t)s * a.C;
  const int32_t H = a.height;
  const int64_t step = (int64_t)a.hp.per_start * kHW;
  for (int64_t e = (int64_t)a.hp.part() * kHW + wid; e < a.E; e += step) {
    const int64_t beg = a.eoff[e], end = a.eoff[e + 1];
    const int32_t n = (int32_t)(end - beg);
    if (n < 2) continue;  // wave-uniform: no pair, no force
    for (int64_t k = beg + lane; k < end; k += kWave) {
      const int32_t u = (int32_t)(a.pins[k] & kIdMask);
      if (u >= a.V) continue;
      const int32_t c = core[u];
      if ((uint32_t)c >= (uint32_t)a.C) continue;  // reported by occ_kernel
      atomicAdd(&hx[wid][c / H], 1);
      atomicAdd(&hy[wid][c % H], 1);
      atomicOr(&nb[wid][u >> 6], 1ull << (u & 63));
    }
    __builtin_amdgcn_wave_barrier();
    px[wid][lane] = wave_scan_incl(hx[wid][lane]);
    py[wid][lane] = wave_scan_incl(hy[wid][lane]);
    __builtin_amdgcn_wave_barrier();
    const int64_t w = a.eta[e];
    for (int64_t k = beg + lane; k < end; k += kWave) {
      const int32_t u = (int32_t)(a.pins[k] & kIdMask);
      if (u >= a.V) continue;
      const int32_t c = core[u];
      if ((uint32_t)c >= (uint32_t)a.C) continue;
      const int32_t x = c / H, y = c % H;
      const int32_t xle = px[wid][x], xlt = xle - hx[wid][x];
      const int32_t yle = py[wid][y], ylt = yle - hy[wid][y];
      auto member = [&](int32_t kc) {
        const int32_t q = oc[kc];
        return q >= 0 && ((nb[wid][q >> 6] >> (q & 63)) & 1ull) ? 1 : 0;
      };
      int64_t* f = &F[u * 4];
      if (x > 0)
        atomicAdd((unsigned long long*)&f[0],
                  (unsigned long long)(w * (2 * xlt - n + 1 - member(c - H))));
      if (y > 0)
        atomicAdd((unsigned long long*)&f[1],
                  (unsigned long long)(w * (2 * ylt - n + 1 - member(c - 1))));
      if (y < H - 1)
        atomicAdd((unsigned long long*)&f[2],
                  (unsigned long long)(w * (n - 2 * yle + 1 - member(c + 1))));
      if (x < a.width - 1)
        atomicAdd((unsigned long long*)&f[3],
                  (unsigned long long)(w * (n - 2 * xle + 1 - member(c + H))));
    }
    __builtin_amdgcn_wave_barrier();
    hx[wid][lane] = 0;
    hy[wid][lane] = 0;
    nb[wid][lane] = 0ull;
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  int64_t* out = a.force + (int64_t)s * a.V * 4;
  for (int32_t i = threadIdx.x; i < a.V * 4; i += kHT)
    if (F[i] != 0) atomicAdd((unsigned long long*)&out[i], (unsigned long long)F[i]);
}

constexpr uint32_t kNone = 0x7FFFFFFFu;

// Proposals (Eq. 15), Eq. 13 over cores and the swap order, one start per
// block.  Writes the swaps sorted by (tension desc, lower core asc) and
// the swap of every moved node: rank << 8 | line << 1 | side, with line
// the column pair (x of the lower core) of a swap along x, width + the row
// pair of one along y, and side 0 for the node on the lower core.
__global__ __launch_bounds__(kPT) void propose_match_kernel(
    int32_t V, int32_t C, int32_t width, int32_t height, const int32_t* __restrict__ occ_g,
    const int64_t* __restrict__ force, const int32_t* __restrict__ done,
    int32_t* __restrict__ sw_a, int32_t* __restrict__ sw_b, int64_t* __restrict__ sw_t,
    int32_t* __restrict__ nsw, int32_t* __restrict__ swinfo, int32_t* __restrict__ err) {
  __shared__ int32_t occ[kMaxNodes], cand[kMaxNodes], bid[kMaxNodes];
  __shared__ uint32_t jmp[kMaxNodes];
  __shared__ unsigned long long bs[kMaxNodes];  // later the swap entries
  __shared__ int64_t score[kMaxNodes];
  SortEnt* const ent = reinterpret_cast<SortEnt*>(bs);
  static_assert(sizeof(SortEnt) * (kMaxNodes / 2) <= sizeof(unsigned long long) * kMaxNodes,
                "the swap entries fit in the best-score words");
  __shared__ int32_t ws[kPT / kWave];
  const int32_t s = blockIdx.x;
  if (done[s]) return;  // block-uniform
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t* F = force + (int64_t)s * V * 4;
  const int32_t H = height;
  for (int32_t h = threadIdx.x; h < C; h += kPT) occ[h] = occ_g[(int64_t)s * C + h];
  for (int32_t p = threadIdx.x; p < V; p += kPT) swinfo[(int64_t)s * V + p] = -1;
  __syncthreads();
  // proposals: the neighbour core of largest positive tension, lowest id on ties
  for (int32_t h = threadIdx.x; h < C; h += kPT) {
    const int32_t p = occ[h];
    int32_t bk = -1;
    int64_t best = 0;
    if (p >= 0) {
      const int32_t x = h / H, y = h % H;
      const int32_t ks[4] = {h - H, h - 1, h + 1, h + H};
      const bool ok[4] = {x > 0, y > 0, y < H - 1, x < width - 1};
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        if (!ok[d]) continue;
        const int32_t q = occ[ks[d]];
        const int64_t t = F[(int64_t)p * 4 + d] + (q >= 0 ? F[(int64_t)q * 4 + 3 - d] : 0);
        if (t > best) {
          best = t;
          bk = ks[d];
        }
      }
    }
    cand[h] = bk;
    score[h] = best;
    bs[h] = 0ull;
    bid[h] = 0x7FFFFFFF;
  }
  __syncthreads();
  for (int32_t h = threadIdx.x; h < C; h += kPT)
    if (cand[h] >= 0) atomicMax(&bs[cand[h]], (unsigned long long)score[h]);
  __syncthreads();
  for (int32_t h = threadIdx.x; h < C; h += kPT)
    if (cand[h] >= 0 && (unsigned long long)score[h] == bs[cand[h]]) atomicMin(&bid[cand[h]], h);
  __syncthreads();
  // up-arcs and the parity of every path (pointer jumping in place: a state
  // read from a pointer is a valid (parity, pointer) pair further down)
  for (int32_t h = threadIdx.x; h < C; h += kPT) {
    const int32_t c = cand[h];
    uint32_t up = kNone;
    if (c >= 0 && cand[c] != h && bid[c] == h) up = (uint32_t)c;
    jmp[h] = up == kNone ? kNone : (0x80000000u | up);
  }
  __syncthreads();
  for (int r = 0; r < 13; ++r) {  // 2^12 >= C: every path resolved
    uint32_t nv[kMaxNodes / kPT];
#pragma unroll
    for (int j = 0; j < kMaxNodes / kPT; ++j) {
      const int32_t h = threadIdx.x + j * kPT;
      nv[j] = 0;
      if (h < C) {
        const uint32_t st = jmp[h], ptr = st & kNone;
        nv[j] = st;
        if (ptr != kNone) {
          const uint32_t t = jmp[ptr];
          nv[j] = ((st ^ t) & 0x80000000u) | (t & kNone);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kMaxNodes / kPT; ++j) {
      const int32_t h = threadIdx.x + j * kPT;
      if (h < C) jmp[h] = nv[j];
    }
    __syncthreads();
  }
  // matches; swaps listed from their lower core
  int32_t mine[kMaxNodes / kPT];
  int32_t cnt = 0;
#pragma unroll
  for (int j = 0; j < kMaxNodes / kPT; ++j) {
    const int32_t h = threadIdx.x + j * kPT;
    mine[j] = -1;
    if (h >= C) continue;
    const int32_t c = cand[h];
    int32_t m;
    if (c >= 0 && cand[c] == h) m = c;
    else if (c >= 0 && (jmp[h] >> 31)) m = c;
    else m = bid[h] == 0x7FFFFFFF ? -1 : bid[h];
    if (m > h) {
      mine[j] = m;
      ++cnt;
    }
  }
  const int32_t inc = wave_scan_incl(cnt);
  if (lane == kWave - 1) ws[wid] = inc;
  __syncthreads();
  int32_t before = 0, total = 0;
  for (int w = 0; w < kPT / kWave; ++w) {
    if (w < wid) before += ws[w];
    total += ws[w];
  }
  // a matching holds at most C / 2 swaps
  if (total > C / 2) {
    if (threadIdx.x == 0) atomicOr(err, kErrWorkCount);
    total = C / 2;
  }
  int32_t at = before + inc - cnt;
#pragma unroll
  for (int j = 0; j < kMaxNodes / kPT; ++j) {
    const int32_t h = threadIdx.x + j * kPT;
    const int32_t m = mine[j];
    if (m < 0) continue;
    const int64_t t = cand[h] == m ? score[h] : score[m];
    if (at < total) ent[at] = SortEnt{t, 0, h};
    ++at;
  }
  int32_t n = 1;
  while (n < total) n <<= 1;
  for (int32_t i = total + threadIdx.x; i < n; i += kPT) ent[i] = SortEnt{0, 1, 0x7FFFFFFF};
  __syncthreads();
  if (total > 1) block_bitonic(ent, n);
  for (int32_t i = threadIdx.x; i < total; i += kPT) {
    const int32_t h = ent[i].id;
    // the partner: the matched neighbour above h
    const int32_t c = cand[h];
    int32_t m;
    if (c >= 0 && cand[c] == h) m = c;
    else if (c >= 0 && (jmp[h] >> 31)) m = c;
    else m = bid[h];
    const int64_t o = (int64_t)s * (C / 2 + 1) + i;
    sw_a[o] = h;
    sw_b[o] = m;
    sw_t[o] = ent[i].val;
    const bool along_x = (m / H) != (h / H);
    const int32_t line = along_x ? h / H : width + h % H;
    const int32_t pa = occ[h], pb = occ[m];
    if (pa >= 0) swinfo[(int64_t)s * V + pa] = (i << 8) | (line << 1);
    if (pb >= 0) swinfo[(int64_t)s * V + pb] = (i << 8) | (line << 1) | 1;
  }
  if (threadIdx.x == 0) nsw[s] = total;
}

struct CorrArgs {
  HPass hp;
  int32_t V, E, C;
  const int64_t* eoff;
  const uint32_t* pins;
  const int32_t* eta;
  const int32_t* swinfo;  // [S][V]
  const int32_t* nsw;
  const int32_t* done;
  int64_t* corr;          // [S][C/2 + 1], zero on entry
};

// Corrections of the tensions along the swap order: for every pair of moved
// pins of a hyperedge on the same line, the later swap gets
// 2 eta * side sign * side sign (+1 for the node on the lower core).
__global__ __launch_bounds__(kHT) void swap_corr_kernel(CorrArgs a) {
  constexpr int kBuf = 1024;
  __shared__ int64_t cr[kMaxNodes / 2 + 1];
  __shared__ int32_t buf[kHW][kBuf];
  const int32_t s = a.hp.start();
  if (a.done[s] || a.nsw[s] < 2) return;  // block-uniform
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int32_t ns = a.nsw[s];
  for (int32_t i = threadIdx.x; i < ns; i += kHT) cr[i] = 0;
  __syncthreads();
  const int32_t* si = a.swinfo + (int64_t)s * a.V;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  const int64_t step = (int64_t)a.hp.per_start * kHW;
  for (int64_t e = (int64_t)a.hp.part() * kHW + wid; e < a.E; e += step) {
    const int64_t beg = a.eoff[e], end = a.eoff[e + 1];
    if (end - beg < 2) continue;  // wave-uniform
    const int64_t w2 = 2 * (int64_t)a.eta[e];
    for (int32_t base = 0;; base += kBuf) {  // wave-uniform
      // the moved pins base .. base + kBuf - 1, in pin order
      int32_t cnt = 0;
      for (int64_t k0 = beg; k0 < end; k0 += kWave) {
        const int64_t k = k0 + lane;
        const uint32_t u = k < end ? (a.pins[k] & kIdMask) : 0xFFFFFFFFu;
        const int32_t inf = u < (uint32_t)a.V ? si[u] : -1;
        const uint64_t m = __ballot(inf >= 0);
        const int32_t idx = cnt + __popcll(m & below);
        if (inf >= 0 && idx >= base && idx < base + kBuf) buf[wid][idx - base] = inf;
        cnt += __popcll(m);
      }
      __builtin_amdgcn_wave_barrier();
      if (cnt < 2) break;
      const int32_t nb = cnt - base < kBuf ? cnt - base : kBuf;
      for (int64_t k0 = beg; k0 < end; k0 += kWave) {
        const int64_t k = k0 + lane;
        const uint32_t u = k < end ? (a.pins[k] & kIdMask) : 0xFFFFFFFFu;
        const int32_t inf = u < (uint32_t)a.V ? si[u] : -1;
        if (inf < 0) continue;
        const int32_t rank = inf >> 8, line = (inf >> 1) & 127;
        int32_t acc = 0;
        for (int32_t t = 0; t < nb; ++t) {
          const int32_t o = buf[wid][t];
          if (((o >> 1) & 127) == line && (o >> 8) < rank) acc += (o & 1) ? -1 : 1;
        }
        if (acc != 0) {
          const int64_t v = w2 * ((inf & 1) ? -acc : acc);
          atomicAdd((unsigned long long*)&cr[rank], (unsigned long long)v);
        }
      }
      __builtin_amdgcn_wave_barrier();
      if (cnt <= base + kBuf) break;
    }
  }
  __syncthreads();
  int64_t* out = a.corr + (int64_t)s * (a.C / 2 + 1);
  for (int32_t i = threadIdx.x; i < ns; i += kHT)
    if (cr[i] != 0) atomicAdd((unsigned long long*)&out[i], (unsigned long long)cr[i]);
}

// Best prefix of the recomputed tensions (largest positive sum, shortest on
// ties) applied, one start per block; a start whose best prefix is empty is
// done.  info[s] = [rounds, swaps applied, decrease of the residual].
__global__ __launch_bounds__(kPT) void apply_prefix_kernel(
    int32_t V, int32_t C, int32_t* __restrict__ core_of, const int32_t* __restrict__ occ,
    const int32_t* __restrict__ sw_a, const int32_t* __restrict__ sw_b,
    const int64_t* __restrict__ sw_t, const int64_t* __restrict__ corr,
    const int32_t* __restrict__ nsw, int32_t* __restrict__ done, int64_t* __restrict__ info,
    int32_t* __restrict__ n_done) {
  __shared__ int64_t ws[kPT / kWave];
  __shared__ unsigned long long best;
  __shared__ int32_t best_i;
  const int32_t s = blockIdx.x;
  if (done[s]) return;  // block-uniform
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int32_t ns = nsw[s];
  const int64_t o = (int64_t)s * (C / 2 + 1);
  // two swaps per thread, in order: thread t holds 2t and 2t + 1
  int64_t v0 = 0, v1 = 0;
  const int32_t i0 = 2 * threadIdx.x, i1 = i0 + 1;
  if (i0 < ns) v0 = sw_t[o + i0] + corr[o + i0];
  if (i1 < ns) v1 = sw_t[o + i1] + corr[o + i1];
  const int64_t inc = wave_scan_incl64(v0 + v1);
  if (lane == kWave - 1) ws[wid] = inc;
  if (threadIdx.x == 0) best = 0ull;
  __syncthreads();
  int64_t before = 0;
  for (int w = 0; w < wid; ++w) before += ws[w];
  const int64_t c1 = before + inc, c0 = c1 - v1;
  // the largest positive cumulative sum, then its first position
  if (threadIdx.x == 0) best_i = 0x7FFFFFFF;
  if (i0 < ns && c0 > 0) atomicMax(&best, (unsigned long long)c0);
  if (i1 < ns && c1 > 0) atomicMax(&best, (unsigned long long)c1);
  __syncthreads();
  const unsigned long long b = best;
  if (b) {
    if (i0 < ns && (unsigned long long)c0 == b && c0 > 0) atomicMin(&best_i, i0);
    else if (i1 < ns && (unsigned long long)c1 == b && c1 > 0) atomicMin(&best_i, i1);
  }
  __syncthreads();
  const int32_t len = b ? best_i + 1 : 0;
  const int64_t gain = (int64_t)b;
  for (int32_t i = threadIdx.x; i < len; i += kPT) {
    const int32_t h = sw_a[o + i], m = sw_b[o + i];
    const int32_t pa = occ[(int64_t)s * C + h], pb = occ[(int64_t)s * C + m];
    if (pa >= 0) core_of[(int64_t)s * V + pa] = m;
    if (pb >= 0) core_of[(int64_t)s * V + pb] = h;
  }
  if (threadIdx.x == 0) {
    info[3 * s] += 1;
    info[3 * s + 1] += len;
    info[3 * s + 2] += gain;
    if (len == 0) {
      done[s] = 1;
      atomicAdd(n_done, 1);
    }
  }
}

// ---- residual distance ---------------------------------------------------------

struct ResidualArgs {
  HPass hp;
  int32_t V, E, C, height;
  const int64_t* eoff;
  const uint32_t* pins;
  const int32_t* eta;
  const int32_t* core_of;
  int64_t* dist;  // [S], zero on entry
  int32_t* err;
};

// Sum over hyperedges of eta times the Manhattan distances of all pin
// pairs: per coordinate, from the histogram, every bin's pins against the
// pins of the bins below.
__global__ __launch_bounds__(kHT) void residual_kernel(ResidualArgs a) {
  __shared__ int32_t hx[kHW][kWave], hy[kHW][kWave];
  __shared__ unsigned long long tot;
  const int32_t s = a.hp.start();
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  hx[wid][lane] = 0;
  hy[wid][lane] = 0;
  if (threadIdx.x == 0) tot = 0ull;
  __syncthreads();
  const int32_t* core = a.core_of + (int64_t)s * a.V;
  const int32_t H = a.height;
  int64_t acc = 0;
  const int64_t step = (int64_t)a.hp.per_start * kHW;
  for (int64_t e = (int64_t)a.hp.part() * kHW + wid; e < a.E; e += step) {
    const int64_t beg = a.eoff[e], end = a.eoff[e + 1];
    if (end - beg < 2) continue;  // wave-uniform
    for (int64_t k = beg + lane; k < end; k += kWave) {
      const uint32_t u = a.pins[k] & kIdMask;
      if (u >= (uint32_t)a.V) continue;
      const int32_t c = core[u];
      if ((uint32_t)c >= (uint32_t)a.C) {
        atomicOr(a.err, kErrPlacement);
        continue;
      }
      atomicAdd(&hx[wid][c / H], 1);
      atomicAdd(&hy[wid][c % H], 1);
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t cx = hx[wid][lane], cy = hy[wid][lane];
    const int64_t nx = wave_scan_incl64(cx) - cx, sx = wave_scan_incl64(cx * lane) - cx * lane;
    const int64_t ny = wave_scan_incl64(cy) - cy, sy = wave_scan_incl64(cy * lane) - cy * lane;
    const int64_t pairs = cx * (lane * nx - sx) + cy * (lane * ny - sy);
    acc += (int64_t)a.eta[e] * wave_sum64(pairs);
    hx[wid][lane] = 0;
    hy[wid][lane] = 0;
    __builtin_amdgcn_wave_barrier();
  }
  if (lane == 0 && acc != 0) atomicAdd(&tot, (unsigned long long)acc);
  __syncthreads();
  if (threadIdx.x == 0 && tot != 0ull)
    atomicAdd((unsigned long long*)&a.dist[s], tot);
}

// The start of least residual distance, lowest index on ties.
__global__ void best_start_kernel(int32_t S, const int64_t* __restrict__ dist,
                                  int32_t* __restrict__ best) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int32_t b = 0;
  for (int32_t s = 1; s < S; ++s)
    if (dist[s] < dist[b]) b = s;
  *best = b;
}

int hpass_blocks(int32_t S) {
  const int cus = device_cu_count();
  int per = (2 * cus + S - 1) / S;
  if (per < 1) per = 1;
  return per;
}

struct PlaceScratch {
  int32_t* hc;
  int32_t* tstart;
  int32_t* tlen;
  int32_t* leaf_of;
  int32_t* seq;
  int32_t* pos;
  int32_t* seen;
  int32_t* active;
  int64_t* gain;
  int64_t* conn;
  template <typename A>
  void carve(A& a, int64_t S, int64_t V, int64_t C) {
    hc = a.template take<int32_t>(C);
    tstart = a.template take<int32_t>(kTreeIds);
    tlen = a.template take<int32_t>(kTreeIds);
    leaf_of = a.template take<int32_t>(V);
    seq = a.template take<int32_t>(S * V);
    pos = a.template take<int32_t>(S * V);
    seen = a.template take<int32_t>(S * V);
    active = a.template take<int32_t>(S * kTreeIds);
    gain = a.template take<int64_t>(S * V);
    conn = a.template take<int64_t>(S * kTreeIds);
  }
};

struct RefineScratch2 {
  int32_t* occ;
  int64_t* force;
  int32_t* sw_a;
  int32_t* sw_b;
  int64_t* sw_t;
  int32_t* nsw;
  int32_t* swinfo;
  int64_t* corr;
  int32_t* done;
  int32_t* n_done;
  template <typename A>
  void carve(A& a, int64_t S, int64_t V, int64_t C) {
    occ = a.template take<int32_t>(S * C);
    force = a.template take<int64_t>(S * V * 4);
    sw_a = a.template take<int32_t>(S * (C / 2 + 1));
    sw_b = a.template take<int32_t>(S * (C / 2 + 1));
    sw_t = a.template take<int64_t>(S * (C / 2 + 1));
    nsw = a.template take<int32_t>(S);
    swinfo = a.template take<int32_t>(S * V);
    corr = a.template take<int64_t>(S * (C / 2 + 1));
    done = a.template take<int32_t>(S);
    n_done = a.template take<int32_t>(1);
  }
};

int check_place(hg_ctx* c, const hg_level* gp, int32_t width, int32_t height, int32_t n_starts) {
  int rc = check_level(c, gp, false);
  if (rc) return rc;
  if (width < 1 || height < 1 || width > kMaxSide || height > kMaxSide)
    return fail(c, HG_ERR_INVALID_ARG, "lattice %d x %d outside 1..%d per side", width, height,
                kMaxSide);
  if (gp->n_vertices < 1 || gp->n_vertices > width * height)
    return fail(c, HG_ERR_INVALID_ARG, "%d nodes for %d cores", gp->n_vertices, width * height);
  if (n_starts < 1) return fail(c, HG_ERR_INVALID_ARG, "n_starts %d below 1", n_starts);
  return HG_OK;
}

}  // namespace
}  // namespace hg

using namespace hg;

extern "C" {

int hg_place_initial(hg_ctx* c, const hg_level* gp, int32_t width, int32_t height,
                     int32_t n_starts, const int32_t* orders, int32_t lp_rounds,
                     int32_t* core_of) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_place(c, gp, width, height, n_starts);
  if (rc) return rc;
  if (!orders || !core_of || lp_rounds < 0)
    return fail(c, HG_ERR_INVALID_ARG, "null orders or core_of, or negative lp_rounds");
  const int64_t S = n_starts, V = gp->n_vertices, C = (int64_t)width * height;
  Sizer sz;
  {
    PlaceScratch P;
    P.carve(sz, S, V, C);
  }
  if ((rc = ensure_arena(c, sz.off)) != HG_OK) return rc;
  Carver cv{c->arena};
  PlaceScratch P;
  P.carve(cv, S, V, C);
  hipStream_t s = c->stream;
  int32_t D = 0;
  while ((1 << D) < V) ++D;
  hilbert_kernel<<<1, kPT, 0, s>>>(width, height, P.hc);
  tree_kernel<<<1, kPT, 0, s>>>((int32_t)V, kTreeIds, P.tstart, P.tlen, P.leaf_of);
  fill_i32(P.seen, 0, S * V, s);
  fill_i32(P.pos, 0, S * V, s);  // defined even where an order is not a permutation
  orders_kernel<<<grid_for(S * V, 256, 4096), 256, 0, s>>>((int32_t)S, (int32_t)V, orders, P.seq,
                                                           P.pos, P.seen, c->dev_err);
  const int per = hpass_blocks((int32_t)S);
  const HPass hp{(int32_t)S, per};
  for (int32_t d = 0; d < D; ++d) {
    fill_i32(P.active, 1, S * kTreeIds, s);
    for (int32_t r = 0; r < lp_rounds; ++r) {
      fill_i64(P.gain, 0, S * V, s);
      GainArgs ga{hp,     (int32_t)V, gp->n_edges, d,         gp->edge_offsets, gp->pins,
                  gp->edge_weight, P.pos, P.tstart, P.tlen, P.leaf_of,        P.active,
                  P.gain};
      lp_gain_kernel<<<(int)(S * per), kHT, 0, s>>>(ga);
      lp_swap_kernel<<<(int)S, kPT, 0, s>>>((int32_t)V, d, P.tstart, P.tlen, P.leaf_of, P.seq,
                                           P.pos, P.gain, P.active);
    }
  }
  fill_i64(P.conn, 0, S * kTreeIds, s);
  ConnArgs2 ca{hp,       (int32_t)V, gp->n_edges, gp->edge_offsets, gp->pins, gp->edge_weight,
               P.pos,    P.tstart,   P.tlen,      P.leaf_of,        P.conn};
  fold_conn_kernel<<<(int)(S * per), kHT, 0, s>>>(ca);
  fold_place_kernel<<<grid_for(S * V, 256, 4096), 256, 0, s>>>(
      (int32_t)S, (int32_t)V, P.seq, P.tlen, P.leaf_of, P.conn, P.hc, core_of);
  return launch_status(c);
}

int hg_place_refine(hg_ctx* c, const hg_level* gp, int32_t width, int32_t height,
                    int32_t n_starts, int32_t* core_of, int32_t max_rounds, int64_t* info) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_place(c, gp, width, height, n_starts);
  if (rc) return rc;
  if (!core_of || !info || max_rounds < 0)
    return fail(c, HG_ERR_INVALID_ARG, "null core_of or info, or negative max_rounds");
  const int64_t S = n_starts, V = gp->n_vertices, C = (int64_t)width * height;
  Sizer sz;
  {
    RefineScratch2 R;
    R.carve(sz, S, V, C);
  }
  if ((rc = ensure_arena(c, sz.off)) != HG_OK) return rc;
  Carver cv{c->arena};
  RefineScratch2 R;
  R.carve(cv, S, V, C);
  hipStream_t s = c->stream;
  fill_i64(info, 0, 3 * S, s);
  fill_i32(R.done, 0, S, s);
  fill_i32(R.n_done, 0, 1, s);
  const int per = hpass_blocks((int32_t)S);
  const HPass hp{(int32_t)S, per};
  const int gSV = grid_for(S * V, 256, 4096);
  for (int32_t round = 0; round < max_rounds; ++round) {
    fill_i32(R.occ, -1, S * C, s);
    occ_kernel<<<gSV, 256, 0, s>>>((int32_t)S, (int32_t)V, (int32_t)C, core_of, R.done, R.occ,
                                   c->dev_err);
    fill_i64(R.force, 0, S * V * 4, s);
    ForceArgs fa{hp,       (int32_t)V, gp->n_edges, (int32_t)C, width,  height, gp->edge_offsets,
                 gp->pins, gp->edge_weight, core_of, R.occ,     R.done, R.force};
    force_kernel<<<(int)(S * per), kHT, 0, s>>>(fa);
    propose_match_kernel<<<(int)S, kPT, 0, s>>>((int32_t)V, (int32_t)C, width, height, R.occ,
                                               R.force, R.done, R.sw_a, R.sw_b, R.sw_t, R.nsw,
                                               R.swinfo, c->dev_err);
    fill_i64(R.corr, 0, S * (C / 2 + 1), s);
    CorrArgs ka{hp,       (int32_t)V, gp->n_edges, (int32_t)C, gp->edge_offsets,
                gp->pins, gp->edge_weight, R.swinfo, R.nsw,    R.done,
                R.corr};
    swap_corr_kernel<<<(int)(S * per), kHT, 0, s>>>(ka);
    apply_prefix_kernel<<<(int)S, kPT, 0, s>>>((int32_t)V, (int32_t)C, core_of, R.occ, R.sw_a,
                                              R.sw_b, R.sw_t, R.corr, R.nsw, R.done, info,
                                              R.n_done);
    if ((rc = launch_status(c)) != HG_OK) return rc;
    int32_t nd = 0;
    hipError_t e = hipMemcpyAsync(&nd, R.n_done, sizeof nd, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "placement refinement read-back");
    if (nd >= S) break;
  }
  return HG_OK;
}

int hg_place_residual(hg_ctx* c, const hg_level* gp, int32_t width, int32_t height,
                      int32_t n_starts, const int32_t* core_of, int64_t* dist, int32_t* best) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_place(c, gp, width, height, n_starts);
  if (rc) return rc;
  if (!core_of || !dist) return fail(c, HG_ERR_INVALID_ARG, "null core_of or dist");
  const int32_t S = n_starts;
  hipStream_t s = c->stream;
  fill_i64(dist, 0, S, s);
  const int per = hpass_blocks(S);
  ResidualArgs ra{HPass{S, per}, gp->n_vertices, gp->n_edges, width * height, height,
                  gp->edge_offsets, gp->pins, gp->edge_weight, core_of, dist, c->dev_err};
  residual_kernel<<<S * per, kHT, 0, s>>>(ra);
  if (best) best_start_kernel<<<1, 64, 0, s>>>(S, dist, best);
  return launch_status(c);
}

}  // extern "C"
