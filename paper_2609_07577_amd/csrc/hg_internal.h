// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hg.h"

namespace hg {

constexpr uint32_t kDst = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;
constexpr int kWave = 64;

// Device error word.  Every data-dependent loop in the library has a bound;
// a kernel that reaches one ORs its bit in here (instead of spinning) and the
// host reports it from hg_sync.
enum : int32_t {
  kErrTableFull = 1,    // S2 score table probe bound
  kErrPassLimit = 2,    // S2 multipass pass bound
  kErrSetFull = 4,      // S8 distinct-set probe bound
  kErrHashFull = 8,     // S7 fingerprint table probe bound
  kErrWorkCount = 16,   // a work-list count above its capacity
  kErrListLength = 32,  // S7 list longer than its source hyperedge
  kErrMapRange = 64,    // a caller's vmap / part value (or n_coarse) out of range
  kErrWeight = 128,     // a hyperedge weight below 1
  kErrWeightSum = 256,  // the weights of a level sum to 2^31 or more
  kErrPlacement = 512,  // a starting order or a placement that is not one node per core
};

// Level sizes kept in device memory so that a chain of kernels can run
// without reading them back on the host.
struct Dims {
  int64_t V;
  int64_t E;
  int64_t P;
};

// Per-graph constants.  A context works on one graph at a time; a batch lays
// several graphs side by side in one level and gives every vertex its graph
// index, so the kernels look the limits up per vertex.
struct GraphConst {
  int32_t omega, phi, delta;
  int32_t max_size, max_syn, max_ax;  // level maxima (validity shortcut)
  int32_t nverts;  // vertices of the graph in this level: bounds a vertex's
                   // distinct neighbours (they lie in the same graph)
  int32_t done;  // 1 once a level of this graph had no candidate (its later
                 // levels are the same level, so the score step skips it)
};

// Run-time choices of the score step (set per context; see hg_tuning).
struct Tuning {
  int32_t load16 = 8;  // single-pass tables take X_n up to load16/16 of their slots
  int32_t fill16 = 5;  // multipass ranges aim at fill16/16 of the stream table
  int32_t dense_ratio = 8;  // dense windows for X_n * dense_ratio >= V (0: never)
  int32_t wide = 1;         // aligned windows with 16-byte body loads (0: one pin per lane)
};

// Device views of a level.
struct LevelView {
  const Dims* dims;
  const int64_t* eoff;
  const uint32_t* pins;
  const int32_t* w;
  const int32_t* mult;
  const int32_t* size;
  const int32_t* syn;
  const int32_t* ax;
  const int32_t* gid;  // graph index per vertex, or null (graph 0)
};

// Simple grid sizing: enough blocks to cover n items with `per_block` items
// per block, capped at `cap` (kernels then loop grid-stride).
inline int grid_for(int64_t n, int per_block, int cap = 65536) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

int device_cu_count();

// Work-list append with one atomic per bucket and wave.  Lane l asks for a
// slot in bucket b (0 <= b < NB, or -1 for none) and gets its position in
// that bucket.  All 64 lanes of the wave must be active: callers loop with a
// wave-uniform trip count and pass b = -1 for lanes past the end.
template <int NB>
__device__ inline int32_t wave_bucket_slot(int b, int32_t* count) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  int32_t pos = 0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const uint64_t m = __ballot(b == k);
    if (m == 0) continue;  // wave-uniform
    const int leader = __ffsll((unsigned long long)m) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(&count[k], (int32_t)__popcll(m));
    base = __builtin_amdgcn_readlane(base, leader);
    if (b == k) pos = base + (int32_t)__popcll(m & below);
  }
  return pos;
}

// Ascending bitonic sort of the KPL * kWave keys of a wave: key r of lane l
// is at position r * kWave + l (pad with the largest value).  Steps whose
// partner distance is below kWave exchange by shuffles, the others between
// a lane's own registers.  All 64 lanes must be active.
template <int KPL>
__device__ inline void wave_sort(uint32_t (&key)[KPL]) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int k = 2; k <= KPL * kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= kWave) {
        const int rj = j / kWave;
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          if (r & rj) continue;
          const bool up = ((r * kWave + lane) & k) == 0;
          const uint32_t x = key[r], y = key[r | rj];
          const uint32_t mn = x < y ? x : y, mx = x < y ? y : x;
          key[r] = up ? mn : mx;
          key[r | rj] = up ? mx : mn;
        }
      } else {
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          const uint32_t other = __shfl_xor(key[r], j, kWave);
          const bool up = ((r * kWave + lane) & k) == 0;
          const bool lower = (lane & j) == 0;
          const uint32_t mn = key[r] < other ? key[r] : other;
          const uint32_t mx = key[r] < other ? other : key[r];
          key[r] = (lower == up) ? mn : mx;
        }
      }
    }
  }
}

// ---- primitives (hg_prims.hip) --------------------------------------------
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
void fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);
void set_dims(Dims* d, int64_t V, int64_t E, int64_t P, hipStream_t s);

// Exclusive scan of n = *count entries of `in` into out[0..n], out[n] = total.
// `partials` needs scan_partials_size() int64 entries.  `count` is device.
int scan_partials_size();
void exclusive_scan_i32(const int32_t* in, int64_t* out, const int64_t* count,
                        int64_t max_count, int64_t* partials, hipStream_t s);
void exclusive_scan_i64(const int64_t* in, int64_t* out, const int64_t* count,
                        int64_t max_count, int64_t* partials, hipStream_t s);

// ---- S0/S1 (hg_transpose.hip) ----------------------------------------------
// Incidence lists: voff [V+1], vinc [P] = edge | flag << 31.
//
// Levels of at most kIncBuckets * 2^kIncBits vertices are transposed without
// global atomics, in buckets of 2^b consecutive vertices (b the smallest
// width giving at most kIncMinBuckets buckets, at most kIncBits): per-work-
// group bucket counts of an even share of the pins, one scan, a scatter of
// (vertex, entry) pairs into the buckets, then one work-group per bucket
// counting, scanning and placing its vertices' entries in LDS.  (Narrow
// buckets keep every CU busy on coarse levels with few vertices and many
// pins.)  That needs an IncScratch (carve it with incidence_scratch_carve);
// without one, or on larger levels, the lists are built with global atomic
// counters.
constexpr int kIncBits = 13;
constexpr int kIncBuckets = 4096;
constexpr int kIncMinBuckets = 1024;
constexpr int kIncBlocks = 1024;
struct IncScratch {
  uint64_t* pairs = nullptr;  // [P] (vertex << 32 | entry); may alias other scratch
  int64_t* boff = nullptr;    // [nb_cap * kIncBlocks + 1]
  int32_t* bcnt = nullptr;    // [nb_cap * kIncBlocks]
  int64_t* n = nullptr;       // [1]
  int64_t nb_cap = 0;         // buckets the arrays were carved for
};
__host__ __device__ inline int incidence_bits(int64_t V) {
  int b = 0;
  while (b < kIncBits && ((V + (1ll << b) - 1) >> b) > kIncMinBuckets) ++b;
  return b;
}
// the most buckets a level of at most maxV vertices can use
inline int64_t incidence_buckets(int64_t maxV) {
  const int64_t wide = (maxV + (1ll << kIncBits) - 1) >> kIncBits;
  if (wide > kIncMinBuckets) return wide;
  return maxV < kIncMinBuckets ? maxV : kIncMinBuckets;
}
// Levels of fewer than kIncMinPins pins keep the atomic path (and need no
// bucket arrays).
constexpr int64_t kIncMinPins = 1 << 20;
template <typename A>
IncScratch incidence_scratch_carve(A& a, int64_t maxV, int64_t maxP, uint64_t* pairs) {
  IncScratch s;
  const int64_t nb = incidence_buckets(maxV);
  if (nb < 1 || nb > kIncBuckets || maxP < kIncMinPins) return s;
  s.pairs = pairs;
  s.boff = a.template take<int64_t>(nb * kIncBlocks + 1);
  s.bcnt = a.template take<int32_t>(nb * kIncBlocks);
  s.n = a.template take<int64_t>(1);
  s.nb_cap = nb;
  return s;
}
void build_incidence(const LevelView& L, int64_t maxV, int64_t maxE, int64_t maxP,
                     int32_t* vcount, int64_t* voff, uint32_t* vinc, int64_t* partials,
                     hipStream_t s, const IncScratch& inc = IncScratch());
// acc[v] += val[e] for every flagged pin v of every hyperedge e, the pins of
// e being pins[eoff[e] .. eoff[e] + (len ? len[e] : eoff[e+1] - eoff[e])),
// E and P from `d`; v < *nv32 (or *nv64); at most maxNV.  Through the same
// buckets as build_incidence (no global atomics) when `inc` allows maxNV,
// else with global atomics.
void scatter_add_flagged(const Dims* d, const int64_t* eoff, const int32_t* len,
                         const uint32_t* pins, const int32_t* val, const int64_t* nv64,
                         const int32_t* nv32, int64_t maxNV, int64_t maxE, int32_t* acc,
                         const IncScratch& inc, int64_t* partials, hipStream_t s);
void level0_state(const Dims* d, const int64_t* eoff, const uint32_t* pins, int64_t maxV,
                  int64_t maxE, int32_t* size, int32_t* syn, int32_t* ax, int32_t* mult,
                  hipStream_t s);

// Expansion X_n = sum over incident hyperedges of their size; level maxima;
// bucket lists for the scoring kernels.
// Buckets 0-3 without, 4-7 with the shared-inbound count: single pass in the
// small table, single pass in the big table, multipass with the incident
// hyperedges staged in LDS (degree <= kWinDeg), multipass with them read
// from global memory; 8 without, 9 with it: dense windows (neighbourhoods
// that visit at least one id in Tuning::dense_ratio of the level and are
// either large or visited at least kDenseMinVisits times: coarse levels
// revisit few super-nodes very often, and one table entry per id takes the
// visits with no hashing).
constexpr int kNumBuckets = 10;
constexpr int kDenseBits = 14;          // ids per dense window: 2^14
constexpr int kMaxDenseWindows = 128;   // levels of at most 2^21 vertices
constexpr int64_t kDenseMinVisits = 1 << 16;
constexpr int kSmallSlots = 4096;
constexpr int kBigSlots = 16384;
constexpr int kBigSlotsOv = 8192;
constexpr int kMetaDeg = 1280;
constexpr int kWinDeg = 768;  // incident hyperedges of a window-kernel vertex
struct Buckets {
  int32_t* count;   // [kNumBuckets] device counters
  int32_t* list;    // [kNumBuckets * maxV]
  int64_t* visits;  // [kNumBuckets] sum of X_n over each list
};
void expansion_and_buckets(const LevelView& L, const int64_t* voff, const uint32_t* vinc,
                           int64_t maxV, int64_t* xn, GraphConst* gc, int32_t n_graphs,
                           Buckets b, Tuning t, hipStream_t s, int32_t dense_windows = 0);

// ---- S2 (hg_score.hip) ----------------------------------------------------
struct ScoreArgs {
  LevelView L;
  const int64_t* voff;
  const uint32_t* vinc;
  const int64_t* xn;
  const GraphConst* gc;
  int32_t* cursor;   // [2 * P] scratch for multipass cursors
  int32_t* cand;
  int32_t* cscore;
  int32_t* work;     // [kNumBuckets] work counters (zeroed by the launcher)
  Buckets b;
  int32_t* err;
  int32_t fill16;    // Tuning::fill16
  // Slices of every hyperedge at the aligned id windows of kWinAlignBits
  // bits: splits[e * (n_win + 1) + w] = pins of e below id w << kWinAlignBits
  // (scratch of [E * (n_win + 1)]).  n_win = 0: the windows of the score
  // step are not aligned (the level has too many ids for the array).
  uint32_t* splits = nullptr;
  int32_t n_win = 0;
  // The same at the dense windows of kDenseBits bits (n_win14 = 0: none).
  uint32_t* splits14 = nullptr;
  int32_t n_win14 = 0;
  int32_t wide = 1;  // Tuning::wide
};
constexpr int kWinAlignBits = 19;
constexpr int kMaxAlignedWindows = 16;
void score_candidates(const ScoreArgs& a, int64_t maxV, int64_t maxP, hipStream_t s);
// Dense-window scoring of work lists 8 and 9 (hg_score_dense.hip); called by
// score_candidates, a no-op on levels without dense windows.
void score_dense(const ScoreArgs& a, int64_t maxV, hipStream_t s);
// Aligned-window scoring of work list `bucket` (2, or 6 with the overlap)
// with 16-byte body loads (hg_score_wide.hip); false when the level has no
// aligned windows or its pins are not 16-byte aligned (nothing launched).
bool score_wide(const ScoreArgs& a, int bucket, bool ov, int64_t maxV, hipStream_t s);

// ---- S3-S5 (hg_match.hip) ---------------------------------------------------
struct MatchArgs {
  const Dims* dims;
  const int32_t* cand;
  const int32_t* cscore;
  uint64_t* bkey;      // [V]
  uint32_t* jump0;     // [V]
  uint32_t* jump1;     // [V]
  int32_t* flag;       // [4] device flags
  int32_t* match;      // [V] out
  int32_t* vmap;       // [V] out
  int32_t* rep;        // [V] scratch
  int64_t* rank;       // [V+1] scratch
  int64_t* partials;
  int32_t* n_coarse;   // device scalar out
  int32_t* any_cand;   // device scalar out
};
void match_and_vmap(const MatchArgs& a, int64_t maxV, hipStream_t s);

// ---- S6/S7 + state (hg_contract.hip) --------------------------------------
struct ContractScratch {
  int32_t* dstmult;     // [V]
  uint32_t* tpin;       // [P]
  int32_t* tlen;        // [E]
  uint64_t* fp;         // [E]
  int32_t* ebucket;     // [4 * E] size-bucket lists
  int32_t* ecount;      // [4] counters
  int32_t* work;        // [4] work counters
  uint64_t* htab_key;   // [T]
  int32_t* htab_lead;   // [T]
  int64_t htab_cap;     // T (power of two)
  int32_t* slot;        // [E]
  int32_t* group;       // [E]
  int32_t* mism;        // [E] mismatch list
  int32_t* lflag;       // [E]
  int64_t* lrank;       // [E+1]
  int32_t* leader_at;   // [E]
  int64_t* llen;        // [E]
  int64_t* partials;
  uint32_t* bitmap;     // huge-hyperedge fallback [n_wg * words]
  int64_t bitmap_words; // per work-group
  Dims* out_dims;       // device Dims of the output level
  IncScratch inc;       // buckets of the flagged-multiplicity sums
  int32_t* err;
  uint64_t fp_mask = ~0ull;  // bits of the S7 fingerprints kept (all but in tests)
};
int contract_level(const LevelView& L, int64_t maxV, int64_t maxE, int64_t maxP,
                   const int32_t* vmap, const int32_t* n_coarse, hg_level_out* out,
                   const ContractScratch& cs, hipStream_t s);

// ---- S8 (hg_conn.hip) -----------------------------------------------------
struct ConnScratch {
  int32_t* ebucket;     // [4 * E]
  int32_t* ecount;      // [4]
  int32_t* work;        // [4]
  uint32_t* bitmap;
  int64_t bitmap_words;
  int32_t* err;
};
void connectivity(const LevelView& L, int64_t maxE, int64_t part_range, const int32_t* part,
                  int64_t* conn, const ConnScratch& cs, hipStream_t s);

// Number of work-groups of the huge-segment fallback kernels.
constexpr int kHugeWG = 64;

}  // namespace hg
