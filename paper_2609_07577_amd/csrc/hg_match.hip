// S3-S5: matching and coarse vertex map (paper, Section 4.1, Eq. 13).
//
// Eq. 13 reads top-down: a vertex is taken by its candidate c when c is not
// itself taken by its own candidate and c's best proposer (largest score,
// lowest id) is this vertex; a vertex that is not taken takes its best
// proposer; two-cycles match each other.  Let up(n) = cand(n) when cand(n)
// picked n as its best proposer and n is not in a two-cycle, else none.  The
// up-arcs form disjoint paths, and n is taken exactly when its distance to
// the end of its path is odd.  The parity is found by walking a few steps and
// then by pointer jumping on packed (parity, pointer) words; jumping in place
// is safe because any state a vertex reads from its pointer is a valid
// (parity, pointer) pair further down the same path.
#include "hg_internal.h"

namespace hg {

namespace {

constexpr uint32_t kNone = 0x7FFFFFFFu;
constexpr int kWalkSteps = 32;
constexpr int kJumpRounds = 27;  // 32 * 2^26 >= 2^31

__device__ inline uint64_t proposer_key(int32_t score, int32_t id) {
  return ((uint64_t)(uint32_t)score << 32) | (uint64_t)(0x7FFFFFFFu - (uint32_t)id);
}

__device__ inline int32_t key_id(uint64_t k) {
  return k == 0 ? -1 : (int32_t)(0x7FFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
}

// S3: best proposer of every vertex; any-candidate flag.
__global__ void best_child_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ cand,
                                  const int32_t* __restrict__ cscore,
                                  uint64_t* __restrict__ bkey, int32_t* __restrict__ any) {
  int64_t V = d->V;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool found = false;
  for (; i < V; i += stride) {
    int32_t c = cand[i];
    if (c >= 0) {
      atomicMax((unsigned long long*)&bkey[c],
                (unsigned long long)proposer_key(cscore[i], (int32_t)i));
      found = true;
    }
  }
  if (__ballot(found) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(any, 1);
}

__device__ inline uint32_t up_of(uint32_t x, const int32_t* __restrict__ cand,
                                 const uint64_t* __restrict__ bkey) {
  int32_t c = cand[x];
  if (c < 0) return kNone;
  if (cand[c] == (int32_t)x) return kNone;  // two-cycle
  return key_id(bkey[c]) == (int32_t)x ? (uint32_t)c : kNone;
}

// S4a: walk up to kWalkSteps up-arcs; record (parity, pointer) or the final
// parity with pointer none.
__global__ void walk_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ cand,
                            const uint64_t* __restrict__ bkey, uint32_t* __restrict__ jump,
                            int32_t* __restrict__ flags) {
  int64_t V = d->V;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool open = false;
  for (; i < V; i += stride) {
    uint32_t x = (uint32_t)i;
    uint32_t par = 0;
    uint32_t nx = up_of(x, cand, bkey);
    int steps = 0;
    while (nx != kNone && steps < kWalkSteps) {
      x = nx;
      par ^= 1u;
      ++steps;
      nx = up_of(x, cand, bkey);
    }
    uint32_t ptr = nx == kNone ? kNone : x;
    if (ptr != kNone) open = true;
    jump[i] = (par << 31) | ptr;
  }
  if (__ballot(open) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&flags[0], 1);
}

// S4b: one in-place pointer-jumping round; skipped when nothing is open.
__global__ void jump_kernel(const Dims* __restrict__ d, uint32_t* __restrict__ jump,
                            const int32_t* __restrict__ flag_in, int32_t* __restrict__ flag_out) {
  if (*flag_in == 0) return;
  int64_t V = d->V;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool open = false;
  for (; i < V; i += stride) {
    uint32_t s = jump[i];
    uint32_t ptr = s & kNone;
    if (ptr == kNone) continue;
    uint32_t t = __atomic_load_n(&jump[ptr], __ATOMIC_RELAXED);
    uint32_t par = (s ^ t) & 0x80000000u;
    uint32_t nptr = t & kNone;
    __atomic_store_n(&jump[i], par | nptr, __ATOMIC_RELAXED);
    if (nptr != kNone) open = true;
  }
  if (__ballot(open) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(flag_out, 1);
}

// S4c + S5a: match and representative flags.
__global__ void match_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ cand,
                             const uint64_t* __restrict__ bkey, const uint32_t* __restrict__ jump,
                             int32_t* __restrict__ match, int32_t* __restrict__ rep) {
  int64_t V = d->V;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < V; i += stride) {
    int32_t c = cand[i];
    int32_t m;
    if (c >= 0 && cand[c] == (int32_t)i) {
      m = c;  // two-cycle
    } else if (c >= 0 && (jump[i] >> 31)) {
      m = c;  // taken by its candidate
    } else {
      m = key_id(bkey[i]);  // takes its best proposer, if any
    }
    match[i] = m;
    rep[i] = (m < 0 || (int32_t)i < m) ? 1 : 0;
  }
}

// S5b: coarse ids.
__global__ void vmap_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ match,
                            const int64_t* __restrict__ rank, int32_t* __restrict__ vmap,
                            int32_t* __restrict__ n_coarse) {
  int64_t V = d->V;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (i == 0) *n_coarse = (int32_t)rank[V];
  for (; i < V; i += stride) {
    int32_t m = match[i];
    int64_t r = (m < 0 || (int32_t)i < m) ? i : m;
    vmap[i] = (int32_t)rank[r];
  }
}

}  // namespace

void match_and_vmap(const MatchArgs& a, int64_t maxV, hipStream_t s) {
  const int grid = grid_for(maxV, 256, 16384);
  fill_u64(a.bkey, 0, maxV, s);
  fill_i32(a.flag, 0, kJumpRounds + 2, s);
  fill_i32(a.any_cand, 0, 1, s);
  best_child_kernel<<<grid, 256, 0, s>>>(a.dims, a.cand, a.cscore, a.bkey, a.any_cand);
  walk_kernel<<<grid, 256, 0, s>>>(a.dims, a.cand, a.bkey, a.jump0, a.flag);
  int rounds = 0;
  for (int64_t reach = kWalkSteps; reach < maxV && rounds < kJumpRounds; reach *= 2) ++rounds;
  for (int r = 0; r < rounds; ++r)
    jump_kernel<<<grid, 256, 0, s>>>(a.dims, a.jump0, a.flag + r, a.flag + r + 1);
  match_kernel<<<grid, 256, 0, s>>>(a.dims, a.cand, a.bkey, a.jump0, a.match, a.rep);
  exclusive_scan_i32(a.rep, a.rank, &a.dims->V, maxV, a.partials, s);
  vmap_kernel<<<grid, 256, 0, s>>>(a.dims, a.match, a.rank, a.vmap, a.n_coarse);
}

}  // namespace hg
