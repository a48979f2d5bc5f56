// Batches of independent hypergraphs coarsened together.
//
// The graphs of a batch are laid side by side as one level (the "union"):
// graph k's vertex ids, hyperedges and pins follow those of the graphs before
// it, every vertex carries its graph's slot, and every slot has its own core
// limits.  Graphs share no hyperedge, so scores, candidates and the matching
// (Section 4.1, Eq. 12-13) never cross graphs, and the contraction (Section 3,
// G_P) keeps every graph's vertices, hyperedges and pins contiguous and in
// order (coarse vertices are numbered by smallest member, coarse hyperedges by
// smallest fine hyperedge).  One union level step therefore advances every
// graph by one level of its own hierarchy, with the same result as a
// separate run.
//
// A graph is finished after the first level at which none of its vertices
// proposes a candidate (its later levels would be the same level); from then
// on the score step skips its vertices.  Graphs may be added between steps
// (graphs at different depths coexist in one union), finished graphs are
// reported, their partitions read out and their slots released; compaction
// removes released graphs from the union.
//
// Every kernel of a level step reads the level sizes from device memory, so a
// step never waits for the host; it can be captured once per direction of
// the two level buffers in a HIP graph and replayed.
#include <algorithm>
#include <new>
#include <type_traits>
#include <vector>

#include "hg_host.h"

namespace hg {
namespace {

__global__ void set_slot_kernel(GraphConst* gc, int32_t* nlev, int32_t* active, int32_t slot,
                                hg_limits lim, int32_t done) {
  GraphConst& g = gc[slot];
  g.omega = lim.max_neurons;
  g.phi = lim.max_synapses;
  g.delta = lim.max_axons;
  g.max_size = g.max_syn = g.max_ax = 0;
  g.nverts = 0;
  g.done = done;
  nlev[slot] = 0;
  active[slot] = 0;
}

// Appends graph pieces at the end of the union, whose current sizes are read
// from device memory (no host synchronisation): offsets shifted by the pins
// before them, vertex ids by the vertices before them (flags kept).
__global__ void append_level_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ seoff,
                                    const uint32_t* __restrict__ spins, const int32_t* __restrict__ sw,
                                    const int32_t* __restrict__ smult, const int32_t* __restrict__ ssize,
                                    const int32_t* __restrict__ ssyn, const int32_t* __restrict__ sax,
                                    int64_t Vg, int64_t Eg, int64_t Pg, int32_t slot,
                                    int64_t* __restrict__ eoff, uint32_t* __restrict__ pins,
                                    int32_t* __restrict__ w, int32_t* __restrict__ mult,
                                    int32_t* __restrict__ size, int32_t* __restrict__ syn,
                                    int32_t* __restrict__ ax, int32_t* __restrict__ gid,
                                    int32_t* __restrict__ part, int32_t* __restrict__ owner,
                                    int64_t pool_off) {
  const int64_t V = d->V, E = d->E, P = d->P;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i <= Eg; i += stride) eoff[E + i] = seoff[i] + P;
  for (int64_t i = i0; i < Pg; i += stride) {
    const uint32_t p = spins[i];
    pins[P + i] = ((p & kIdMask) + (uint32_t)V) | (p & kDst);
  }
  for (int64_t i = i0; i < Eg; i += stride) {
    w[E + i] = sw[i];
    mult[E + i] = smult[i];
  }
  for (int64_t i = i0; i < Vg; i += stride) {
    size[V + i] = ssize[i];
    syn[V + i] = ssyn[i];
    ax[V + i] = sax[i];
    gid[V + i] = slot;
    part[pool_off + i] = (int32_t)(V + i);
    owner[pool_off + i] = slot;
  }
}

__global__ void grow_dims_kernel(Dims* d, int64_t Vg, int64_t Eg, int64_t Pg) {
  d->V += Vg;
  d->E += Eg;
  d->P += Pg;
}

// ---- compaction: drop the vertices, hyperedges and pins of released graphs
__global__ void keep_marks_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
                                  const uint32_t* __restrict__ pins, const int32_t* __restrict__ gid,
                                  const int32_t* __restrict__ alive, int32_t* __restrict__ keepv,
                                  int32_t* __restrict__ keepe, int32_t* __restrict__ elen) {
  const int64_t V = d->V, E = d->E;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = i0; v < V; v += stride) keepv[v] = alive[gid[v]];
  for (int64_t e = i0; e < E; e += stride) {
    const int64_t len = eoff[e + 1] - eoff[e];
    const int32_t k = len > 0 ? alive[gid[pins[eoff[e]] & kIdMask]] : 0;
    keepe[e] = k;
    elen[e] = k ? (int32_t)len : 0;
  }
}

__global__ void compact_vertices_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ keepv,
                                        const int64_t* __restrict__ vpos,
                                        const int32_t* __restrict__ size, const int32_t* __restrict__ syn,
                                        const int32_t* __restrict__ ax, const int32_t* __restrict__ gid,
                                        int32_t* __restrict__ osize, int32_t* __restrict__ osyn,
                                        int32_t* __restrict__ oax, int32_t* __restrict__ ogid) {
  const int64_t V = d->V;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = i0; v < V; v += stride) {
    if (!keepv[v]) continue;
    const int64_t q = vpos[v];
    osize[q] = size[v];
    osyn[q] = syn[v];
    oax[q] = ax[v];
    ogid[q] = gid[v];
  }
}

// A wave per hyperedge: kept hyperedges move to their new slot, their pins
// are relabelled through the new vertex positions.
__global__ void compact_edges_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
                                     const uint32_t* __restrict__ pins, const int32_t* __restrict__ w,
                                     const int32_t* __restrict__ mult, const int32_t* __restrict__ keepe,
                                     const int64_t* __restrict__ epos, const int64_t* __restrict__ ppos,
                                     const int64_t* __restrict__ vpos, int64_t* __restrict__ oeoff,
                                     uint32_t* __restrict__ opins, int32_t* __restrict__ ow,
                                     int32_t* __restrict__ omult) {
  const int64_t E = d->E;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x / kWave) +
                     __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (int64_t e = w0; e < E; e += nwaves) {  // wave-uniform
    if (!keepe[e]) continue;
    const int64_t q = epos[e], dst = ppos[e];
    if (lane == 0) {
      oeoff[q] = dst;
      ow[q] = w[e];
      omult[q] = mult[e];
    }
    const int64_t s0 = eoff[e], n = eoff[e + 1] - s0;
    for (int64_t k = lane; k < n; k += kWave) {
      const uint32_t p = pins[s0 + k];
      opins[dst + k] = (uint32_t)vpos[p & kIdMask] | (p & kDst);
    }
  }
}

__global__ void compact_finish_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ vpos,
                                      const int64_t* __restrict__ epos,
                                      const int64_t* __restrict__ ppos, int64_t* __restrict__ oeoff,
                                      Dims* __restrict__ od) {
  const int64_t V2 = vpos[d->V], E2 = epos[d->E], P2 = ppos[d->E];
  oeoff[E2] = P2;
  od->V = V2;
  od->E = E2;
  od->P = P2;
}

__global__ void pool_marks_kernel(const int64_t* __restrict__ pool_n,
                                  const int32_t* __restrict__ owner, int32_t* __restrict__ keep) {
  const int64_t n = *pool_n;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n; i += stride) keep[i] = owner[i] >= 0;
}

__global__ void pool_compact_kernel(const int64_t* __restrict__ pool_n,
                                    const int32_t* __restrict__ keep,
                                    const int64_t* __restrict__ pos, const int64_t* __restrict__ vpos,
                                    const int32_t* __restrict__ part, const int32_t* __restrict__ owner,
                                    int32_t* __restrict__ opart, int32_t* __restrict__ oowner) {
  const int64_t n = *pool_n;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n; i += stride) {
    if (!keep[i]) continue;
    const int64_t q = pos[i];
    opart[q] = (int32_t)vpos[part[i]];
    oowner[q] = owner[i];
  }
}

__global__ void set_dims_dev_kernel(Dims* d, int64_t V, int64_t E, int64_t P) {
  d->V = V;
  d->E = E;
  d->P = P;
}

__global__ void set_i64_kernel(int64_t* p, int64_t v) { *p = v; }

// Graphs with a candidate at this level.
__global__ void activity_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ cand,
                                const int32_t* __restrict__ gid, int32_t* __restrict__ active) {
  int64_t V = d->V;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < V; i += stride)
    if (cand[i] >= 0) active[gid[i]] = 1;
}

__global__ void graph_update_kernel(int32_t n_slots, int32_t* __restrict__ active,
                                    int32_t* __restrict__ nlev, GraphConst* __restrict__ gc) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_slots) return;
  if (!gc[g].done) {
    if (active[g]) nlev[g] += 1;
    else gc[g].done = 1;
  }
  active[g] = 0;
}

// The coarse vertex of a pair inherits the pair's graph.
__global__ void gid_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ vmap,
                           const int32_t* __restrict__ gid, int32_t* __restrict__ gid_out) {
  int64_t V = d->V;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < V; i += stride) gid_out[vmap[i]] = gid[i];
}

// Composed vertex map of every original vertex still owned by a graph.
__global__ void compose_kernel(const int64_t* __restrict__ pool_n, const int32_t* __restrict__ owner,
                               const int32_t* __restrict__ vmap, int32_t* __restrict__ part) {
  int64_t n = *pool_n;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride)
    if (owner[i] >= 0) part[i] = vmap[part[i]];
}

// First and last vertex and hyperedge of every graph in the current level.
// Graphs are contiguous, so a wave usually sees one graph: it reduces its
// range first and makes one atomic per bound.
__device__ inline void wave_range(int g, int32_t x, bool ok, int32_t* mn, int32_t* mx) {
  const int lane = threadIdx.x & (kWave - 1);
  const int g0 = __builtin_amdgcn_readfirstlane(g);
  if (__ballot(ok && g != g0) == 0) {  // wave-uniform
    int32_t lo = ok ? x : 0x7FFFFFFF, hi = ok ? x : -1;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
      const int32_t a = __shfl_xor(lo, d, kWave), b = __shfl_xor(hi, d, kWave);
      lo = a < lo ? a : lo;
      hi = b > hi ? b : hi;
    }
    if (lane == 0 && hi >= 0) {
      atomicMin(&mn[g0], lo);
      atomicMax(&mx[g0], hi);
    }
  } else if (ok) {
    atomicMin(&mn[g], x);
    atomicMax(&mx[g], x);
  }
}

__global__ void ranges_kernel(const Dims* __restrict__ d, const int64_t* __restrict__ eoff,
                              const uint32_t* __restrict__ pins, const int32_t* __restrict__ gid,
                              int32_t* __restrict__ vmin, int32_t* __restrict__ vmax,
                              int32_t* __restrict__ emin, int32_t* __restrict__ emax) {
  const int64_t V = d->V, E = d->E;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = (int64_t)blockIdx.x * blockDim.x +
                        __builtin_amdgcn_readfirstlane(threadIdx.x & ~(kWave - 1));
  for (int64_t base = start; base < V; base += stride) {  // wave-uniform
    const int64_t v = base + lane;
    const bool ok = v < V;
    wave_range(ok ? gid[v] : -1, (int32_t)v, ok, vmin, vmax);
  }
  for (int64_t base = start; base < E; base += stride) {  // wave-uniform
    const int64_t e = base + lane;
    bool ok = e < E && eoff[e + 1] > eoff[e];
    const int g = ok ? gid[pins[eoff[e]] & kIdMask] : -1;
    wave_range(g, (int32_t)e, ok, emin, emax);
  }
}

__global__ void relative_kernel(const int32_t* __restrict__ part, int64_t n, int32_t base,
                                int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = part[i] - base;
}

template <typename T>
__global__ void copy_kernel(const T* __restrict__ src, int64_t n, T* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

int blocks_for(int64_t n) { return grid_for(n, 256, 8192); }

}  // namespace
}  // namespace hg

using namespace hg;

namespace {

struct LevelBuf {
  Dims* dims;
  int64_t* eoff;
  uint32_t* pins;
  int32_t* w;
  int32_t* mult;
  int32_t* size;
  int32_t* syn;
  int32_t* ax;
  int32_t* gid;
};

enum SlotState : int { kFree = 0, kLive = 1, kReported = 2, kReleased = 3 };

struct SlotInfo {
  int state = kFree;
  int64_t pool_off = 0;  // original vertices of the graph in the part pool
  int64_t v0 = 0;        // number of original vertices
};

}  // namespace

struct hg_batch {
  hg_ctx* ctx = nullptr;
  int32_t max_graphs = 0;
  int64_t capV = 0, capE = 0, capP = 0;
  char* mem = nullptr;
  size_t mem_bytes = 0;
  LevelBuf buf[2] = {};
  int cur = 0;
  // products of a level step
  int32_t *cand = nullptr, *cscore = nullptr, *match = nullptr, *vmap = nullptr;
  int32_t *n_coarse = nullptr, *any_cand = nullptr;
  // per slot
  GraphConst* gc = nullptr;
  int32_t *nlev = nullptr, *active = nullptr;
  int32_t *vmin = nullptr, *vmax = nullptr, *emin = nullptr, *emax = nullptr;
  // original vertex -> current union vertex, with the owning slot (-1: free)
  int32_t *part = nullptr, *owner = nullptr, *part_tmp = nullptr;
  int64_t* pool_n = nullptr;  // device copy of pool_used
  int64_t pool_used = 0;
  CoarsenScratch<Carver> cs;
  ContractLayout<Carver> ks;
  std::vector<SlotInfo> slots;
  hipStream_t cap_stream = nullptr;  // private stream used only for capture
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  Tuning captured_tuning;
  int levels_run = 0;
  // compaction scratch
  int32_t *c_keepv = nullptr, *c_keepe = nullptr, *c_elen = nullptr, *c_alive = nullptr;
  int32_t *c_pkeep = nullptr, *owner_tmp = nullptr;
  int64_t *c_vpos = nullptr, *c_epos = nullptr, *c_ppos = nullptr, *c_pool = nullptr;
  int64_t* c_partials = nullptr;
  std::vector<int32_t> alive_h;
  // upper bounds of the current level's sizes (exact after a compaction;
  // levels only shrink, adds are counted in)
  int64_t ubV = 0, ubE = 0, ubP = 0;
  int64_t version = 0;        // bumped whenever the level changes
  int64_t ranges_version = -1;
  std::vector<int32_t> rv_min, rv_max, re_min, re_max;  // ranges of `ranges_version`
};

namespace {

template <typename A>
void carve_batch(hg_batch* b, A& a) {
  for (int k = 0; k < 2; ++k) {
    LevelBuf& L = b->buf[k];
    L.dims = a.template take<Dims>(1);
    L.eoff = a.template take<int64_t>(b->capE + 1);
    L.pins = a.template take<uint32_t>(b->capP);
    L.w = a.template take<int32_t>(b->capE);
    L.mult = a.template take<int32_t>(b->capE);
    L.size = a.template take<int32_t>(b->capV);
    L.syn = a.template take<int32_t>(b->capV);
    L.ax = a.template take<int32_t>(b->capV);
    L.gid = a.template take<int32_t>(b->capV);
  }
  b->cand = a.template take<int32_t>(b->capV);
  b->cscore = a.template take<int32_t>(b->capV);
  b->match = a.template take<int32_t>(b->capV);
  b->vmap = a.template take<int32_t>(b->capV);
  b->n_coarse = a.template take<int32_t>(1);
  b->any_cand = a.template take<int32_t>(1);
  b->gc = a.template take<GraphConst>(b->max_graphs);
  b->nlev = a.template take<int32_t>(b->max_graphs);
  b->active = a.template take<int32_t>(b->max_graphs);
  b->vmin = a.template take<int32_t>(b->max_graphs);
  b->vmax = a.template take<int32_t>(b->max_graphs);
  b->emin = a.template take<int32_t>(b->max_graphs);
  b->emax = a.template take<int32_t>(b->max_graphs);
  b->part = a.template take<int32_t>(b->capV);
  b->owner = a.template take<int32_t>(b->capV);
  b->part_tmp = a.template take<int32_t>(b->capV);
  b->pool_n = a.template take<int64_t>(1);
  b->c_keepv = a.template take<int32_t>(b->capV);
  b->c_vpos = a.template take<int64_t>(b->capV + 1);
  b->c_keepe = a.template take<int32_t>(b->capE);
  b->c_elen = a.template take<int32_t>(b->capE);
  b->c_epos = a.template take<int64_t>(b->capE + 1);
  b->c_ppos = a.template take<int64_t>(b->capE + 1);
  b->c_alive = a.template take<int32_t>(b->max_graphs);
  b->c_pkeep = a.template take<int32_t>(b->capV);
  b->c_pool = a.template take<int64_t>(b->capV + 1);
  b->owner_tmp = a.template take<int32_t>(b->capV);
  b->c_partials = a.template take<int64_t>(scan_partials_size());
  CoarsenScratch<A> cs;
  cs.carve(a, b->capV, b->capE, b->capP);
  ContractLayout<A> ks;
  ks.carve(a, b->capV, b->capE, b->capP);
  if constexpr (std::is_same<A, Carver>::value) {
    b->cs = cs;
    b->ks = ks;
  }
}

// One level of every graph in the union: buffer `from` -> buffer `to`.
void level_step(hg_batch* b, int from, int to) {
  hg_ctx* c = b->ctx;
  hipStream_t s = c->stream;
  const LevelBuf& F = b->buf[from];
  const LevelBuf& T = b->buf[to];
  const int64_t V = b->capV, E = b->capE, P = b->capP;
  auto& S = b->cs;
  LevelView L{F.dims, F.eoff, F.pins, F.w, F.mult, F.size, F.syn, F.ax, F.gid};
  build_incidence(L, V, E, P, S.vcount, S.voff, S.vinc, S.partials, s, S.inc);
  Buckets bk{S.bcount, S.blist, S.bvisits};
  expansion_and_buckets(L, S.voff, S.vinc, V, S.xn, b->gc, b->max_graphs, bk, c->tuning, s,
                        S.n_win14);
  ScoreArgs sa{L,  S.voff, S.vinc, S.xn,      b->gc, S.cursor,         b->cand,
               b->cscore, S.work, bk, c->dev_err, c->tuning.fill16};
  sa.wide = c->tuning.wide;
  // aligned and dense windows over the union's ids, where the capacity
  // allows their split tables
  sa.splits = S.splits;
  sa.n_win = S.n_win;
  sa.splits14 = S.splits14;
  sa.n_win14 = S.n_win14;
  score_candidates(sa, V, P, s);
  MatchArgs ma{F.dims, b->cand, b->cscore, S.bkey, S.jump, S.jump, S.flags, b->match, b->vmap,
               S.rep, S.rank, S.partials, b->n_coarse, b->any_cand};
  match_and_vmap(ma, V, s);
  activity_kernel<<<blocks_for(V), 256, 0, s>>>(F.dims, b->cand, F.gid, b->active);
  graph_update_kernel<<<(b->max_graphs + 255) / 256, 256, 0, s>>>(b->max_graphs, b->active,
                                                                   b->nlev, b->gc);
  hg_level_out out{(int32_t)V, (int32_t)E, P,    T.eoff, T.pins, T.w,
                   T.mult,     T.size,     T.syn, T.ax,   reinterpret_cast<int64_t*>(T.dims)};
  b->ks.cs.err = c->dev_err;
  b->ks.cs.fp_mask = c->fp_mask;
  contract_level(L, V, E, P, b->vmap, b->n_coarse, &out, b->ks.cs, s);
  gid_kernel<<<blocks_for(V), 256, 0, s>>>(F.dims, b->vmap, F.gid, T.gid);
  compose_kernel<<<blocks_for(V), 256, 0, s>>>(b->pool_n, b->owner, b->vmap, b->part);
}

int read_dims(hg_batch* b, Dims* h) {
  hipError_t e = hipMemcpyAsync(h, b->buf[b->cur].dims, sizeof(Dims), hipMemcpyDeviceToHost,
                                b->ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->ctx->stream);
  if (e != hipSuccess) return hip_fail(b->ctx, e, "reading the batch level sizes");
  return HG_OK;
}

void drop_graphs(hg_batch* b) {
  for (int k = 0; k < 2; ++k) {
    if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
    if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
    b->exec[k] = nullptr;
    b->graph[k] = nullptr;
  }
}

// Current vertex and hyperedge ranges of every slot (synchronous).
int read_ranges(hg_batch* b, std::vector<int32_t>& vmn, std::vector<int32_t>& vmx,
                std::vector<int32_t>& emn, std::vector<int32_t>& emx) {
  if (b->ranges_version == b->version) {
    vmn = b->rv_min;
    vmx = b->rv_max;
    emn = b->re_min;
    emx = b->re_max;
    return HG_OK;
  }
  hipStream_t s = b->ctx->stream;
  const int G = b->max_graphs;
  fill_i32(b->vmin, 0x7FFFFFFF, G, s);
  fill_i32(b->vmax, -1, G, s);
  fill_i32(b->emin, 0x7FFFFFFF, G, s);
  fill_i32(b->emax, -1, G, s);
  const LevelBuf& L = b->buf[b->cur];
  int64_t m = b->capV > b->capE ? b->capV : b->capE;
  ranges_kernel<<<blocks_for(m), 256, 0, s>>>(L.dims, L.eoff, L.pins, L.gid, b->vmin, b->vmax,
                                               b->emin, b->emax);
  vmn.resize(G);
  vmx.resize(G);
  emn.resize(G);
  emx.resize(G);
  hipError_t e = hipMemcpyAsync(vmn.data(), b->vmin, G * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(vmx.data(), b->vmax, G * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(emn.data(), b->emin, G * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(emx.data(), b->emax, G * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(b->ctx, e, "reading the batch ranges");
  b->rv_min = vmn;
  b->rv_max = vmx;
  b->re_min = emn;
  b->re_max = emx;
  b->ranges_version = b->version;
  return HG_OK;
}

}  // namespace

extern "C" {

int hg_batch_create(hg_ctx* c, int32_t max_graphs, int32_t cap_vertices, int32_t cap_edges,
                    int64_t cap_pins, hg_batch** out) {
  if (!c || !out) return HG_ERR_INVALID_ARG;
  *out = nullptr;
  if (max_graphs < 1 || cap_vertices < 0 || cap_edges < 0 || cap_pins < 0)
    return fail(c, HG_ERR_INVALID_ARG, "bad batch capacities");
  if (cap_vertices > 0x7FFFFFFE) return fail(c, HG_ERR_OVERFLOW, "too many vertices");
  if (cap_pins > 0x7FFFFFFF) return fail(c, HG_ERR_OVERFLOW, "2^31 or more pins");
  hg_batch* b = new (std::nothrow) hg_batch();
  if (!b) return fail(c, HG_ERR_NO_MEMORY, "host allocation failed");
  b->ctx = c;
  b->max_graphs = max_graphs;
  b->capV = cap_vertices;
  b->capE = cap_edges;
  b->capP = cap_pins;
  Sizer sz;
  carve_batch(b, sz);
  hipError_t e = hipMalloc((void**)&b->mem, sz.off);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete b;
    return fail(c, HG_ERR_NO_MEMORY, "cannot allocate %zu bytes for the batch", sz.off);
  }
  b->mem_bytes = sz.off;
  Carver cv{b->mem};
  carve_batch(b, cv);
  b->slots.assign(max_graphs, SlotInfo{});
  hipStream_t s = c->stream;
  for (int k = 0; k < 2; ++k) {
    set_dims_dev_kernel<<<1, 1, 0, s>>>(b->buf[k].dims, 0, 0, 0);
    fill_i64(b->buf[k].eoff, 0, 1, s);
  }
  hg_limits none{0, 0, 0};
  for (int32_t g = 0; g < max_graphs; ++g)
    set_slot_kernel<<<1, 1, 0, s>>>(b->gc, b->nlev, b->active, g, none, 1);
  set_i64_kernel<<<1, 1, 0, s>>>(b->pool_n, 0);
  fill_i32(b->owner, -1, b->capV, s);
  fill_i32(b->any_cand, 0, 1, s);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(b->mem);
    delete b;
    return hip_fail(c, e, "batch initialisation");
  }
  *out = b;
  return HG_OK;
}

int hg_batch_destroy(hg_batch* b) {
  if (!b) return HG_OK;
  (void)hipStreamSynchronize(b->ctx->stream);
  drop_graphs(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->mem) (void)hipFree(b->mem);
  delete b;
  return HG_OK;
}

int64_t hg_batch_bytes(hg_batch* b) { return b ? (int64_t)b->mem_bytes : 0; }

int hg_batch_add_graph(hg_batch* b, const hg_level* lvl, const hg_limits* lim, int32_t* slot) {
  if (!b || !slot) return HG_ERR_INVALID_ARG;
  hg_ctx* c = b->ctx;
  int rc = check_level(c, lvl, true);
  if (rc) return rc;
  if (!lim || lim->max_neurons < 0 || lim->max_synapses < 0 || lim->max_axons < 0)
    return fail(c, HG_ERR_INVALID_ARG, "bad limits");
  int32_t g = -1;
  for (int32_t k = 0; k < b->max_graphs; ++k)
    if (b->slots[k].state == kFree) {
      g = k;
      break;
    }
  if (g < 0) return fail(c, HG_ERR_CAPACITY, "all %d graph slots are in use", b->max_graphs);
  const int64_t Vg = lvl->n_vertices, Eg = lvl->n_edges, Pg = lvl->n_pins;
  if (b->ubV + Vg > b->capV || b->ubE + Eg > b->capE || b->ubP + Pg > b->capP)
    return fail(c, HG_ERR_CAPACITY,
                "batch level full: at most (%lld, %lld, %lld) + (%lld, %lld, %lld) above "
                "capacity; compact first",
                (long long)b->ubV, (long long)b->ubE, (long long)b->ubP, (long long)Vg,
                (long long)Eg, (long long)Pg);
  if (b->pool_used + Vg > b->capV)
    return fail(c, HG_ERR_CAPACITY, "original-vertex pool full; release or compact first");
  hipStream_t s = c->stream;
  LevelBuf& L = b->buf[b->cur];
  // offsets and ids come from the device sizes: no host synchronisation
  const int64_t m = std::max(Vg, std::max(Eg + 1, Pg));
  append_level_kernel<<<blocks_for(m), 256, 0, s>>>(
      L.dims, lvl->edge_offsets, lvl->pins, lvl->edge_weight, lvl->edge_mult, lvl->v_size,
      lvl->v_syn, lvl->v_axons, Vg, Eg, Pg, g, L.eoff, L.pins, L.w, L.mult, L.size, L.syn, L.ax,
      L.gid, b->part, b->owner, b->pool_used);
  grow_dims_kernel<<<1, 1, 0, s>>>(L.dims, Vg, Eg, Pg);
  set_slot_kernel<<<1, 1, 0, s>>>(b->gc, b->nlev, b->active, g, *lim, 0);
  b->ubV += Vg;
  b->ubE += Eg;
  b->ubP += Pg;
  b->version += 1;
  b->slots[g].state = kLive;
  b->slots[g].pool_off = b->pool_used;
  b->slots[g].v0 = Vg;
  b->pool_used += Vg;
  set_i64_kernel<<<1, 1, 0, s>>>(b->pool_n, b->pool_used);
  *slot = g;
  return launch_status(c);
}

int hg_batch_step(hg_batch* b, int32_t n_levels, int32_t use_graph) {
  if (!b || n_levels < 0) return HG_ERR_INVALID_ARG;
  hg_ctx* c = b->ctx;
  hipStream_t s = c->stream;
  if (use_graph) {
    if (b->exec[0] && (b->captured_tuning.load16 != c->tuning.load16 ||
                       b->captured_tuning.fill16 != c->tuning.fill16 ||
                       b->captured_tuning.dense_ratio != c->tuning.dense_ratio ||
                       b->captured_tuning.wide != c->tuning.wide))
      drop_graphs(b);
    if (!b->exec[0]) {
      // capture on a private stream (the context's may be the null stream,
      // which cannot be captured); the graphs are launched on the context's
      if (!b->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreateWithFlags");
      }
      for (int from = 0; from < 2; ++from) {
        hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
        c->stream = b->cap_stream;
        level_step(b, from, 1 - from);
        c->stream = s;
        e = hipStreamEndCapture(b->cap_stream, &b->graph[from]);
        if (e != hipSuccess) {
          drop_graphs(b);
          return hip_fail(c, e, "hipStreamEndCapture");
        }
        e = hipGraphInstantiate(&b->exec[from], b->graph[from], nullptr, nullptr, 0);
        if (e != hipSuccess) {
          drop_graphs(b);
          return hip_fail(c, e, "hipGraphInstantiate");
        }
      }
      b->captured_tuning = c->tuning;
    }
  }
  for (int32_t l = 0; l < n_levels; ++l) {
    const int from = b->cur;
    if (use_graph) {
      hipError_t e = hipGraphLaunch(b->exec[from], s);
      if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    } else {
      level_step(b, from, 1 - from);
      int rc = launch_status(c);
      if (rc) return rc;
    }
    b->cur = 1 - from;
    b->levels_run += 1;
    b->version += 1;
  }
  return HG_OK;
}

int hg_batch_done(hg_batch* b, int32_t* slots, int32_t cap, int32_t* n_done, int32_t* n_live) {
  if (!b || !n_done || (cap > 0 && !slots)) return HG_ERR_INVALID_ARG;
  hg_ctx* c = b->ctx;
  std::vector<GraphConst> h(b->max_graphs);
  hipError_t e = hipMemcpyAsync(h.data(), b->gc, sizeof(GraphConst) * b->max_graphs,
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "reading the batch graph states");
  int32_t n = 0, live = 0;
  for (int32_t g = 0; g < b->max_graphs; ++g) {
    if (b->slots[g].state != kLive) continue;
    if (h[g].done && n < cap) {
      slots[n++] = g;
      b->slots[g].state = kReported;
    } else {
      ++live;
    }
  }
  *n_done = n;
  if (n_live) *n_live = live;
  return HG_OK;
}

int hg_batch_result(hg_batch* b, int32_t g, int32_t* part, int32_t* n_parts, int32_t* n_levels) {
  if (!b || g < 0 || g >= b->max_graphs) return HG_ERR_INVALID_ARG;
  hg_ctx* c = b->ctx;
  SlotInfo& si = b->slots[g];
  if (si.state != kReported)
    return fail(c, HG_ERR_INVALID_ARG, "slot %d holds no finished graph (poll hg_batch_done)", g);
  if (si.v0 > 0 && !part) return fail(c, HG_ERR_INVALID_ARG, "part is null");
  std::vector<int32_t> vmn, vmx, emn, emx;
  int rc = read_ranges(b, vmn, vmx, emn, emx);
  if (rc) return rc;
  hipStream_t s = c->stream;
  int32_t lv = 0;
  hipError_t e = hipMemcpyAsync(&lv, b->nlev + g, 4, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(c, e, "reading the level count");
  if (si.v0 > 0)
    relative_kernel<<<blocks_for(si.v0), 256, 0, s>>>(b->part + si.pool_off, si.v0, vmn[g], part);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "reading the partition");
  if (n_parts) *n_parts = si.v0 > 0 ? vmx[g] - vmn[g] + 1 : 0;
  if (n_levels) *n_levels = lv;
  // release: the graph's vertices stay in the union (skipped) until compaction
  if (si.v0 > 0) fill_i32(b->owner + si.pool_off, -1, si.v0, s);
  si.state = kReleased;
  return launch_status(c);
}

int hg_batch_compact(hg_batch* b) {
  if (!b) return HG_ERR_INVALID_ARG;
  hg_ctx* c = b->ctx;
  hipStream_t s = c->stream;
  // graphs that stay: running and reported-but-unread ones
  b->alive_h.assign(b->max_graphs, 0);
  for (int32_t g = 0; g < b->max_graphs; ++g)
    b->alive_h[g] = (b->slots[g].state == kLive || b->slots[g].state == kReported) ? 1 : 0;
  hipError_t e = hipMemcpyAsync(b->c_alive, b->alive_h.data(), 4 * (size_t)b->max_graphs,
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "uploading the kept graphs");
  const LevelBuf& F = b->buf[b->cur];
  const LevelBuf& T = b->buf[1 - b->cur];
  const int64_t m = std::max(b->capV, b->capE);
  keep_marks_kernel<<<blocks_for(m), 256, 0, s>>>(F.dims, F.eoff, F.pins, F.gid, b->c_alive,
                                                  b->c_keepv, b->c_keepe, b->c_elen);
  exclusive_scan_i32(b->c_keepv, b->c_vpos, &F.dims->V, b->capV, b->c_partials, s);
  exclusive_scan_i32(b->c_keepe, b->c_epos, &F.dims->E, b->capE, b->c_partials, s);
  exclusive_scan_i32(b->c_elen, b->c_ppos, &F.dims->E, b->capE, b->c_partials, s);
  compact_vertices_kernel<<<blocks_for(b->capV), 256, 0, s>>>(
      F.dims, b->c_keepv, b->c_vpos, F.size, F.syn, F.ax, F.gid, T.size, T.syn, T.ax, T.gid);
  compact_edges_kernel<<<grid_for(b->capE, 4, 16384), 256, 0, s>>>(
      F.dims, F.eoff, F.pins, F.w, F.mult, b->c_keepe, b->c_epos, b->c_ppos, b->c_vpos, T.eoff,
      T.pins, T.w, T.mult);
  compact_finish_kernel<<<1, 1, 0, s>>>(F.dims, b->c_vpos, b->c_epos, b->c_ppos, T.eoff, T.dims);
  // the part pool keeps the unreleased graphs, in order, relabelled
  pool_marks_kernel<<<blocks_for(b->capV), 256, 0, s>>>(b->pool_n, b->owner, b->c_pkeep);
  exclusive_scan_i32(b->c_pkeep, b->c_pool, b->pool_n, b->capV, b->c_partials, s);
  pool_compact_kernel<<<blocks_for(b->capV), 256, 0, s>>>(b->pool_n, b->c_pkeep, b->c_pool,
                                                          b->c_vpos, b->part, b->owner,
                                                          b->part_tmp, b->owner_tmp);
  std::vector<int32_t> order;
  for (int32_t g = 0; g < b->max_graphs; ++g)
    if (b->alive_h[g]) order.push_back(g);
  std::sort(order.begin(), order.end(),
            [&](int32_t x, int32_t y) { return b->slots[x].pool_off < b->slots[y].pool_off; });
  int64_t pool = 0;
  for (int32_t g : order) {
    b->slots[g].pool_off = pool;
    pool += b->slots[g].v0;
  }
  if (pool > 0) {
    copy_kernel<int32_t><<<blocks_for(pool), 256, 0, s>>>(b->part_tmp, pool, b->part);
    copy_kernel<int32_t><<<blocks_for(pool), 256, 0, s>>>(b->owner_tmp, pool, b->owner);
  }
  if (b->pool_used > pool) fill_i32(b->owner + pool, -1, b->pool_used - pool, s);
  b->pool_used = pool;
  set_i64_kernel<<<1, 1, 0, s>>>(b->pool_n, pool);
  // released slots become free
  hg_limits none{0, 0, 0};
  for (int32_t g = 0; g < b->max_graphs; ++g)
    if (b->slots[g].state == kReleased) {
      set_slot_kernel<<<1, 1, 0, s>>>(b->gc, b->nlev, b->active, g, none, 1);
      b->slots[g] = SlotInfo{};
    }
  b->cur = 1 - b->cur;
  b->version += 1;
  int rc = launch_status(c);
  if (rc) return rc;
  // exact sizes again for admission
  Dims h;
  rc = read_dims(b, &h);
  if (rc) return rc;
  b->ubV = h.V;
  b->ubE = h.E;
  b->ubP = h.P;
  return HG_OK;
}

int hg_batch_sizes(hg_batch* b, int64_t* sizes) {
  if (!b || !sizes) return HG_ERR_INVALID_ARG;
  Dims h;
  int rc = read_dims(b, &h);
  if (rc) return rc;
  sizes[0] = h.V;
  sizes[1] = h.E;
  sizes[2] = h.P;
  sizes[3] = b->pool_used;
  b->ubV = h.V;  // exact again
  b->ubE = h.E;
  b->ubP = h.P;
  return HG_OK;
}

}  // extern "C"
