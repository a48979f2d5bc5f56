// Partitions across the hierarchy (paper, Section 4.1: when no candidate is
// proposed the final super-nodes form the initial partitions, and in the
// uncoarsening the super-nodes come undone level by level), and the
// evaluation of a partition of a level (Section 3: connectivity, Eq. 1, and
// the three per-core limits).
//
// hg_project      part_fine[v] = part_coarse[vmap[v]]: a partition of level
//                 l + 1 seen on level l.
// hg_partition_report
//                 Eq. 1 and the size, synapse and distinct-axon totals of
//                 every part.  The level is contracted with the partition as
//                 vertex map (the contraction of hg_contract): the coarse
//                 vertices are the parts, with their summed size and
//                 synapses and their distinct original axons (recomputed from
//                 the destination flags and the merge multiplicities), and
//                 Eq. 1 of the level under the partition equals the closed
//                 form sum of w(e) (|e| - 1) over the coarse hyperedges.
#include "hg_host.h"

namespace hg {
namespace {

__global__ void project_kernel(int64_t n, const int32_t* __restrict__ vmap,
                               const int32_t* __restrict__ n_coarse,
                               const int32_t* __restrict__ part_coarse,
                               int32_t* __restrict__ part_fine, int32_t* __restrict__ err) {
  const int64_t nc = *n_coarse;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = nc < 0;
  for (; i < n; i += stride) {
    const int32_t c = vmap[i];
    const bool ok = c >= 0 && (int64_t)c < nc;
    bad |= !ok;
    part_fine[i] = ok ? part_coarse[c] : 0;
  }
  if (bad) atomicOr(err, kErrMapRange);
}

// Over the contracted level: Eq. 1 as the closed form, and the totals of the
// parts against the limits.  summary: conn, max size, max synapses, max
// axons, parts over each of the three limits, number of parts.
__global__ void report_kernel(const Dims* __restrict__ od, const int64_t* __restrict__ eoff,
                              const int32_t* __restrict__ w, const int32_t* __restrict__ size,
                              const int32_t* __restrict__ syn, const int32_t* __restrict__ ax,
                              hg_limits lim, int64_t* __restrict__ summary,
                              int32_t* __restrict__ out_size, int32_t* __restrict__ out_syn,
                              int32_t* __restrict__ out_ax) {
  const int64_t E = od->E, V = od->V;
  const int lane = threadIdx.x & (kWave - 1);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t conn = 0;
  for (int64_t e = i; e < E; e += stride) conn += (int64_t)w[e] * (eoff[e + 1] - eoff[e] - 1);
  int64_t msz = 0, msy = 0, max_ = 0, o1 = 0, o2 = 0, o3 = 0;
  for (int64_t p = i; p < V; p += stride) {
    const int64_t a = size[p], b = syn[p], c = ax[p];
    msz = a > msz ? a : msz;
    msy = b > msy ? b : msy;
    max_ = c > max_ ? c : max_;
    o1 += a > lim.max_neurons;
    o2 += b > lim.max_synapses;
    o3 += c > lim.max_axons;
    if (out_size) out_size[p] = (int32_t)a;
    if (out_syn) out_syn[p] = (int32_t)b;
    if (out_ax) out_ax[p] = (int32_t)c;
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    conn += __shfl_xor(conn, d, kWave);
    const int64_t x = __shfl_xor(msz, d, kWave), y = __shfl_xor(msy, d, kWave),
                  z = __shfl_xor(max_, d, kWave);
    msz = x > msz ? x : msz;
    msy = y > msy ? y : msy;
    max_ = z > max_ ? z : max_;
    o1 += __shfl_xor(o1, d, kWave);
    o2 += __shfl_xor(o2, d, kWave);
    o3 += __shfl_xor(o3, d, kWave);
  }
  if (lane == 0) {
    atomicAdd((unsigned long long*)&summary[0], (unsigned long long)conn);
    atomicMax((unsigned long long*)&summary[1], (unsigned long long)msz);
    atomicMax((unsigned long long*)&summary[2], (unsigned long long)msy);
    atomicMax((unsigned long long*)&summary[3], (unsigned long long)max_);
    atomicAdd((unsigned long long*)&summary[4], (unsigned long long)o1);
    atomicAdd((unsigned long long*)&summary[5], (unsigned long long)o2);
    atomicAdd((unsigned long long*)&summary[6], (unsigned long long)o3);
  }
  if (i == 0) summary[7] = V;
}

__global__ void zero8_kernel(int64_t* __restrict__ p) {
  if (threadIdx.x < 8) p[threadIdx.x] = 0;
}

}  // namespace
}  // namespace hg

using namespace hg;

extern "C" {

int hg_project(hg_ctx* c, int32_t n_fine, const int32_t* vmap, const int32_t* n_coarse,
               const int32_t* part_coarse, int32_t* part_fine) {
  if (!c) return HG_ERR_INVALID_ARG;
  if (n_fine < 0) return fail(c, HG_ERR_INVALID_ARG, "negative vertex count");
  if (!n_coarse || (n_fine > 0 && (!vmap || !part_coarse || !part_fine)))
    return fail(c, HG_ERR_INVALID_ARG, "null argument");
  if (n_fine == 0) return HG_OK;
  project_kernel<<<grid_for(n_fine, 256, 8192), 256, 0, c->stream>>>(n_fine, vmap, n_coarse,
                                                                    part_coarse, part_fine,
                                                                    c->dev_err);
  return launch_status(c);
}

int hg_partition_report(hg_ctx* c, const hg_level* lvl, const int32_t* part,
                        const int32_t* n_parts, const hg_limits* lim, int64_t* summary,
                        int32_t* part_size, int32_t* part_syn, int32_t* part_axons) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_level(c, lvl, true);
  if (rc) return rc;
  if ((lvl->n_vertices > 0 && !part) || !n_parts || !lim || !summary)
    return fail(c, HG_ERR_INVALID_ARG, "null argument");
  if (c->validate && (rc = hg_validate_level(c, lvl)) != HG_OK) return rc;
  const int64_t V = lvl->n_vertices, E = lvl->n_edges, P = lvl->n_pins;
  auto carve = [&](auto& a, ContractLayout<std::decay_t<decltype(a)>>& S, int32_t*& map,
                   int32_t*& nc, hg_level_out& o) {
    S.carve(a, V, E, P);
    map = a.template take<int32_t>(V);
    nc = a.template take<int32_t>(1);
    o.cap_vertices = (int32_t)V;
    o.cap_edges = (int32_t)E;
    o.cap_pins = P;
    o.edge_offsets = a.template take<int64_t>(E + 1);
    o.pins = a.template take<uint32_t>(P);
    o.edge_weight = a.template take<int32_t>(E);
    o.edge_mult = a.template take<int32_t>(E);
    o.v_size = a.template take<int32_t>(V);
    o.v_syn = a.template take<int32_t>(V);
    o.v_axons = a.template take<int32_t>(V);
    o.sizes = a.template take<int64_t>(3);
  };
  Sizer sz;
  {
    ContractLayout<Sizer> S;
    int32_t *map, *nc;
    hg_level_out o;
    carve(sz, S, map, nc, o);
  }
  rc = ensure_arena(c, sz.off);
  if (rc) return rc;
  Carver cv{c->arena};
  ContractLayout<Carver> S;
  int32_t *map, *nc;
  hg_level_out o;
  carve(cv, S, map, nc, o);
  hipStream_t s = c->stream;
  set_dims(S.dims, V, E, P, s);
  LevelView L = view_of(lvl, S.dims);
  S.cs.err = c->dev_err;
  S.cs.fp_mask = c->fp_mask;
  check_map_kernel_launch(part, V, n_parts, map, nc, c->dev_err, s);
  contract_level(L, V, E, P, map, nc, &o, S.cs, s);
  zero8_kernel<<<1, 64, 0, s>>>(summary);
  const int64_t m = V > E ? V : E;
  report_kernel<<<grid_for(m, 256, 4096), 256, 0, s>>>(S.cs.out_dims, o.edge_offsets,
                                                       o.edge_weight, o.v_size, o.v_syn,
                                                       o.v_axons, *lim, summary, part_size,
                                                       part_syn, part_axons);
  return launch_status(c);
}

}  // extern "C"
