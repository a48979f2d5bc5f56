// C ABI entry points: context, scratch arena, argument checks, dispatch.
#include <stdlib.h>

#include <new>

#include "hg_host.h"

namespace hg {
namespace {

__global__ void set_graph_const_kernel(GraphConst* gc, hg_limits lim) {
  gc->omega = lim.max_neurons;
  gc->phi = lim.max_synapses;
  gc->delta = lim.max_axons;
  gc->max_size = gc->max_syn = gc->max_ax = 0;
  gc->nverts = 0;
  gc->done = 0;
}

// ---- validation kernel -----------------------------------------------------
__global__ void validate_kernel(LevelView L, int64_t V, int64_t E, int64_t P,
                                unsigned long long* wsum, int32_t* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (i == 0 && (L.eoff[0] != 0 || L.eoff[E] != P)) atomicOr(bad, 1);
  for (int64_t e = i; e < E; e += stride) {
    int64_t s = L.eoff[e], t = L.eoff[e + 1];
    if (t < s || s < 0 || t > P) {
      atomicOr(bad, 1);
      continue;
    }
    if (L.w[e] < 1) atomicOr(bad, 4);
    if (L.mult && L.mult[e] < 1) atomicOr(bad, 4);
    atomicAdd(wsum, (unsigned long long)(L.w[e] > 0 ? L.w[e] : 0));
    uint32_t prev = 0;
    for (int64_t k = s; k < t; ++k) {
      uint32_t id = L.pins[k] & kIdMask;
      if ((int64_t)id >= V) atomicOr(bad, 2);
      if (k > s && id <= prev) atomicOr(bad, 2);
      prev = id;
    }
  }
  for (int64_t v = i; v < V; v += stride) {
    if (L.size && (L.size[v] < 1)) atomicOr(bad, 8);
    if (L.syn && L.syn[v] < 0) atomicOr(bad, 8);
    if (L.ax && L.ax[v] < 0) atomicOr(bad, 8);
  }
}

// Weights of a level (Section 2 model: spike rates, integers >= 1 here) and
// their sum, which must stay below 2^31 so that every score and every merged
// weight fits an int32 (the score step packs scores next to ids).  Runs on
// the device before the scores; a violation is recorded in the error word
// and reported by hg_sync.
__global__ void weight_check_kernel(const Dims* __restrict__ d, const int32_t* __restrict__ w,
                                    unsigned long long* __restrict__ wsum,
                                    int32_t* __restrict__ err) {
  const int64_t E = d->E;
  const int lane = threadIdx.x & (kWave - 1);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long acc = 0;
  bool bad = false;
  for (; i < E; i += stride) {
    const int32_t x = w[i];
    bad |= x < 1;
    acc += (unsigned long long)(x > 0 ? x : 0);
  }
#pragma unroll
  for (int k = kWave / 2; k > 0; k >>= 1) acc += __shfl_xor(acc, k, kWave);
  if (lane == 0 && acc) atomicAdd(wsum, acc);
  if (bad) atomicOr(err, kErrWeight);
}

__global__ void weight_sum_kernel(unsigned long long* __restrict__ wsum,
                                  int32_t* __restrict__ err) {
  if (*wsum >= (1ull << 31)) atomicOr(err, kErrWeightSum);
  *wsum = 0;
}

// Keeps the score step's census (vertices and neighbour visits per work
// list) of the last level in the context's own memory.
__global__ void census_kernel(const int32_t* __restrict__ count,
                              const int64_t* __restrict__ visits, int64_t* __restrict__ out) {
  const int k = threadIdx.x;
  if (k < kNumBuckets) {
    out[k] = count[k];
    out[kNumBuckets + k] = visits[k];
  }
}

// Checked copy of a map supplied by the caller (vmap of hg_contract, part of
// hg_connectivity).  The range is [0, bound) with bound = *n_range clamped to
// [min(1, V), V] (or V when n_range is null); a value outside it becomes 0 in
// the copy, a bound outside that interval is clamped, and either is recorded
// in the error word.  Every kernel after this one indexes with the copy, so
// no input can send a write outside the arrays sized from V.
__global__ void check_map_kernel(const int32_t* __restrict__ in, int64_t V,
                                 const int32_t* __restrict__ n_range, int32_t* __restrict__ out,
                                 int32_t* __restrict__ out_range, int32_t* __restrict__ err) {
  int64_t bound = V;
  bool bad_bound = false;
  if (n_range) {
    const int64_t r = *n_range;
    const int64_t lo = V > 0 ? 1 : 0;
    bad_bound = r < 0 || r > V;
    bound = r < lo ? lo : (r > V ? V : r);
  }
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    if (out_range) *out_range = (int32_t)bound;
    if (bad_bound) atomicOr(err, kErrMapRange);
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (; i < V; i += stride) {
    const int32_t x = in[i];
    const bool ok = (uint32_t)x < (uint64_t)bound;
    bad |= !ok;
    out[i] = ok ? x : 0;
  }
  if (bad) atomicOr(err, kErrMapRange);
}

}  // namespace
}  // namespace hg

using namespace hg;

extern "C" {

int hg_create(int device, void* hip_stream, hg_ctx** out) {
  if (!out) return HG_ERR_INVALID_ARG;
  *out = nullptr;
  hg_ctx* c = new (std::nothrow) hg_ctx();
  if (!c) return HG_ERR_NO_MEMORY;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (const char* v = getenv("HG_VALIDATE")) c->validate = atoi(v) != 0;
  if (const char* v = getenv("HG_SCRATCH_CAP")) c->scratch_cap = (size_t)strtoull(v, nullptr, 10);
  if (const char* v = getenv("HG_TEST_FP_BITS")) {
    const int bits = atoi(v);
    if (bits >= 1 && bits < 64) c->fp_mask = (1ull << bits) - 1;
  }
  hipError_t e = hipSetDevice(device);
  char* blk = nullptr;
  if (e == hipSuccess) e = hipMalloc((void**)&blk, 1024);
  if (e != hipSuccess) {
    delete c;
    return HG_ERR_HIP;
  }
  // the fixed scratch of hg_connectivity_static, once per device (the
  // device is current here); a failure only disables that call
  (void)static_scratch_setup(device);
  c->dev_err = reinterpret_cast<int32_t*>(blk);
  c->dev_wsum = reinterpret_cast<unsigned long long*>(blk + 64);
  c->dev_census = reinterpret_cast<int64_t*>(blk + 128);
  fill_i32(c->dev_err, 0, 1, c->stream);
  fill_u64((uint64_t*)c->dev_wsum, 0, 1, c->stream);
  fill_i64(c->dev_census, 0, 2 * kNumBuckets, c->stream);
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    (void)hipFree(c->dev_err);
    delete c;
    return HG_ERR_HIP;
  }
  *out = c;
  return HG_OK;
}

int hg_destroy(hg_ctx* c) {
  if (!c) return HG_OK;
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->arena) (void)hipFree(c->arena);
  if (c->dev_err) (void)hipFree(c->dev_err);
  delete c;
  return HG_OK;
}

int hg_set_stream(hg_ctx* c, void* hip_stream) {
  if (!c) return HG_ERR_INVALID_ARG;
  c->stream = (hipStream_t)hip_stream;
  return HG_OK;
}

const char* hg_last_error(hg_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

int hg_sync(hg_ctx* c) {
  if (!c) return HG_ERR_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  int32_t flags = 0;
  e = hipMemcpy(&flags, c->dev_err, sizeof flags, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "error word read-back");
  if (flags) {
    fill_i32(c->dev_err, 0, 1, c->stream);
    (void)hipStreamSynchronize(c->stream);
    if (flags & kErrMapRange)
      return fail(c, HG_ERR_INVALID_ARG,
                  "a vmap or part value, or n_coarse, was outside its range; the outputs of "
                  "that call are undefined (flags 0x%x)",
                  flags);
    if (flags & kErrPlacement)
      return fail(c, HG_ERR_INVALID_ARG,
                  "a starting order that is not a permutation of the nodes, or a placement "
                  "that is not one node per core of the lattice; the outputs of that call are "
                  "undefined (flags 0x%x)",
                  flags);
    if (flags & kErrWeight)
      return fail(c, HG_ERR_INVALID_LEVEL,
                  "a hyperedge weight below 1; the outputs of that call are undefined "
                  "(flags 0x%x)",
                  flags);
    if (flags & kErrWeightSum)
      return fail(c, HG_ERR_OVERFLOW,
                  "the hyperedge weights of a level sum to 2^31 or more; the outputs of that "
                  "call are undefined (flags 0x%x)",
                  flags);
    return fail(c, HG_ERR_INTERNAL,
                "a kernel reached an internal bound (flags 0x%x: 1 score table, 2 passes, "
                "4 distinct set, 8 fingerprint table, 16 work count, 32 list length)",
                flags);
  }
  return HG_OK;
}

int64_t hg_scratch_bytes(hg_ctx* c) { return c ? (int64_t)c->arena_bytes : 0; }

int hg_set_tuning(hg_ctx* c, const hg_tuning* t) {
  if (!c || !t) return HG_ERR_INVALID_ARG;
  if (t->single_pass_load16 < 1 || t->single_pass_load16 > 12)
    return fail(c, HG_ERR_INVALID_ARG, "single_pass_load16 %d outside 1..12",
                t->single_pass_load16);
  if (t->pass_fill16 < 1 || t->pass_fill16 > 10)
    return fail(c, HG_ERR_INVALID_ARG, "pass_fill16 %d outside 1..10", t->pass_fill16);
  if (t->dense_ratio < 0 || t->dense_ratio > 64)
    return fail(c, HG_ERR_INVALID_ARG, "dense_ratio %d outside 0..64", t->dense_ratio);
  if (t->wide_loads < 0 || t->wide_loads > 1)
    return fail(c, HG_ERR_INVALID_ARG, "wide_loads %d outside 0..1", t->wide_loads);
  c->tuning.load16 = t->single_pass_load16;
  c->tuning.fill16 = t->pass_fill16;
  c->tuning.dense_ratio = t->dense_ratio;
  c->tuning.wide = t->wide_loads;
  return HG_OK;
}

int hg_get_tuning(hg_ctx* c, hg_tuning* t) {
  if (!c || !t) return HG_ERR_INVALID_ARG;
  t->single_pass_load16 = c->tuning.load16;
  t->pass_fill16 = c->tuning.fill16;
  t->dense_ratio = c->tuning.dense_ratio;
  t->wide_loads = c->tuning.wide;
  return HG_OK;
}

int hg_enable_timing(hg_ctx* c, int on) {
  if (!c) return HG_ERR_INVALID_ARG;
  if (on && !c->ev[0]) {
    for (auto& e : c->ev) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return hip_fail(c, r, "hipEventCreate");
    }
  }
  c->timing = on != 0;
  for (bool& r : c->recorded) r = false;
  return HG_OK;
}

int hg_phase_times(hg_ctx* c, float* ms) {
  if (!c || !ms) return HG_ERR_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  for (int p = 0; p < HG_NUM_PHASES; ++p) {
    ms[p] = 0.0f;
    if (c->timing && c->recorded[p]) {
      e = hipEventElapsedTime(&ms[p], c->ev[2 * p], c->ev[2 * p + 1]);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
    }
    c->recorded[p] = false;
  }
  return HG_OK;
}

int hg_init_state(hg_ctx* c, int32_t V, int32_t E, int64_t P, const int64_t* eoff,
                  const uint32_t* pins, int32_t* size, int32_t* syn, int32_t* ax,
                  int32_t* mult) {
  if (!c) return HG_ERR_INVALID_ARG;
  if (V < 0 || E < 0 || P < 0) return fail(c, HG_ERR_INVALID_ARG, "negative size");
  if (!eoff || (P > 0 && !pins) || (V > 0 && (!size || !syn || !ax)) || (E > 0 && !mult))
    return fail(c, HG_ERR_INVALID_ARG, "null pointer");
  Sizer sz;
  sz.take<Dims>(1);
  int rc = ensure_arena(c, sz.off);
  if (rc) return rc;
  Carver cv{c->arena};
  Dims* d = cv.take<Dims>(1);
  set_dims(d, V, E, P, c->stream);
  level0_state(d, eoff, pins, V, E, size, syn, ax, mult, c->stream);
  return launch_status(c);
}

int hg_coarsen_level(hg_ctx* c, const hg_level* in, const hg_limits* lim, int32_t* cand,
                     int32_t* cscore, int32_t* match, int32_t* vmap, int32_t* n_coarse,
                     int32_t* any_candidate) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_level(c, in, true);
  if (rc) return rc;
  if (!lim || lim->max_neurons < 0 || lim->max_synapses < 0 || lim->max_axons < 0)
    return fail(c, HG_ERR_INVALID_ARG, "bad limits");
  if ((in->n_vertices > 0 && (!match || !vmap)) || !n_coarse || !any_candidate)
    return fail(c, HG_ERR_INVALID_ARG, "null output");
  if (c->validate && (rc = hg_validate_level(c, in)) != HG_OK) return rc;
  const int64_t V = in->n_vertices, E = in->n_edges, P = in->n_pins;
  Sizer sz;
  CoarsenScratch<Sizer> ls;
  ls.carve(sz, V, E, P);
  rc = ensure_arena(c, sz.off);
  if (rc) return rc;
  Carver cv{c->arena};
  CoarsenScratch<Carver> S;
  S.carve(cv, V, E, P);
  hipStream_t s = c->stream;
  set_dims(S.dims, V, E, P, s);
  set_graph_const_kernel<<<1, 1, 0, s>>>(S.gc, *lim);
  LevelView L = view_of(in, S.dims);
  // S0, S1
  mark(c, 0, 0);
  weight_check_kernel<<<grid_for(E, 256 * 8, 1024), 256, 0, s>>>(S.dims, in->edge_weight,
                                                                  c->dev_wsum, c->dev_err);
  weight_sum_kernel<<<1, 1, 0, s>>>(c->dev_wsum, c->dev_err);
  build_incidence(L, V, E, P, S.vcount, S.voff, S.vinc, S.partials, s, S.inc);
  Buckets b{S.bcount, S.blist, S.bvisits};
  expansion_and_buckets(L, S.voff, S.vinc, V, S.xn, S.gc, 1, b, c->tuning, s, S.n_win14);
  census_kernel<<<1, 64, 0, s>>>(S.bcount, S.bvisits, c->dev_census);
  mark(c, 0, 1);
  // S2
  int32_t* cd = cand ? cand : S.cand;
  int32_t* cs = cscore ? cscore : S.cscore;
  ScoreArgs sa{L,  S.voff, S.vinc, S.xn, S.gc, S.cursor, cd,
               cs, S.work, b,      c->dev_err, c->tuning.fill16};
  sa.splits = S.splits;
  sa.n_win = S.n_win;
  sa.splits14 = S.splits14;
  sa.n_win14 = S.n_win14;
  sa.wide = c->tuning.wide;
  mark(c, 1, 0);
  score_candidates(sa, V, P, s);
  mark(c, 1, 1);
  // S3-S5
  MatchArgs ma{S.dims, cd, cs, S.bkey, S.jump, S.jump, S.flags, match, vmap, S.rep, S.rank,
               S.partials, n_coarse, any_candidate};
  mark(c, 2, 0);
  match_and_vmap(ma, V, s);
  mark(c, 2, 1);
  return launch_status(c);
}

int hg_contract(hg_ctx* c, const hg_level* in, const int32_t* vmap, const int32_t* n_coarse,
                hg_level_out* out) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_level(c, in, true);
  if (rc) return rc;
  if ((in->n_vertices > 0 && !vmap) || !n_coarse || !out)
    return fail(c, HG_ERR_INVALID_ARG, "null argument");
  if (!out->edge_offsets || !out->pins || !out->edge_weight || !out->edge_mult ||
      !out->v_size || !out->v_syn || !out->v_axons || !out->sizes)
    return fail(c, HG_ERR_INVALID_ARG, "null output array");
  const int64_t V = in->n_vertices, E = in->n_edges, P = in->n_pins;
  if (out->cap_vertices < V || out->cap_edges < E || out->cap_pins < P)
    return fail(c, HG_ERR_CAPACITY, "output capacities (%d, %d, %lld) below input sizes",
                out->cap_vertices, out->cap_edges, (long long)out->cap_pins);
  if (c->validate && (rc = hg_validate_level(c, in)) != HG_OK) return rc;
  Sizer sz;
  ContractLayout<Sizer> ls;
  ls.carve(sz, V, E, P);
  sz.take<int32_t>(V);
  sz.take<int32_t>(1);
  rc = ensure_arena(c, sz.off);
  if (rc) return rc;
  Carver cv{c->arena};
  ContractLayout<Carver> S;
  S.carve(cv, V, E, P);
  int32_t* map = cv.take<int32_t>(V);
  int32_t* nc = cv.take<int32_t>(1);
  hipStream_t s = c->stream;
  set_dims(S.dims, V, E, P, s);
  LevelView L = view_of(in, S.dims);
  S.cs.err = c->dev_err;
  S.cs.fp_mask = c->fp_mask;
  mark(c, 3, 0);
  weight_check_kernel<<<grid_for(E, 256 * 8, 1024), 256, 0, s>>>(S.dims, in->edge_weight,
                                                                  c->dev_wsum, c->dev_err);
  weight_sum_kernel<<<1, 1, 0, s>>>(c->dev_wsum, c->dev_err);
  check_map_kernel<<<grid_for(V, 256, 4096), 256, 0, s>>>(vmap, V, n_coarse, map, nc,
                                                        c->dev_err);
  contract_level(L, V, E, P, map, nc, out, S.cs, s);
  mark(c, 3, 1);
  return launch_status(c);
}

int hg_connectivity(hg_ctx* c, const hg_level* lvl, const int32_t* part, int64_t* conn) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_level(c, lvl, false);
  if (rc) return rc;
  if ((lvl->n_vertices > 0 && !part) || !conn) return fail(c, HG_ERR_INVALID_ARG, "null argument");
  if (c->validate && (rc = hg_validate_level(c, lvl)) != HG_OK) return rc;
  rc = ensure_arena(c, connectivity_scratch_bytes(lvl->n_vertices, lvl->n_edges));
  if (rc) return rc;
  return run_connectivity(c, lvl, part, conn, c->arena);
}

int hg_score_census(hg_ctx* c, int64_t* out) {
  if (!c || !out) return HG_ERR_INVALID_ARG;
  hipError_t e = hipMemcpyAsync(out, c->dev_census, 2 * kNumBuckets * sizeof(int64_t),
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "census read-back");
  return HG_OK;
}

int hg_validate_level(hg_ctx* c, const hg_level* L) {
  if (!c) return HG_ERR_INVALID_ARG;
  int rc = check_level(c, L, false);
  if (rc) return rc;
  rc = ensure_arena(c, validate_scratch_bytes());
  if (rc) return rc;
  return validate_with(c, L, c->arena);
}

}  // extern "C"

namespace hg {

void check_map_kernel_launch(const int32_t* in, int64_t V, const int32_t* n_range,
                             int32_t* out, int32_t* out_range, int32_t* err, hipStream_t s) {
  check_map_kernel<<<grid_for(V, 256, 4096), 256, 0, s>>>(in, V, n_range, out, out_range, err);
}

int run_connectivity(hg_ctx* c, const hg_level* lvl, const int32_t* part, int64_t* conn,
                     char* base) {
  const int64_t V = lvl->n_vertices, E = lvl->n_edges, P = lvl->n_pins;
  Carver cv{base};
  ConnLayout<Carver> S;
  S.carve(cv, V, E);
  int32_t* map = cv.take<int32_t>(V);
  hipStream_t s = c->stream;
  set_dims(S.dims, V, E, P, s);
  LevelView L = view_of(lvl, S.dims);
  S.cs.err = c->dev_err;
  mark(c, 4, 0);
  check_map_kernel<<<grid_for(V, 256, 4096), 256, 0, s>>>(part, V, nullptr, map, nullptr,
                                                        c->dev_err);
  connectivity(L, E, V, map, conn, S.cs, s);
  mark(c, 4, 1);
  return launch_status(c);
}

int validate_with(hg_ctx* c, const hg_level* L, char* base) {
  Carver cv{base};
  unsigned long long* wsum = cv.take<unsigned long long>(1);
  int32_t* bad = cv.take<int32_t>(1);
  hipStream_t s = c->stream;
  fill_u64((uint64_t*)wsum, 0, 1, s);
  fill_i32(bad, 0, 1, s);
  LevelView lv{nullptr, L->edge_offsets, L->pins, L->edge_weight, L->edge_mult,
               L->v_size, L->v_syn, L->v_axons, nullptr};
  validate_kernel<<<grid_for(L->n_edges > L->n_vertices ? L->n_edges : L->n_vertices, 256, 4096),
                    256, 0, s>>>(lv, L->n_vertices, L->n_edges, L->n_pins, wsum, bad);
  int rc = launch_status(c);
  if (rc) return rc;
  unsigned long long hw = 0;
  int32_t hb = 0;
  hipError_t e = hipMemcpyAsync(&hw, wsum, sizeof hw, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof hb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "validate read-back");
  if (hb) return fail(c, HG_ERR_INVALID_LEVEL, "malformed level (flags 0x%x)", hb);
  if (hw >= (1ull << 31)) return fail(c, HG_ERR_OVERFLOW, "total weight %llu >= 2^31", hw);
  return HG_OK;
}

}  // namespace hg
