// Host-side pieces shared by the C ABI translation units: the context, the
// scratch carving, argument checks and the scratch layouts of the calls.
#pragma once

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <type_traits>

#include "hg_internal.h"

struct hg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int32_t* dev_err = nullptr;  // device error word (bounds reached by kernels)
  // small device block owned by the context: the error word, the weight sum
  // of the level check and the score-step census of the last level
  unsigned long long* dev_wsum = nullptr;
  int64_t* dev_census = nullptr;  // [2 * kNumBuckets]: vertices, visits
  bool timing = false;
  hipEvent_t ev[2 * HG_NUM_PHASES] = {};
  bool recorded[HG_NUM_PHASES] = {};
  hg::Tuning tuning;
  // switches read from the environment at hg_create
  bool validate = false;       // HG_VALIDATE=1: check every input level first
  size_t scratch_cap = 0;      // HG_SCRATCH_CAP=bytes: refuse a larger arena
  uint64_t fp_mask = ~0ull;    // HG_TEST_FP_BITS=n: keep n fingerprint bits
};

namespace hg {

// Bump allocator over the arena; every block 256-byte aligned.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(int64_t n) {
    size_t bytes = ((size_t)(n > 0 ? n : 1) * sizeof(T) + 255) & ~(size_t)255;
    T* p = reinterpret_cast<T*>(base + off);
    off += bytes;
    return p;
  }
};

// Sizing pass: same sequence of take() calls with a null base.
struct Sizer {
  size_t off = 0;
  template <typename T>
  T* take(int64_t n) {
    off += ((size_t)(n > 0 ? n : 1) * sizeof(T) + 255) & ~(size_t)255;
    return nullptr;
  }
};

inline int fail(hg_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
inline int fail(hg_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

inline int hip_fail(hg_ctx* c, hipError_t e, const char* what) {
  return fail(c, HG_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

inline int ensure_arena(hg_ctx* c, size_t bytes) {
  if (bytes <= c->arena_bytes) return HG_OK;
  if (c->scratch_cap && bytes > c->scratch_cap)
    return fail(c, HG_ERR_NO_MEMORY, "%zu bytes of scratch needed, above the cap of %zu", bytes,
                c->scratch_cap);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  if (c->arena) {
    (void)hipFree(c->arena);
    c->arena = nullptr;
    c->arena_bytes = 0;
  }
  size_t want = bytes + bytes / 8;
  if (c->scratch_cap && want > c->scratch_cap) want = c->scratch_cap;
  e = hipMalloc((void**)&c->arena, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->arena = nullptr;
    return fail(c, HG_ERR_NO_MEMORY, "cannot allocate %zu bytes of scratch", want);
  }
  c->arena_bytes = want;
  return HG_OK;
}

inline void mark(hg_ctx* c, int phase, int end) {
  if (!c->timing) return;
  (void)hipEventRecord(c->ev[2 * phase + end], c->stream);
  if (end) c->recorded[phase] = true;
}

inline int launch_status(hg_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return HG_OK;
}

inline int check_level(hg_ctx* c, const hg_level* L, bool need_state) {
  if (!L) return fail(c, HG_ERR_INVALID_ARG, "level is null");
  if (L->n_vertices < 0 || L->n_edges < 0 || L->n_pins < 0)
    return fail(c, HG_ERR_INVALID_ARG, "negative level size");
  if (L->n_vertices > 0x7FFFFFFE) return fail(c, HG_ERR_OVERFLOW, "too many vertices");
  if (L->n_pins > 0x7FFFFFFF) return fail(c, HG_ERR_OVERFLOW, "2^31 or more pins");
  if (!L->edge_offsets) return fail(c, HG_ERR_INVALID_ARG, "edge_offsets is null");
  if (L->n_pins > 0 && !L->pins) return fail(c, HG_ERR_INVALID_ARG, "pins is null");
  if (L->n_edges > 0 && !L->edge_weight) return fail(c, HG_ERR_INVALID_ARG, "edge_weight is null");
  if (need_state) {
    if (L->n_edges > 0 && !L->edge_mult) return fail(c, HG_ERR_INVALID_ARG, "edge_mult is null");
    if (L->n_vertices > 0 && (!L->v_size || !L->v_syn || !L->v_axons))
      return fail(c, HG_ERR_INVALID_ARG, "vertex state is null");
  }
  return HG_OK;
}

inline LevelView view_of(const hg_level* L, const Dims* d) {
  return LevelView{d, L->edge_offsets, L->pins, L->edge_weight, L->edge_mult,
                   L->v_size, L->v_syn, L->v_axons, nullptr};
}

// ---- scratch layouts -------------------------------------------------------
template <typename A>
struct CoarsenScratch {
  Dims* dims;
  GraphConst* gc;
  int32_t* vcount;
  int64_t* voff;
  uint32_t* vinc;
  int64_t* xn;
  int32_t* bcount;
  int32_t* blist;
  int64_t* bvisits;
  int32_t* work;
  int32_t* cursor;
  int32_t* cand;
  int32_t* cscore;
  uint64_t* bkey;
  uint32_t* jump;
  int32_t* flags;
  int32_t* rep;
  int64_t* rank;
  int64_t* partials;
  uint32_t* splits;
  int32_t n_win;
  uint32_t* splits14;
  int32_t n_win14;
  IncScratch inc;  // its pairs alias `cursor`, which the score step uses later
  void carve(A& a, int64_t V, int64_t E, int64_t P) {
    dims = a.template take<Dims>(1);
    gc = a.template take<GraphConst>(1);
    vcount = a.template take<int32_t>(V);
    voff = a.template take<int64_t>(V + 1);
    vinc = a.template take<uint32_t>(P);
    xn = a.template take<int64_t>(V);
    bcount = a.template take<int32_t>(kNumBuckets);
    blist = a.template take<int32_t>(kNumBuckets * V);
    bvisits = a.template take<int64_t>(kNumBuckets);
    work = a.template take<int32_t>(kNumBuckets);
    cursor = a.template take<int32_t>(2 * P);
    inc = incidence_scratch_carve(a, V, P, reinterpret_cast<uint64_t*>(cursor));
    cand = a.template take<int32_t>(V);
    cscore = a.template take<int32_t>(V);
    bkey = a.template take<uint64_t>(V);
    jump = a.template take<uint32_t>(V);
    flags = a.template take<int32_t>(32);
    rep = a.template take<int32_t>(V);
    rank = a.template take<int64_t>(V + 1);
    partials = a.template take<int64_t>(scan_partials_size());
    const int64_t w = (V + (1ll << kWinAlignBits) - 1) >> kWinAlignBits;
    n_win = (w >= 1 && w <= kMaxAlignedWindows) ? (int32_t)w : 0;
    splits = n_win ? a.template take<uint32_t>(E * (n_win + 1)) : nullptr;
    const int64_t w14 = (V + (1ll << kDenseBits) - 1) >> kDenseBits;
    n_win14 = (w14 >= 1 && w14 <= kMaxDenseWindows) ? (int32_t)w14 : 0;
    splits14 = n_win14 ? a.template take<uint32_t>(E * (n_win14 + 1)) : nullptr;
  }
};

inline int64_t pow2_at_least(int64_t x) {
  int64_t c = 64;
  while (c < x) c <<= 1;
  return c;
}

template <typename A>
struct ContractLayout {
  Dims* dims;
  ContractScratch cs;
  void carve(A& a, int64_t V, int64_t E, int64_t P) {
    dims = a.template take<Dims>(1);
    cs.out_dims = a.template take<Dims>(1);
    cs.dstmult = a.template take<int32_t>(V);
    cs.tpin = a.template take<uint32_t>(P);
    cs.tlen = a.template take<int32_t>(E);
    cs.fp = a.template take<uint64_t>(E);
    cs.ebucket = a.template take<int32_t>(4 * E);
    cs.ecount = a.template take<int32_t>(8);
    cs.work = a.template take<int32_t>(4);
    cs.htab_cap = pow2_at_least(2 * E);
    cs.htab_key = a.template take<uint64_t>(cs.htab_cap);
    cs.htab_lead = a.template take<int32_t>(cs.htab_cap);
    cs.slot = a.template take<int32_t>(E);
    cs.group = a.template take<int32_t>(E);
    cs.mism = a.template take<int32_t>(E);
    cs.lflag = a.template take<int32_t>(E);
    cs.lrank = a.template take<int64_t>(E + 1);
    cs.leader_at = a.template take<int32_t>(E);
    cs.llen = a.template take<int64_t>(E);
    cs.partials = a.template take<int64_t>(scan_partials_size());
    cs.bitmap_words = (V + 31) / 32 + 1;
    cs.bitmap = a.template take<uint32_t>((int64_t)kHugeWG * 2 * cs.bitmap_words);
    uint64_t* pairs = P >= kIncMinPins ? a.template take<uint64_t>(P) : nullptr;
    cs.inc = incidence_scratch_carve(a, V, P, pairs);
  }
};

template <typename A>
struct ConnLayout {
  Dims* dims;
  ConnScratch cs;
  void carve(A& a, int64_t V, int64_t E) {
    dims = a.template take<Dims>(1);
    cs.ebucket = a.template take<int32_t>(4 * E);
    cs.ecount = a.template take<int32_t>(4);
    cs.work = a.template take<int32_t>(4);
    cs.bitmap_words = (V + 31) / 32 + 1;
    cs.bitmap = a.template take<uint32_t>((int64_t)kHugeWG * cs.bitmap_words);
  }
};

inline size_t connectivity_scratch_bytes(int64_t V, int64_t E) {
  Sizer sz;
  ConnLayout<Sizer> ls;
  ls.carve(sz, V, E);
  sz.take<int32_t>(V);  // checked copy of the partition
  return sz.off;
}

inline size_t validate_scratch_bytes() {
  Sizer sz;
  sz.take<unsigned long long>(1);
  sz.take<int32_t>(1);
  return sz.off;
}

// Bodies of hg_connectivity and hg_validate_level over a given scratch base
// (the context's arena, or the library's fixed scratch).
int run_connectivity(hg_ctx* c, const hg_level* lvl, const int32_t* part, int64_t* conn,
                     char* base);
int validate_with(hg_ctx* c, const hg_level* L, char* base);
// Checked copy of a caller's map (values in [0, *n_range), see hg_contract).
void check_map_kernel_launch(const int32_t* in, int64_t V, const int32_t* n_range,
                             int32_t* out, int32_t* out_range, int32_t* err, hipStream_t s);

// The library's fixed device scratch (hg_static.hip): its address on the
// current device is looked up once per device by hg_create.
int static_scratch_setup(int device);
}  // namespace hg
