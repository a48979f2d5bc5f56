// CPU oracle for one coarsening level of an SNN hypergraph and for the
// (lambda - 1) connectivity objective.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
// GPU library is checked against.  Only the test-suite, the smoke check and
// the CPU-baseline leg of the benchmark may load it; the product path never
// does.  It shares no code with the GPU library.
//
// Everything is integer arithmetic.  Each function follows one passage of
// Ronzani & Silvano, "GPU-Accelerated Hypergraph Partitioning and Placement to
// Map SNNs on Neuromorphic Hardware":
//
//   * level-0 model ............ Section 2, "SNN and Hardware Models"
//   * constraints .............. Section 3, "Partitioning Definition"
//                                (|p| <= Omega, |U in(n)| <= Delta,
//                                 sum |in(n)| <= Phi)
//   * score / candidate ........ Section 4.1, "Coarsening", Eq. (12)
//   * matching ................. Section 4.1, "Coarsening", Eq. (13)
//   * coarse hypergraph ........ Section 3, "Partitioning Definition" (G_P),
//                                and Section 4.1 (state propagated per level)
//   * connectivity ............. Section 3, Eq. (1)
//
// Readings of passages the paper leaves open (also listed in the design notes):
//   R1 ties in every argmax go to the lowest vertex id;
//   R2 a super-node's inbound set is the set of ORIGINAL axons with at least
//      one destination inside it; it is propagated as an explicit set, the
//      way the paper propagates "size, inbound hyperedges set, and pin count";
//   R3 pins of a coarse hyperedge carry a destination flag (set iff the
//      super-node holds a destination of one of its axons); coarse hyperedges
//      are merged only when their (vertex, flag) lists are identical, and the
//      number of merged original axons is carried as `mult`;
//   R4 coarse hyperedges with fewer than two distinct pins are dropped;
//   R5 coarse vertices are numbered by their smallest member, coarse
//      hyperedges by their smallest fine hyperedge, pins ascending;
//   R6 Eq. (13)'s first case takes precedence over its second;
//   R7 the level loop stops when no vertex proposes a candidate.
//
// Plainness is the point: per-vertex dense score arrays, std::map for
// grouping, explicit sets for inbound axons.  The only parallelism is an
// OpenMP loop over vertices in the candidate step.
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const uint32_t DST = 0x80000000u;
const uint32_t IDMASK = 0x7FFFFFFFu;

// Incidence lists I(n) = in(n) U out(n) (Section 2): for every vertex the
// hyperedges that contain it, as (edge, is_destination) pairs.
struct Incidence {
  std::vector<int64_t> off;
  std::vector<int32_t> edge;
  std::vector<uint8_t> is_dst;
};

Incidence build_incidence(int32_t V, int32_t E, const int64_t* eoff,
                          const uint32_t* pins) {
  Incidence inc;
  inc.off.assign((size_t)V + 1, 0);
  for (int32_t e = 0; e < E; ++e)
    for (int64_t k = eoff[e]; k < eoff[e + 1]; ++k) inc.off[(pins[k] & IDMASK) + 1]++;
  for (int32_t v = 0; v < V; ++v) inc.off[v + 1] += inc.off[v];
  inc.edge.resize(inc.off[V]);
  inc.is_dst.resize(inc.off[V]);
  std::vector<int64_t> pos(inc.off.begin(), inc.off.end() - 1);
  for (int32_t e = 0; e < E; ++e)
    for (int64_t k = eoff[e]; k < eoff[e + 1]; ++k) {
      uint32_t v = pins[k] & IDMASK;
      inc.edge[pos[v]] = e;
      inc.is_dst[pos[v]] = (pins[k] & DST) ? 1 : 0;
      pos[v]++;
    }
  return inc;
}

// |A n B| for two ascending id lists.
int64_t intersect_count(const int32_t* a, int64_t na, const int32_t* b, int64_t nb) {
  int64_t i = 0, j = 0, c = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) ++i;
    else if (b[j] < a[i]) ++j;
    else { ++c; ++i; ++j; }
  }
  return c;
}

struct Limits {
  int32_t omega, phi, delta;
};

struct Level {
  int32_t V, E;
  const int64_t* eoff;
  const uint32_t* pins;
  const int32_t* w;
  const int32_t* size;
  const int32_t* syn;
  const int64_t* soff;   // inbound-axon sets, CSR over vertices
  const int32_t* sids;
};

// Merge constraint check between super-nodes n and m (Section 3 constraints
// applied to the union n U m; R2 for the inbound set).
bool merge_valid(const Level& L, const Limits& lim, int32_t n, int32_t m) {
  if ((int64_t)L.size[n] + L.size[m] > lim.omega) return false;
  if ((int64_t)L.syn[n] + L.syn[m] > lim.phi) return false;
  int64_t an = L.soff[n + 1] - L.soff[n];
  int64_t am = L.soff[m + 1] - L.soff[m];
  if (an + am <= lim.delta) return true;  // |A U B| <= |A| + |B|
  int64_t ov = intersect_count(L.sids + L.soff[n], an, L.sids + L.soff[m], am);
  return an + am - ov <= lim.delta;
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Level-0 state (Section 2 model; Section 3 constraint quantities).
// size = 1 neuron; syn = |in(n)| inbound pins; inbound set = in(n), the axons
// that have n as a destination; every hyperedge stands for one axon (mult 1).
// soff must hold V+1 entries; sids as many entries as there are destination
// pins.  Returns 0.
int oracle_level0_state(int32_t V, int32_t E, const int64_t* eoff, const uint32_t* pins,
                        int32_t* size, int32_t* syn, int32_t* mult, int64_t* soff,
                        int32_t* sids) {
  std::vector<std::vector<int32_t>> in(V);
  for (int32_t e = 0; e < E; ++e) {
    mult[e] = 1;
    for (int64_t k = eoff[e]; k < eoff[e + 1]; ++k)
      if (pins[k] & DST) in[pins[k] & IDMASK].push_back(e);
  }
  soff[0] = 0;
  for (int32_t v = 0; v < V; ++v) {
    size[v] = 1;
    syn[v] = (int32_t)in[v].size();
    std::sort(in[v].begin(), in[v].end());
    soff[v + 1] = soff[v] + (int64_t)in[v].size();
    std::copy(in[v].begin(), in[v].end(), sids + soff[v]);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Score and candidate, Section 4.1 Eq. (12).
//   score(n, m) = sum of w(e) over hyperedges e incident to n that contain m;
//   cand(n)     = the valid neighbour with the largest score, lowest id on a
//                 tie (R1); -1 when no neighbour is valid.
// Computes cand/cscore for the `nq` vertices listed in `query` (all vertices
// when query is null; then nq must equal V).  cscore is score(n, cand(n)), or
// 0 when there is no candidate.  `seconds` (may be null) receives the wall
// time of building the incidence lists and of the per-vertex loop.
int oracle_candidates(int32_t V, int32_t E, const int64_t* eoff, const uint32_t* pins,
                      const int32_t* w, const int32_t* size, const int32_t* syn,
                      const int64_t* soff, const int32_t* sids, int32_t omega,
                      int32_t phi, int32_t delta, int32_t nq, const int32_t* query,
                      int32_t* cand, int32_t* cscore, int32_t nthreads, double* seconds) {
  Level L{V, E, eoff, pins, w, size, syn, soff, sids};
  Limits lim{omega, phi, delta};
  auto t0 = std::chrono::steady_clock::now();
  Incidence inc = build_incidence(V, E, eoff, pins);
  auto t1 = std::chrono::steady_clock::now();
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    // Sparse accumulator: a dense score array over all vertices plus the
    // list of touched entries, reset after every vertex.
    std::vector<int64_t> score((size_t)V, 0);
    std::vector<int32_t> touched;
#pragma omp for schedule(dynamic, 64)
    for (int32_t qi = 0; qi < nq; ++qi) {
      int32_t n = query ? query[qi] : qi;
      touched.clear();
      for (int64_t j = inc.off[n]; j < inc.off[n + 1]; ++j) {
        int32_t e = inc.edge[j];
        for (int64_t k = eoff[e]; k < eoff[e + 1]; ++k) {
          int32_t m = (int32_t)(pins[k] & IDMASK);
          if (m == n) continue;
          if (score[m] == 0) touched.push_back(m);
          score[m] += w[e];
        }
      }
      int32_t best = -1;
      int64_t best_s = 0;
      for (int32_t m : touched) {
        int64_t s = score[m];
        bool better = s > best_s || (s == best_s && m < best);
        if (better && merge_valid(L, lim, n, m)) {
          best = m;
          best_s = s;
        }
      }
      for (int32_t m : touched) score[m] = 0;
      cand[qi] = best;
      cscore[qi] = best < 0 ? 0 : (int32_t)best_s;
    }
  }
  auto t2 = std::chrono::steady_clock::now();
  if (seconds) {
    seconds[0] = std::chrono::duration<double>(t1 - t0).count();
    seconds[1] = std::chrono::duration<double>(t2 - t1).count();
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Matching, Section 4.1 Eq. (13), evaluated as written:
//   match(n) = cand(n)           if cand(cand(n)) = n or match(cand(n)) = n,
//            = argmax_{m : cand(m) = n} score(n, m)   otherwise, if such m,
//            = -1                otherwise.
// score(n, m) for a child m is cscore[m] because scores are symmetric.  The
// recursion "match(cand(n)) = n" climbs the candidate arcs; it is evaluated
// with an explicit stack and memoised.  Returns 0, or -1 if a candidate cycle
// longer than two is found (impossible per Section 4.1).
int oracle_match(int32_t V, const int32_t* cand, const int32_t* cscore, int32_t* match) {
  // best child by (score desc, id asc), R1
  std::vector<int32_t> bc(V, -1);
  for (int32_t m = 0; m < V; ++m) {
    int32_t p = cand[m];
    if (p < 0) continue;
    int32_t cur = bc[p];
    if (cur < 0 || cscore[m] > cscore[cur] || (cscore[m] == cscore[cur] && m < cur))
      bc[p] = m;
  }
  // state: 0 unknown, 1 in progress, 2 known
  std::vector<uint8_t> state(V, 0);
  std::vector<int32_t> memo(V, -1);
  std::vector<int32_t> stack;
  for (int32_t s = 0; s < V; ++s) {
    if (state[s] == 2) continue;
    stack.clear();
    stack.push_back(s);
    while (!stack.empty()) {
      int32_t n = stack.back();
      int32_t c = cand[n];
      bool ready = true;
      bool taken = false;
      if (c >= 0) {
        if (cand[c] == n) {
          taken = true;  // two-cycle
        } else if (state[c] == 2) {
          taken = (memo[c] == n);
        } else {
          if (state[c] == 1) return -1;  // longer cycle
          state[n] = 1;
          stack.push_back(c);
          ready = false;
        }
      }
      if (!ready) continue;
      memo[n] = taken ? c : bc[n];
      state[n] = 2;
      stack.pop_back();
    }
  }
  for (int32_t n = 0; n < V; ++n) match[n] = memo[n];
  return 0;
}

// ---------------------------------------------------------------------------
// Coarse vertex map from a matching (R5): a vertex is a representative when it
// is unmatched or smaller than its partner; coarse ids rank representatives in
// ascending order and a matched pair shares its representative's id.
// Returns the number of coarse vertices.
int32_t oracle_vmap_from_match(int32_t V, const int32_t* match, int32_t* vmap) {
  std::vector<int32_t> rank(V, -1);
  int32_t r = 0;
  for (int32_t n = 0; n < V; ++n)
    if (match[n] < 0 || n < match[n]) rank[n] = r++;
  for (int32_t n = 0; n < V; ++n) {
    int32_t rep = (match[n] < 0 || n < match[n]) ? n : match[n];
    vmap[n] = rank[rep];
  }
  return r;
}

// ---------------------------------------------------------------------------
// Coarse hypergraph G_P for an arbitrary vertex map rho = vmap with values in
// [0, n_coarse) (Section 3, "Partitioning Definition", and Section 4.1 state
// propagation):
//   * each fine hyperedge becomes its set of distinct coarse vertices, a
//     vertex's destination flag being the OR over its members (R3);
//     hyperedges left with fewer than two vertices are dropped (R4);
//   * hyperedges with identical (vertex, flag) lists are one coarse hyperedge;
//     eta = sum of w (Section 3), mult = sum of mult;
//   * coarse hyperedges are ordered by their smallest fine hyperedge (R5);
//   * super-node state: size and syn summed, inbound set = union (R2).
// Output arrays must have the input capacities (E+1, P, E, E, V', V', V'+1 and
// the input's inbound-set length).  Writes the output sizes to `sizes`:
// [E', P', total inbound-set length].  Returns 0, or -1 on a vmap value out of
// range.
int oracle_contract(int32_t V, int32_t E, const int64_t* eoff, const uint32_t* pins,
                    const int32_t* w, const int32_t* mult, const int32_t* size,
                    const int32_t* syn, const int64_t* soff, const int32_t* sids,
                    const int32_t* vmap, int32_t n_coarse, int64_t* out_eoff,
                    uint32_t* out_pins, int32_t* out_w, int32_t* out_mult,
                    int32_t* out_size, int32_t* out_syn, int64_t* out_soff,
                    int32_t* out_sids, int64_t* sizes) {
  for (int32_t v = 0; v < V; ++v)
    if (vmap[v] < 0 || vmap[v] >= n_coarse) return -1;
  // hyperedges
  std::map<std::vector<uint32_t>, int32_t> group;  // list -> coarse edge id
  std::vector<std::vector<uint32_t>> lists;
  std::vector<int64_t> eta, mu;
  for (int32_t e = 0; e < E; ++e) {
    std::map<int32_t, uint32_t> flags;  // coarse vertex -> destination flag
    for (int64_t k = eoff[e]; k < eoff[e + 1]; ++k) {
      int32_t c = vmap[pins[k] & IDMASK];
      uint32_t d = (pins[k] & DST) ? 1u : 0u;
      auto it = flags.find(c);
      if (it == flags.end()) flags[c] = d;
      else it->second |= d;
    }
    if (flags.size() < 2) continue;
    std::vector<uint32_t> key;
    for (auto& kv : flags) key.push_back((uint32_t)kv.first | (kv.second ? DST : 0u));
    auto it = group.find(key);
    if (it == group.end()) {
      int32_t id = (int32_t)lists.size();
      group.emplace(key, id);
      lists.push_back(key);
      eta.push_back(w[e]);
      mu.push_back(mult[e]);
    } else {
      eta[it->second] += w[e];
      mu[it->second] += mult[e];
    }
  }
  int64_t p = 0;
  out_eoff[0] = 0;
  for (size_t a = 0; a < lists.size(); ++a) {
    for (uint32_t x : lists[a]) out_pins[p++] = x;
    out_eoff[a + 1] = p;
    out_w[a] = (int32_t)eta[a];
    out_mult[a] = (int32_t)mu[a];
  }
  // super-node state
  std::vector<std::vector<int32_t>> members(n_coarse);
  for (int32_t v = 0; v < V; ++v) members[vmap[v]].push_back(v);
  int64_t s = 0;
  out_soff[0] = 0;
  for (int32_t c = 0; c < n_coarse; ++c) {
    int64_t sz = 0, sy = 0;
    std::vector<int32_t> uni;
    for (int32_t v : members[c]) {
      sz += size[v];
      sy += syn[v];
      uni.insert(uni.end(), sids + soff[v], sids + soff[v + 1]);
    }
    std::sort(uni.begin(), uni.end());
    uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
    out_size[c] = (int32_t)sz;
    out_syn[c] = (int32_t)sy;
    for (int32_t x : uni) out_sids[s++] = x;
    out_soff[c + 1] = s;
  }
  sizes[0] = (int64_t)lists.size();
  sizes[1] = p;
  sizes[2] = s;
  return 0;
}

// ---------------------------------------------------------------------------
// Connectivity, Section 3 Eq. (1):
//   Conn(rho) = sum over hyperedges e of w(e) * (|{rho(n) : n in e}| - 1).
// Every pin counts, the source included.  int64 accumulation.
int64_t oracle_connectivity(int32_t E, const int64_t* eoff, const uint32_t* pins,
                            const int32_t* w, const int32_t* part) {
  int64_t conn = 0;
  std::vector<int32_t> blocks;
  for (int32_t e = 0; e < E; ++e) {
    blocks.clear();
    for (int64_t k = eoff[e]; k < eoff[e + 1]; ++k) blocks.push_back(part[pins[k] & IDMASK]);
    std::sort(blocks.begin(), blocks.end());
    int64_t lambda = std::unique(blocks.begin(), blocks.end()) - blocks.begin();
    if (lambda > 0) conn += (int64_t)w[e] * (lambda - 1);
  }
  return conn;
}

// ---------------------------------------------------------------------------
// Evaluation of a partition `part` (values in [0, n_parts)) of a level
// (Section 3): Eq. (1) and, per part p, |p| in neurons (sum of size), its
// inbound synapses (sum of syn) and its distinct inbound original axons
// |U in(n)| (the union of the members' explicit inbound sets, R2).  Writes
// per-part totals (n_parts entries each) and the summary
// [conn, max size, max syn, max axons, parts over Omega, over Phi,
// over Delta, n_parts].  Returns 0, or -1 on a part value out of range.
int oracle_partition_report(int32_t V, int32_t E, const int64_t* eoff, const uint32_t* pins,
                            const int32_t* w, const int32_t* size, const int32_t* syn,
                            const int64_t* soff, const int32_t* sids, const int32_t* part,
                            int32_t n_parts, int32_t omega, int32_t phi, int32_t delta,
                            int64_t* summary, int32_t* out_size, int32_t* out_syn,
                            int32_t* out_ax) {
  for (int32_t v = 0; v < V; ++v)
    if (part[v] < 0 || part[v] >= n_parts) return -1;
  std::vector<std::vector<int32_t>> members(n_parts);
  for (int32_t v = 0; v < V; ++v) members[part[v]].push_back(v);
  for (int i = 0; i < 8; ++i) summary[i] = 0;
  summary[0] = oracle_connectivity(E, eoff, pins, w, part);
  for (int32_t p = 0; p < n_parts; ++p) {
    int64_t sz = 0, sy = 0;
    std::vector<int32_t> uni;
    for (int32_t v : members[p]) {
      sz += size[v];
      sy += syn[v];
      uni.insert(uni.end(), sids + soff[v], sids + soff[v + 1]);
    }
    std::sort(uni.begin(), uni.end());
    const int64_t ax = std::unique(uni.begin(), uni.end()) - uni.begin();
    out_size[p] = (int32_t)sz;
    out_syn[p] = (int32_t)sy;
    out_ax[p] = (int32_t)ax;
    summary[1] = std::max(summary[1], sz);
    summary[2] = std::max(summary[2], sy);
    summary[3] = std::max(summary[3], ax);
    summary[4] += sz > omega;
    summary[5] += sy > phi;
    summary[6] += ax > delta;
  }
  summary[7] = n_parts;
  return 0;
}

// ---------------------------------------------------------------------------
// One refinement round on a level (Section 4.1, "Uncoarsening and
// Refinement"), written step by step as the paper states it.  `part` (values
// in [0, n_parts)) is updated in place.  Readings (design notes R8-R12):
//   R8  the parts a vertex may move to are those sharing a hyperedge with it
//       (any other part has loss(n, p) = the vertex's whole incident weight);
//   R9  every vertex with a feasible target proposes its best move, whatever
//       the sign of its gain; best = largest gain, then lowest part id;
//   R10 moves are ordered by gain (descending), then vertex id (ascending);
//   R11 a prefix is valid when no part that was within a limit before the
//       round is above it after the prefix's moves; the chosen prefix has
//       the largest cumulative recomputed gain among valid prefixes with a
//       positive one (the shortest on ties); no prefix, no move;
//   R12 "inbound" for a part: a hyperedge is inbound to p when p holds one
//       of its destination-flagged pins; the distinct axons of p are the
//       members' axons already internal to them plus the multiplicities of
//       the hyperedges inbound to p (the same count as the level's state).
// Writes info = [proposals, moves applied, Eq. (1) decrease].  Returns 0, or
// -1 on a part value out of range.
int oracle_refine_round(int32_t V, int32_t E, const int64_t* eoff, const uint32_t* pins,
                        const int32_t* w, const int32_t* mult, const int32_t* size,
                        const int32_t* syn, const int32_t* ax, int32_t* part, int32_t n_parts,
                        int32_t omega, int32_t phi, int32_t delta, int64_t* info) {
  for (int32_t v = 0; v < V; ++v)
    if (part[v] < 0 || part[v] >= n_parts) return -1;
  Incidence inc = build_incidence(V, E, eoff, pins);
  // pins(p, e) and the destination-flagged pins of p in e
  std::vector<std::map<int32_t, int64_t>> pc(E), dpc(E);
  for (int32_t e = 0; e < E; ++e)
    for (int64_t k = eoff[e]; k < eoff[e + 1]; ++k) {
      int32_t v = (int32_t)(pins[k] & IDMASK);
      pc[e][part[v]] += 1;
      if (pins[k] & DST) dpc[e][part[v]] += 1;
    }
  // per-vertex axons internal to the vertex (not on any flagged pin)
  std::vector<int64_t> internal(V);
  for (int32_t v = 0; v < V; ++v) {
    int64_t flagged = 0;
    for (int64_t j = inc.off[v]; j < inc.off[v + 1]; ++j)
      if (inc.is_dst[j]) flagged += mult[inc.edge[j]];
    internal[v] = ax[v] - flagged;
  }
  // part state
  std::vector<int64_t> psize(n_parts, 0), psyn(n_parts, 0), pax(n_parts, 0);
  for (int32_t v = 0; v < V; ++v) {
    psize[part[v]] += size[v];
    psyn[part[v]] += syn[v];
    pax[part[v]] += internal[v];
  }
  for (int32_t e = 0; e < E; ++e)
    for (auto& kv : dpc[e])
      if (kv.second > 0) pax[kv.first] += mult[e];
  // proposals: save(n), loss(n, p), the best feasible move
  struct Move {
    int64_t gain;
    int32_t n, from, to;
  };
  std::vector<Move> moves;
  for (int32_t n = 0; n < V; ++n) {
    const int32_t a = part[n];
    int64_t save = 0, whole = 0;
    std::map<int32_t, int64_t> touch, hit;  // part -> weight with pins > 0; flagged overlap
    for (int64_t j = inc.off[n]; j < inc.off[n + 1]; ++j) {
      const int32_t e = inc.edge[j];
      whole += w[e];
      if (pc[e][a] == 1) save += w[e];
      for (auto& kv : pc[e]) {
        if (kv.first == a || kv.second == 0) continue;
        touch[kv.first] += w[e];
        if (inc.is_dst[j] && dpc[e].count(kv.first) && dpc[e][kv.first] > 0)
          hit[kv.first] += mult[e];
      }
    }
    bool found = false;
    Move best{0, n, a, -1};
    for (auto& kv : touch) {
      const int32_t p = kv.first;
      const int64_t loss = whole - kv.second;
      const int64_t gain = save - loss;
      const int64_t h = hit.count(p) ? hit[p] : 0;
      const bool ok = psize[p] + size[n] <= omega && psyn[p] + syn[n] <= phi &&
                      pax[p] + ax[n] - h <= delta;
      if (!ok) continue;
      if (!found || gain > best.gain) {  // parts visited in ascending order
        best = Move{gain, n, a, p};
        found = true;
      }
    }
    if (found) moves.push_back(best);
  }
  std::sort(moves.begin(), moves.end(), [](const Move& x, const Move& y) {
    return x.gain != y.gain ? x.gain > y.gain : x.n < y.n;
  });
  // the prefixes, applied one move at a time: recomputed gains and validity
  std::vector<uint8_t> within(3 * (size_t)n_parts);
  for (int32_t p = 0; p < n_parts; ++p) {
    within[3 * p] = psize[p] <= omega;
    within[3 * p + 1] = psyn[p] <= phi;
    within[3 * p + 2] = pax[p] <= delta;
  }
  auto over = [&](int32_t p) {
    return (within[3 * p] && psize[p] > omega) || (within[3 * p + 1] && psyn[p] > phi) ||
           (within[3 * p + 2] && pax[p] > delta);
  };
  int64_t newly_over = 0, cum = 0, best_cum = 0;
  int64_t best_len = 0;
  for (size_t i = 0; i < moves.size(); ++i) {
    const Move& m = moves[i];
    const int32_t a = m.from, b = m.to;
    newly_over -= over(a) + over(b);
    int64_t g = 0;
    for (int64_t j = inc.off[m.n]; j < inc.off[m.n + 1]; ++j) {
      const int32_t e = inc.edge[j];
      if (pc[e][a] == 1) g += w[e];
      if (pc[e][b] == 0) g -= w[e];
      pc[e][a] -= 1;
      pc[e][b] += 1;
      if (inc.is_dst[j]) {
        if (--dpc[e][a] == 0) pax[a] -= mult[e];
        if (dpc[e][b]++ == 0) pax[b] += mult[e];
      }
    }
    psize[a] -= size[m.n];
    psize[b] += size[m.n];
    psyn[a] -= syn[m.n];
    psyn[b] += syn[m.n];
    pax[a] -= internal[m.n];
    pax[b] += internal[m.n];
    newly_over += over(a) + over(b);
    cum += g;
    if (newly_over == 0 && cum > 0 && cum > best_cum) {
      best_cum = cum;
      best_len = (int64_t)i + 1;
    }
  }
  for (int64_t i = 0; i < best_len; ++i) part[moves[i].n] = moves[i].to;
  info[0] = (int64_t)moves.size();
  info[1] = best_len;
  info[2] = best_cum;
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Placement (Section 4.2).  The lattice H has width x height cores; core c
// is (x, y) = (c / height, c % height), so core ids ascend lexicographically
// over (x, y); dist is the Manhattan distance (Section 2).  The hypergraph is
// G_P (parts as nodes); only its pins and weights are used.  Readings (design
// notes P1-P6):
//   P1 the Hilbert order of H is that of the smallest 2^k x 2^k square
//      holding H, cores outside H skipped;
//   P2 a section of s nodes splits into its first ceil(s/2) and last
//      floor(s/2) positions; a label-propagation round computes every
//      node's gain of crossing to the other half (cut = hyperedges with pins
//      in both halves, counting only the section's own nodes), sorts both
//      halves by (gain desc, id asc) and swaps the i-th pairs while their
//      gains sum above 0; rounds stop after `lp_rounds` or a round without
//      swaps;
//   P3 folding: the connection of a section c to a section u is the weight of
//      the hyperedges with pins in both; the child of a left (right) section
//      more connected to the section's sibling goes right (left); ties keep
//      the order; a flip reverses the pair's concatenation;
//   P4 a node proposes the swap with the adjacent core of largest tension
//      (Eq. 15), lowest core id on ties, when that tension is positive;
//      empty cores propose nothing;
//   P5 the objective is the residual distance D = sum over hyperedges of
//      eta(a) times the distances of all unordered pin pairs; the tension of
//      a swap is exactly its decrease of D;
//   P6 swaps are matched by Eq. 13 over cores (lowest core id on ties),
//      ordered by tension (descending) then smaller core id; the prefix of
//      largest positive cumulative recomputed tension (the shortest on ties)
//      is applied; rounds until none is applied.

namespace {

// Hilbert curve index -> (x, y) on an n x n square (n a power of two), the
// classic iterative construction quadrant by quadrant.
void hilbert_xy(int64_t n, int64_t d, int64_t& x, int64_t& y) {
  x = y = 0;
  int64_t t = d;
  for (int64_t s = 1; s < n; s *= 2) {
    const int64_t rx = 1 & (t / 2);
    const int64_t ry = 1 & (t ^ rx);
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - x;
        y = s - 1 - y;
      }
      std::swap(x, y);
    }
    x += s * rx;
    y += s * ry;
    t /= 4;
  }
}

struct PlaceGraph {
  int32_t V, E;
  const int64_t* eoff;
  const uint32_t* pins;
  const int32_t* eta;
  std::vector<std::vector<int32_t>> inc;  // hyperedges of each node
  PlaceGraph(int32_t V_, int32_t E_, const int64_t* eo, const uint32_t* pi, const int32_t* et)
      : V(V_), E(E_), eoff(eo), pins(pi), eta(et), inc(V_) {
    for (int32_t e = 0; e < E; ++e)
      for (int64_t k = eoff[e]; k < eoff[e + 1]; ++k) inc[pins[k] & IDMASK].push_back(e);
  }
  int32_t pin(int64_t k) const { return (int32_t)(pins[k] & IDMASK); }
};

int64_t manhattan(int32_t a, int32_t b, int32_t height) {
  const int64_t dx = (int64_t)(a / height) - (b / height);
  const int64_t dy = (int64_t)(a % height) - (b % height);
  return (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy);
}

// One section [start, start + len) of the sequence: split, then label
// propagation between the halves (P2).
void bisect_section(const PlaceGraph& G, std::vector<int32_t>& seq, int64_t start, int64_t len,
                    int32_t lp_rounds) {
  const int64_t nl = len - len / 2;
  for (int32_t round = 0; round < lp_rounds; ++round) {
    std::map<int32_t, int> side;  // node -> 0 left, 1 right
    for (int64_t i = 0; i < len; ++i) side[seq[start + i]] = i < nl ? 0 : 1;
    std::map<int32_t, std::pair<int64_t, int64_t>> cnt;  // hyperedge -> (left, right) pins
    for (auto& kv : side)
      for (int32_t e : G.inc[kv.first]) {
        auto& c = cnt[e];
        (kv.second ? c.second : c.first) += 1;
      }
    std::vector<std::pair<int64_t, int32_t>> L, R;  // (-gain, node)
    for (auto& kv : side) {
      const int32_t u = kv.first;
      const bool left = kv.second == 0;
      int64_t g = 0;
      for (int32_t e : G.inc[u]) {
        const auto& c = cnt[e];
        const int64_t mine = left ? c.first : c.second, other = left ? c.second : c.first;
        if (mine == 1 && other > 0) g += G.eta[e];
        if (other == 0 && mine > 1) g -= G.eta[e];
      }
      (left ? L : R).push_back({-g, u});
    }
    std::sort(L.begin(), L.end());
    std::sort(R.begin(), R.end());
    std::map<int32_t, int64_t> pos;
    for (int64_t i = 0; i < len; ++i) pos[seq[start + i]] = start + i;
    int64_t swaps = 0;
    for (size_t i = 0; i < L.size() && i < R.size(); ++i) {
      if (-L[i].first - R[i].first <= 0) break;
      std::swap(seq[pos[L[i].second]], seq[pos[R[i].second]]);
      ++swaps;
    }
    if (swaps == 0) break;
  }
}

int64_t section_conn(const PlaceGraph& G, const std::vector<int32_t>& a, int64_t as, int64_t al,
                     const std::vector<int32_t>& b, int64_t bs, int64_t bl) {
  std::vector<uint8_t> in_b(G.E, 0);
  for (int64_t i = 0; i < bl; ++i)
    for (int32_t e : G.inc[b[bs + i]]) in_b[e] = 1;
  std::vector<uint8_t> seen(G.E, 0);
  int64_t c = 0;
  for (int64_t i = 0; i < al; ++i)
    for (int32_t e : G.inc[a[as + i]])
      if (in_b[e] && !seen[e]) {
        seen[e] = 1;
        c += G.eta[e];
      }
  return c;
}

// Folding (P3): returns the folded order of section [start, start + len) of
// the bisected sequence `bis`; `side` is 0 / 1 for a left / right section,
// -1 for the root; (us, ul) the section's sibling.
std::vector<int32_t> fold(const PlaceGraph& G, const std::vector<int32_t>& bis, int64_t start,
                          int64_t len, int side, int64_t us, int64_t ul) {
  if (len == 1) return {bis[start]};
  const int64_t nl = len - len / 2;
  std::vector<int32_t> c0 = fold(G, bis, start, nl, 0, start + nl, len - nl);
  std::vector<int32_t> c1 = fold(G, bis, start + nl, len - nl, 1, start, nl);
  bool flip = false;
  if (side >= 0) {
    const int64_t k0 = section_conn(G, bis, start, nl, bis, us, ul);
    const int64_t k1 = section_conn(G, bis, start + nl, len - nl, bis, us, ul);
    flip = side == 0 ? k0 > k1 : k1 > k0;
  }
  std::vector<int32_t> out(c0);
  out.insert(out.end(), c1.begin(), c1.end());
  if (flip) std::reverse(out.begin(), out.end());
  return out;
}

int64_t residual(const PlaceGraph& G, const int32_t* core_of, int32_t height) {
  int64_t d = 0;
  for (int32_t e = 0; e < G.E; ++e) {
    int64_t s = 0;
    for (int64_t i = G.eoff[e]; i < G.eoff[e + 1]; ++i)
      for (int64_t j = i + 1; j < G.eoff[e + 1]; ++j)
        s += manhattan(core_of[G.pin(i)], core_of[G.pin(j)], height);
    d += (int64_t)G.eta[e] * s;
  }
  return d;
}

// Eq. 14: force(p, k) with p at h = core_of[p].
int64_t force(const PlaceGraph& G, const int32_t* core_of, int32_t height, int32_t p,
              int32_t k) {
  const int32_t h = core_of[p];
  int64_t f = 0;
  for (int32_t e : G.inc[p]) {
    int64_t s = 0;
    for (int64_t i = G.eoff[e]; i < G.eoff[e + 1]; ++i) {
      const int32_t q = G.pin(i);
      if (q == p) continue;
      const int64_t dk = manhattan(k, core_of[q], height);
      s += manhattan(h, core_of[q], height) - (dk > 1 ? dk : 1);
    }
    f += (int64_t)G.eta[e] * s;
  }
  return f;
}

}  // namespace

extern "C" {

// The cores of the width x height lattice in Hilbert order (P1); writes
// width * height core ids.
int oracle_hilbert_cores(int32_t width, int32_t height, int32_t* out) {
  int64_t n = 1;
  while (n < width || n < height) n *= 2;
  int64_t k = 0;
  for (int64_t d = 0; d < n * n; ++d) {
    int64_t x, y;
    hilbert_xy(n, d, x, y);
    if (x < width && y < height) out[k++] = (int32_t)(x * height + y);
  }
  return (int32_t)k;
}

// Initial placement of one start (Section 4.2, "Initial Placement"): the
// nodes in the order `order0`, recursive bisection with label propagation
// (P2), folding (P3), and the i-th node of the result on the i-th core of
// the Hilbert order.  Writes core_of[V]; returns 0, or -1 if V exceeds the
// cores.
int oracle_initial_placement(int32_t V, int32_t E, const int64_t* eoff, const uint32_t* pins,
                             const int32_t* eta, int32_t width, int32_t height,
                             const int32_t* order0, int32_t lp_rounds, int32_t* core_of) {
  if ((int64_t)V > (int64_t)width * height) return -1;
  PlaceGraph G(V, E, eoff, pins, eta);
  std::vector<int32_t> seq(order0, order0 + V);
  // bisection, depth by depth: the sections of a depth are disjoint ranges
  std::vector<std::pair<int64_t, int64_t>> cur = {{0, V}};
  while (!cur.empty()) {
    std::vector<std::pair<int64_t, int64_t>> next;
    for (auto& sl : cur) {
      if (sl.second < 2) continue;
      bisect_section(G, seq, sl.first, sl.second, lp_rounds);
      const int64_t nl = sl.second - sl.second / 2;
      next.push_back({sl.first, nl});
      next.push_back({sl.first + nl, sl.second - nl});
    }
    cur.swap(next);
  }
  std::vector<int32_t> order = V > 0 ? fold(G, seq, 0, V, -1, 0, 0) : std::vector<int32_t>();
  std::vector<int32_t> hc((size_t)width * height);
  oracle_hilbert_cores(width, height, hc.data());
  for (int32_t i = 0; i < V; ++i) core_of[order[i]] = hc[i];
  return 0;
}

// Residual distance D (P5) of a placement.
int64_t oracle_residual_distance(int32_t V, int32_t E, const int64_t* eoff, const uint32_t* pins,
                                 const int32_t* eta, int32_t height, const int32_t* core_of) {
  PlaceGraph G(V, E, eoff, pins, eta);
  return residual(G, core_of, height);
}

// Swap refinement (Section 4.2, "Swap Proposals" and "Placement
// Refinement"): rounds of proposals (Eq. 14, 15; P4), matching (Eq. 13 over
// cores; P6), ordering, recomputed tensions and the best prefix, until a
// round applies nothing or max_rounds.  core_of[V] is updated in place.
// info = [rounds, swaps applied, decrease of D].  Returns 0.
int oracle_place_refine(int32_t V, int32_t E, const int64_t* eoff, const uint32_t* pins,
                        const int32_t* eta, int32_t width, int32_t height, int32_t* core_of,
                        int32_t max_rounds, int64_t* info) {
  PlaceGraph G(V, E, eoff, pins, eta);
  const int32_t C = width * height;
  info[0] = info[1] = info[2] = 0;
  for (int32_t round = 0; round < max_rounds; ++round) {
    info[0] = round + 1;
    std::vector<int32_t> occ(C, -1);
    for (int32_t p = 0; p < V; ++p) occ[core_of[p]] = p;
    // proposals: tension (Eq. 15) to each adjacent core
    std::vector<int32_t> cand(C, -1);
    std::vector<int64_t> score(C, 0);
    auto tension = [&](int32_t h, int32_t k) {
      int64_t t = 0;
      if (occ[h] >= 0) t += force(G, core_of, height, occ[h], k);
      if (occ[k] >= 0) t += force(G, core_of, height, occ[k], h);
      return t;
    };
    for (int32_t h = 0; h < C; ++h) {
      if (occ[h] < 0) continue;
      const int32_t x = h / height, y = h % height;
      const int32_t nb[4][2] = {{x - 1, y}, {x, y - 1}, {x, y + 1}, {x + 1, y}};
      int64_t best = 0;
      int32_t bk = -1;
      for (auto& q : nb) {  // ascending core ids
        if (q[0] < 0 || q[0] >= width || q[1] < 0 || q[1] >= height) continue;
        const int32_t k = q[0] * height + q[1];
        const int64_t t = tension(h, k);
        if (t > best) {
          best = t;
          bk = k;
        }
      }
      cand[h] = bk;
      score[h] = best;
    }
    // Eq. 13 over cores (the same rule as the coarsening's matching)
    std::vector<int32_t> bc(C, -1);
    for (int32_t m = 0; m < C; ++m) {
      const int32_t pp = cand[m];
      if (pp < 0) continue;
      const int32_t cur = bc[pp];
      if (cur < 0 || score[m] > score[cur] || (score[m] == score[cur] && m < cur)) bc[pp] = m;
    }
    std::vector<int32_t> mt(C, -2);  // -2 unknown
    std::function<int32_t(int32_t)> match_of = [&](int32_t h) -> int32_t {
      if (mt[h] != -2) return mt[h];
      const int32_t c = cand[h];
      bool taken = false;
      if (c >= 0) taken = cand[c] == h || match_of(c) == h;
      mt[h] = taken ? c : bc[h];
      return mt[h];
    };
    struct Swap {
      int64_t t;
      int32_t a, b;
    };
    std::vector<Swap> sw;
    for (int32_t h = 0; h < C; ++h) {
      const int32_t m = match_of(h);
      if (m > h) sw.push_back({tension(h, m), h, m});
    }
    std::sort(sw.begin(), sw.end(), [](const Swap& x, const Swap& y) {
      return x.t != y.t ? x.t > y.t : x.a < y.a;
    });
    // recomputed tensions along the order, the best prefix
    std::vector<int32_t> trial(core_of, core_of + V);
    std::vector<int32_t> tocc(occ);
    int64_t cum = 0, best_cum = 0, best_len = 0;
    for (size_t i = 0; i < sw.size(); ++i) {
      const int32_t a = sw[i].a, b = sw[i].b;
      int64_t t = 0;
      if (tocc[a] >= 0) t += force(G, trial.data(), height, tocc[a], b);
      if (tocc[b] >= 0) t += force(G, trial.data(), height, tocc[b], a);
      const int32_t pa = tocc[a], pb = tocc[b];
      if (pa >= 0) trial[pa] = b;
      if (pb >= 0) trial[pb] = a;
      tocc[a] = pb;
      tocc[b] = pa;
      cum += t;
      if (cum > best_cum) {
        best_cum = cum;
        best_len = (int64_t)i + 1;
      }
    }
    if (best_len == 0) break;
    for (int64_t i = 0; i < best_len; ++i) {
      const int32_t a = sw[i].a, b = sw[i].b;
      const int32_t pa = occ[a], pb = occ[b];
      if (pa >= 0) core_of[pa] = b;
      if (pb >= 0) core_of[pb] = a;
      occ[a] = pb;
      occ[b] = pa;
    }
    info[1] += best_len;
    info[2] += best_cum;
  }
  return 0;
}

}  // extern "C"
