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
