// Seeded synthetic SNN hypergraph generator.
//
// Builds the level-0 hypergraph of a spiking network in the paper's model
// (Section 2, "SNN and Hardware Models"): one hyperedge per axon, holding the
// source neuron and every synapse target.  The output is an int64 CSR over
// hyperedges whose pins are uint32 words `vertex_id | is_destination << 31`,
// ascending by vertex id inside each hyperedge, plus an int32 spike-rate
// weight per hyperedge.
//
// This module draws random numbers and lays out arrays; it computes nothing of
// the coarsening method itself.  It is the single input source shared by the
// CPU oracle and the GPU library.
//
// Randomness is counter based: every draw is SplitMix64 applied to a key made
// of (seed, graph, neuron, draw index), so the output does not depend on the
// number of threads or on the order of evaluation.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

inline uint64_t mix64(uint64_t z) {
  // SplitMix64 output function (Steele, Lea, Flood 2014).
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Stream tags keep the different kinds of draws independent.
enum : uint64_t {
  TAG_DEGREE = 1, TAG_TARGET = 2, TAG_WEIGHT = 3, TAG_INHIB = 4,
  TAG_GRAPH = 5, TAG_FANOUT = 6,
};

inline uint64_t draw(uint64_t seed, uint64_t graph, uint64_t tag,
                     uint64_t item, uint64_t idx) {
  uint64_t k = mix64(seed);
  k = mix64(k ^ (graph * 0xD6E8FEB86659FD93ULL));
  k = mix64(k ^ (tag * 0xA0761D6478BD642FULL));
  k = mix64(k ^ (item * 0xE7037ED1A0B428DBULL));
  return mix64(k ^ idx);
}

// Uniform integer in [0, n) by 128-bit multiply-shift.
inline uint64_t below(uint64_t x, uint64_t n) {
  return (uint64_t)(((__uint128_t)x * n) >> 64);
}

// Uniform double in (0, 1].
inline double unit_open0(uint64_t x) {
  return (double)((x >> 11) + 1) * (1.0 / 9007199254740992.0);
}

// Uniform double in [0, 1).
inline double unit(uint64_t x) {
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

// Generator kinds.
enum Kind : int32_t {
  K_LAYERED = 1,    // feed-forward layers, uniform distinct targets in next layer
  K_CONV = 2,       // 3x3 convolution window over all channels of next layer
  K_POWERLAW = 3,   // recurrent, out-degree ~ discrete power law
  K_BATCHGRAPH = 4, // one graph of the mixed batch (feed-forward or recurrent)
  K_UNIFORM = 5,    // small recurrent graph with uniform out-degree (tests)
};

struct Spec {
  int32_t kind;
  uint64_t seed;
  uint64_t graph;
  // layered / conv / uniform
  int32_t layers, width, height, channels;
  int32_t fan_min, fan_max;         // out-degree range (inclusive)
  // power law
  int32_t n;                        // neuron count (minimum for batch graphs)
  int32_t n_max;                    // batch graphs: log-uniform n in [n, n_max)
  int32_t dmin, dmax;
  double alpha;
  double inhib_frac;
  double w_mean;                    // exponential weight mean
  int32_t w_min, w_max;             // uniform weight range
  int32_t w_mode;                   // 0 uniform int, 1 log-uniform 1..w_max, 2 exponential
};

struct Model {
  Spec s;
  int32_t V = 0;
  int32_t E = 0;
  bool feedforward = false;
  std::vector<int32_t> layer_start;  // layer boundaries (size layers+1)
  std::vector<double> cdf;           // power-law CDF over [dmin, dmax]

  void init(const Spec& spec) {
    s = spec;
    if (s.kind == K_LAYERED) {
      feedforward = true;
      V = s.layers * s.width;
      layer_start.resize(s.layers + 1);
      for (int l = 0; l <= s.layers; ++l) layer_start[l] = l * s.width;
      E = layer_start[s.layers - 1];
    } else if (s.kind == K_CONV) {
      feedforward = true;
      int per = s.height * s.width * s.channels;
      V = s.layers * per;
      layer_start.resize(s.layers + 1);
      for (int l = 0; l <= s.layers; ++l) layer_start[l] = l * per;
      E = layer_start[s.layers - 1];
    } else if (s.kind == K_POWERLAW) {
      V = s.n;
      E = s.n;
      cdf.resize(s.dmax - s.dmin + 1);
      double acc = 0.0;
      for (int d = s.dmin; d <= s.dmax; ++d) {
        acc += std::pow((double)d, -s.alpha);
        cdf[d - s.dmin] = acc;
      }
      for (double& c : cdf) c /= acc;
    } else if (s.kind == K_BATCHGRAPH) {
      // Graph-level draws: topology coin and neuron count.
      uint64_t coin = draw(s.seed, s.graph, TAG_GRAPH, 0, 0);
      feedforward = (coin >> 63) != 0;
      double u = unit(draw(s.seed, s.graph, TAG_GRAPH, 0, 1));
      // n = floor(n_min * ratio^u), log-uniform in [n_min, n_min * ratio).
      double nn = (double)s.n * std::pow((double)s.n_max / (double)s.n, u);
      V = (int32_t)std::floor(nn);
      if (V < 8) V = 8;
      if (feedforward) {
        layer_start.resize(5);
        for (int l = 0; l <= 4; ++l) layer_start[l] = (int32_t)(((int64_t)l * V) / 4);
        E = layer_start[3];
      } else {
        E = V;
      }
    } else if (s.kind == K_UNIFORM) {
      V = s.n;
      E = s.n;
    }
  }

  int32_t layer_of(int32_t v) const {
    int l = (int)(std::upper_bound(layer_start.begin(), layer_start.end(), v) -
                  layer_start.begin()) - 1;
    return l;
  }

  // Number of synapse targets of the axon of neuron e.
  int32_t out_degree(int32_t e) const {
    switch (s.kind) {
      case K_LAYERED:
        return s.fan_min;
      case K_CONV: {
        int per = s.height * s.width * s.channels;
        int local = e % per;
        int y = local / (s.width * s.channels);
        int x = (local / s.channels) % s.width;
        int ny = std::min(y + 1, s.height - 1) - std::max(y - 1, 0) + 1;
        int nx = std::min(x + 1, s.width - 1) - std::max(x - 1, 0) + 1;
        return ny * nx * s.channels;
      }
      case K_POWERLAW: {
        double u = unit(draw(s.seed, s.graph, TAG_DEGREE, e, 0));
        int idx = (int)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin());
        if (idx >= (int)cdf.size()) idx = (int)cdf.size() - 1;
        int d = s.dmin + idx;
        if (d > V - 1) d = V - 1;
        return d;
      }
      case K_BATCHGRAPH:
      case K_UNIFORM: {
        uint64_t r = draw(s.seed, s.graph, TAG_FANOUT, e, 0);
        int d = s.fan_min + (int)below(r, (uint64_t)(s.fan_max - s.fan_min + 1));
        int pool;
        if (feedforward) {
          int l = layer_of(e);
          pool = layer_start[l + 2] - layer_start[l + 1];
        } else {
          pool = V - 1;
        }
        if (d > pool) d = pool;
        return d;
      }
    }
    return 0;
  }

  int32_t weight(int32_t e) const {
    uint64_t r = draw(s.seed, s.graph, TAG_WEIGHT, e, 0);
    int32_t w = 1;
    if (s.w_mode == 0) {
      w = s.w_min + (int32_t)below(r, (uint64_t)(s.w_max - s.w_min + 1));
    } else if (s.w_mode == 1) {
      // log-uniform: floor((w_max + 1)^U), U in [0, 1)
      double v = std::floor(std::pow((double)(s.w_max + 1), unit(r)));
      w = (int32_t)v;
      if (w < 1) w = 1;
      if (w > s.w_max) w = s.w_max;
    } else {
      // exponential with mean w_mean, rounded up, at least 1
      double v = std::ceil(-s.w_mean * std::log(unit_open0(r)));
      if (v < 1.0) v = 1.0;
      if (v > 1.0e6) v = 1.0e6;
      w = (int32_t)v;
    }
    if (s.inhib_frac > 0.0) {
      uint64_t h = draw(s.seed, s.graph, TAG_INHIB, e, 0);
      double lim = s.inhib_frac * 18446744073709551616.0;
      if ((double)h < lim) w = (w + 1) >> 1;
    }
    return w;
  }

  // Distinct synapse targets of neuron e, ascending.
  void targets(int32_t e, int32_t d, std::vector<int32_t>& out,
               std::vector<int32_t>& table) const {
    out.clear();
    if (s.kind == K_CONV) {
      int per = s.height * s.width * s.channels;
      int l = e / per;
      int local = e % per;
      int y = local / (s.width * s.channels);
      int x = (local / s.channels) % s.width;
      int base = (l + 1) * per;
      for (int yy = std::max(y - 1, 0); yy <= std::min(y + 1, s.height - 1); ++yy)
        for (int xx = std::max(x - 1, 0); xx <= std::min(x + 1, s.width - 1); ++xx)
          for (int c = 0; c < s.channels; ++c)
            out.push_back(base + (yy * s.width + xx) * s.channels + c);
      std::sort(out.begin(), out.end());
      return;
    }
    // Pool of candidate targets: next layer, or every other neuron.
    int32_t lo = 0, pool = 0;
    bool skip_self = false;
    if (feedforward) {
      int l = layer_of(e);
      lo = layer_start[l + 1];
      pool = layer_start[l + 2] - lo;
    } else {
      lo = 0;
      pool = V - 1;
      skip_self = true;
    }
    // Floyd's sampling of d distinct values in [0, pool), with an
    // open-addressing set sized to a power of two >= 2d.
    uint32_t cap = 16;
    while (cap < (uint32_t)(2 * d + 2)) cap <<= 1;
    table.assign(cap, -1);
    auto insert = [&](int32_t v) -> bool {
      uint32_t h = (uint32_t)(mix64((uint64_t)v) & (cap - 1));
      while (true) {
        if (table[h] == v) return false;
        if (table[h] < 0) { table[h] = v; return true; }
        h = (h + 1) & (cap - 1);
      }
    };
    uint64_t k = 0;
    for (int32_t j = pool - d; j < pool; ++j, ++k) {
      int32_t t = (int32_t)below(draw(s.seed, s.graph, TAG_TARGET, e, k),
                                 (uint64_t)j + 1);
      if (!insert(t)) insert(j), t = j;
      out.push_back(t);
    }
    for (int32_t& t : out) {
      t += lo;
      if (skip_self && t >= e) t += 1;
    }
    std::sort(out.begin(), out.end());
  }
};

}  // namespace

extern "C" {

// Parameter block passed from Python (field order matters).
typedef struct {
  int32_t kind;
  int32_t layers, width, height, channels;
  int32_t fan_min, fan_max;
  int32_t n, dmin, dmax;
  int32_t w_min, w_max, w_mode;
  int32_t n_max;
  uint64_t seed;
  uint64_t graph;
  double alpha, inhib_frac, w_mean;
} synth_params;

static Spec to_spec(const synth_params* p) {
  Spec s{};
  s.kind = p->kind;
  s.seed = p->seed;
  s.graph = p->graph;
  s.layers = p->layers;
  s.width = p->width;
  s.height = p->height;
  s.channels = p->channels;
  s.fan_min = p->fan_min;
  s.fan_max = p->fan_max;
  s.n = p->n;
  s.n_max = p->n_max;
  s.dmin = p->dmin;
  s.dmax = p->dmax;
  s.alpha = p->alpha;
  s.inhib_frac = p->inhib_frac;
  s.w_mean = p->w_mean;
  s.w_min = p->w_min;
  s.w_max = p->w_max;
  s.w_mode = p->w_mode;
  return s;
}

// Sizes of the generated hypergraph: vertices, hyperedges, pins.
int synth_sizes(const synth_params* p, int32_t* n_vertices, int32_t* n_edges,
                int64_t* n_pins) {
  Model m;
  m.init(to_spec(p));
  int64_t pins = 0;
#pragma omp parallel for reduction(+ : pins) schedule(static)
  for (int32_t e = 0; e < m.E; ++e) pins += 1 + (int64_t)m.out_degree(e);
  *n_vertices = m.V;
  *n_edges = m.E;
  *n_pins = pins;
  return 0;
}

// Fill edge_offsets[E+1], pins[P], weight[E].  Hyperedge e is the axon of
// neuron e; its pins are the source (destination bit 0) merged with the
// sorted targets (destination bit 1).
int synth_fill(const synth_params* p, int64_t* edge_offsets, uint32_t* pins,
               int32_t* weight) {
  Model m;
  m.init(to_spec(p));
  std::vector<int64_t> deg(m.E);
#pragma omp parallel for schedule(static)
  for (int32_t e = 0; e < m.E; ++e) deg[e] = 1 + m.out_degree(e);
  edge_offsets[0] = 0;
  for (int32_t e = 0; e < m.E; ++e) edge_offsets[e + 1] = edge_offsets[e] + deg[e];
#pragma omp parallel
  {
    std::vector<int32_t> tg, table;
#pragma omp for schedule(dynamic, 256)
    for (int32_t e = 0; e < m.E; ++e) {
      int32_t d = (int32_t)deg[e] - 1;
      m.targets(e, d, tg, table);
      uint32_t* out = pins + edge_offsets[e];
      int k = 0;
      bool src_done = false;
      for (int32_t t : tg) {
        if (!src_done && e < t) { out[k++] = (uint32_t)e; src_done = true; }
        out[k++] = (uint32_t)t | 0x80000000u;
      }
      if (!src_done) out[k++] = (uint32_t)e;
      weight[e] = m.weight(e);
    }
  }
  return 0;
}

}  // extern "C"
