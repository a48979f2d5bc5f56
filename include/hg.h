/*
 * hg.h — C ABI of the MI355X SNN-hypergraph coarsening library.
 *
 * One coarsening level of the multi-level partitioner of Ronzani & Silvano,
 * "GPU-Accelerated Hypergraph Partitioning and Placement to Map SNNs on
 * Neuromorphic Hardware", plus the (lambda - 1) connectivity objective.
 *
 * Model (paper, Section 2 "SNN and Hardware Models"): a spiking network is a
 * hypergraph with one hyperedge per axon; its pins are the source neuron and
 * the synapse targets; the hyperedge weight is the spike rate.  Every level
 * of the hierarchy keeps this shape, with super-nodes for vertices.
 *
 * Data layout (all arrays are DEVICE memory owned by the caller):
 *   edge_offsets  int64  [E+1]  CSR offsets of hyperedges into `pins`
 *   pins          uint32 [P]    vertex_id | (flag << 31); ids strictly
 *                               ascending inside each hyperedge; flag = 1
 *                               when the vertex holds a destination of the
 *                               hyperedge's axon(s), 0 for the source only
 *   edge_weight   int32  [E]    spike rate, >= 1; the sum over all hyperedges
 *                               must stay below 2^31
 *   edge_mult     int32  [E]    number of original axons merged into the
 *                               hyperedge (1 at level 0)
 *   v_size        int32  [V]    neurons in the super-node
 *   v_syn         int32  [V]    inbound synapses (sum of in-degrees)
 *   v_axons       int32  [V]    distinct original axons with a destination
 *                               inside the super-node
 *
 * Limits (Section 3, "Partitioning Definition"): a super-node p must satisfy
 * |p| <= Omega, sum |in(n)| <= Phi, |U in(n)| <= Delta; a merge is valid iff
 * all three hold for the union (inclusive bounds).
 *
 * Execution: every call is asynchronous on the context's HIP stream unless
 * stated; scalar results are written to device memory.  The library owns
 * only its scratch arena, grown on demand and freed by hg_destroy.  A context
 * must not be used from two host threads at once.  No call throws; each
 * returns an hg_status and hg_last_error() holds a message.
 *
 * Environment, read by hg_create for the context it creates:
 *   HG_VALIDATE=1        hg_coarsen_level, hg_contract and hg_connectivity
 *                        first run hg_validate_level on their input level
 *                        (synchronously) and return its status
 *   HG_SCRATCH_CAP=B     the scratch arena never grows above B bytes; a call
 *                        that needs more fails with HG_ERR_NO_MEMORY
 *   HG_TEST_FP_BITS=n    (tests only) keeps n bits of the fingerprints that
 *                        group identical coarse hyperedges, so that unequal
 *                        lists share fingerprints and the exact comparison of
 *                        such collisions is exercised; results are unchanged
 */
#ifndef HG_H_
#define HG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HG_OK = 0,
  HG_ERR_INVALID_ARG = 1,   /* null pointer, negative size, bad limits,
                               vmap / part out of range (from hg_sync)     */
  HG_ERR_OVERFLOW = 2,      /* V, E or P >= 2^31, sum of weights >= 2^31     */
  HG_ERR_CAPACITY = 3,      /* an output capacity is smaller than needed     */
  HG_ERR_NO_MEMORY = 4,     /* the scratch arena could not be grown          */
  HG_ERR_HIP = 5,           /* a HIP runtime call failed                     */
  HG_ERR_UNIMPLEMENTED = 6,
  HG_ERR_INVALID_LEVEL = 7, /* hg_validate_level found a malformed level     */
  HG_ERR_INTERNAL = 8       /* a kernel reached an internal bound (reported
                               by hg_sync); results of the calls since the
                               previous hg_sync are not to be used         */
} hg_status;

typedef struct hg_ctx hg_ctx;

typedef struct {
  int32_t max_neurons;  /* Omega */
  int32_t max_synapses; /* Phi   */
  int32_t max_axons;    /* Delta */
} hg_limits;

/* A read-only level.  Sizes are host values. */
typedef struct {
  int32_t n_vertices;
  int32_t n_edges;
  int64_t n_pins;
  const int64_t* edge_offsets;
  const uint32_t* pins;
  const int32_t* edge_weight;
  const int32_t* edge_mult;
  const int32_t* v_size;
  const int32_t* v_syn;
  const int32_t* v_axons;
} hg_level;

/* Output level of hg_contract.  Capacities are host values; a contraction
 * never grows a level, so capacities equal to the input's sizes always
 * suffice.  `sizes` is device int64[3] receiving (V', E', P'). */
typedef struct {
  int32_t cap_vertices;
  int32_t cap_edges;
  int64_t cap_pins;
  int64_t* edge_offsets;
  uint32_t* pins;
  int32_t* edge_weight;
  int32_t* edge_mult;
  int32_t* v_size;
  int32_t* v_syn;
  int32_t* v_axons;
  int64_t* sizes;
} hg_level_out;

/* Context on device `device`, issuing work on `hip_stream` (a hipStream_t;
 * NULL means the default stream). */
int hg_create(int device, void* hip_stream, hg_ctx** out);
int hg_destroy(hg_ctx* ctx);
int hg_set_stream(hg_ctx* ctx, void* hip_stream);
/* Message of the last failing call on this context (never NULL). */
const char* hg_last_error(hg_ctx* ctx);
/* Blocks until all work queued on the context's stream is done, then checks
 * the context's device error word: every data-dependent loop in the kernels
 * is bounded, and a kernel that reaches a bound records it there instead of
 * spinning; hg_sync then returns HG_ERR_INTERNAL and clears the word.  A
 * vmap / part value that the device check found out of range makes it
 * return HG_ERR_INVALID_ARG instead. */
int hg_sync(hg_ctx* ctx);
/* Bytes currently held by the scratch arena. */
int64_t hg_scratch_bytes(hg_ctx* ctx);

/* Phase timing.  When enabled, the calls record HIP events on the context
 * stream around their phases; hg_phase_times synchronises the stream and
 * writes the device time in milliseconds of each phase of the most recent
 * calls since the previous query (0 when a phase did not run):
 *   ms[0] incidence lists and expansion sizes (hg_coarsen_level)
 *   ms[1] scores and candidates, Eq. 12 (hg_coarsen_level)
 *   ms[2] matching and coarse vertex map, Eq. 13 (hg_coarsen_level)
 *   ms[3] contraction (hg_contract)
 *   ms[4] connectivity, Eq. 1 (hg_connectivity)
 * `ms` has HG_NUM_PHASES entries. */
#define HG_NUM_PHASES 5
int hg_enable_timing(hg_ctx* ctx, int on);
int hg_phase_times(hg_ctx* ctx, float* ms);

/*
 * Level-0 state (Section 2 model; Section 3 constraint quantities):
 * v_size = 1, v_syn = v_axons = number of hyperedges in which the vertex has
 * the destination flag, edge_mult = 1.  Outputs are device arrays of V, V, V
 * and E entries.
 */
int hg_init_state(hg_ctx* ctx, int32_t n_vertices, int32_t n_edges, int64_t n_pins,
                  const int64_t* edge_offsets, const uint32_t* pins, int32_t* v_size,
                  int32_t* v_syn, int32_t* v_axons, int32_t* edge_mult);

/*
 * One coarsening level (Section 4.1, "Coarsening"):
 *   score(n, m) = sum of edge_weight over hyperedges holding both n and m
 *                 (Eq. 12; symmetric);
 *   cand(n)     = the neighbour m maximising score(n, m) among those whose
 *                 merge with n is valid (limits above; the distinct-axon
 *                 count of the union is v_axons[n] + v_axons[m] minus the
 *                 edge_mult of hyperedges where both carry the destination
 *                 flag), lowest id on ties; -1 if none;
 *   match       = Eq. 13: two-cycles match; otherwise a vertex is taken by
 *                 its candidate when the candidate is not itself taken and
 *                 picked it as best proposer (score, then lowest id); a
 *                 vertex not taken takes its best proposer; else -1;
 *   vmap[n]     = rank, among representatives (unmatched vertices and the
 *                 smaller vertex of each pair), of n's representative.
 * Outputs (device): cand, cscore (may be NULL; cscore = score(n, cand(n)) or
 * 0), match [V], vmap [V], n_coarse (int32 scalar), any_candidate (int32
 * scalar, 1 iff some vertex has a candidate; 0 means the level is final).
 */
int hg_coarsen_level(hg_ctx* ctx, const hg_level* in, const hg_limits* limits,
                     int32_t* cand, int32_t* cscore, int32_t* match, int32_t* vmap,
                     int32_t* n_coarse, int32_t* any_candidate);
/* Input weights are checked on the device before the scores: a weight below
 * 1 makes the next hg_sync return HG_ERR_INVALID_LEVEL, weights summing to
 * 2^31 or more HG_ERR_OVERFLOW (scores are exact int32 sums); the outputs of
 * the call are then undefined.  hg_contract runs the same check. */

/*
 * Contraction G -> G_P for any vertex map (Section 3, "Partitioning
 * Definition"; Section 4.1 state propagation).  `vmap` [V] holds values in
 * [0, n_coarse); `n_coarse` is a device int32 scalar in [1, V] (0 when V is
 * 0), e.g. written by hg_coarsen_level.  Both are checked on the device
 * before use: an out-of-range value is recorded in the context's error word
 * (hg_sync then fails with HG_ERR_INVALID_ARG and the outputs of the call
 * are undefined, but no memory outside them is written).
 *   * a fine hyperedge becomes its distinct coarse vertices, ascending, the
 *     flag of a coarse vertex being the OR of its members' flags; if fewer
 *     than two remain it is dropped;
 *   * coarse hyperedges with identical (vertex, flag) lists are merged:
 *     weights summed (eta of G_P) and multiplicities summed;
 *   * coarse hyperedges are numbered by their smallest fine hyperedge;
 *   * v_size and v_syn are summed; v_axons of a coarse vertex counts the
 *     original axons with a destination in it, recomputed from the flags.
 * Output sizes go to out->sizes.  Fails with HG_ERR_CAPACITY when a capacity
 * is below the input's size (checked on the host before any work).
 */
int hg_contract(hg_ctx* ctx, const hg_level* in, const int32_t* vmap,
                const int32_t* n_coarse, hg_level_out* out);

/*
 * Connectivity (Section 3, Eq. 1):
 *   conn = sum over hyperedges e of edge_weight[e] * (number of distinct
 *          part[v] over the pins v of e, minus 1).
 * `part` [V] holds values in [0, V), checked on the device as `vmap` of
 * hg_contract is (hg_sync fails with HG_ERR_INVALID_ARG on a value outside
 * it).  Writes the int64 result to device
 * memory `conn`.  Uses only offsets, pins and weights of the level.
 */
int hg_connectivity(hg_ctx* ctx, const hg_level* lvl, const int32_t* part, int64_t* conn);

/*
 * Projection of a partition one level down (Section 4.1, "Uncoarsening and
 * Refinement": super-nodes come undone level by level, each member starting
 * in its super-node's part): part_fine[v] = part_coarse[vmap[v]] for the
 * n_fine vertices of the finer level.  `vmap` is that level's vertex map
 * (hg_coarsen_level), with values in [0, *n_coarse) (device int32 scalar);
 * a value outside is recorded in the error word (hg_sync then returns
 * HG_ERR_INVALID_ARG and the entry is written as 0).  All arrays
 * are device memory; part_coarse has *n_coarse entries.
 */
int hg_project(hg_ctx* ctx, int32_t n_fine, const int32_t* vmap, const int32_t* n_coarse,
               const int32_t* part_coarse, int32_t* part_fine);

/*
 * Evaluation of a partition of a level (Section 3): `part` [V] holds part
 * ids in [0, *n_parts) (device int32 scalar; checked on the device as
 * hg_contract checks its vmap).  Writes to device int64 summary[8]:
 *   [0] Eq. 1, sum over hyperedges of w(e) (lambda(e) - 1)
 *   [1..3] the largest part size (neurons), inbound synapses and distinct
 *          inbound original axons over the parts
 *   [4..6] the number of parts above Omega, Phi and Delta of `limits`
 *   [7] the number of parts
 * and, where the pointers are not NULL, each part's three totals to device
 * int32 arrays of *n_parts entries.  Needs the level's state (v_size, v_syn,
 * v_axons, edge_mult): a part's distinct axons count every original axon
 * with a destination in the part, as in hg_contract, which this call runs
 * with `part` as the vertex map (its scratch is the context's arena).
 */
int hg_partition_report(hg_ctx* ctx, const hg_level* lvl, const int32_t* part,
                        const int32_t* n_parts, const hg_limits* limits, int64_t* summary,
                        int32_t* part_size, int32_t* part_syn, int32_t* part_axons);

/*
 * Refinement of a partition on one level (Section 4.1, "Uncoarsening and
 * Refinement").  `part` [V] (device int32, values in [0, n_parts), checked
 * on the device as hg_contract checks its vmap) is refined in place, in
 * rounds of:
 *   * pins(p, e), and per vertex n in part A: save(n) = weight of its
 *     hyperedges in which n is A's only pin, loss(n, p) = weight of its
 *     hyperedges without a pin in p, for every part p sharing a hyperedge
 *     with n; gain = save - loss; each vertex proposes its best move whose
 *     target stays within `limits` with n added (largest gain, lowest part);
 *   * the moves sorted by gain (descending), vertex (ascending); each gain
 *     recomputed as if the moves before it were applied; the prefix sums of
 *     the recomputed gains; per move, the limits crossed by the part totals
 *     (neurons, inbound synapses, distinct inbound axons: axons internal to
 *     the part's vertices plus the multiplicities of the hyperedges in which
 *     the part holds a destination-flagged pin) in move order, for limits a
 *     part met before the round;
 *   * the valid prefix (no crossing left) with the largest positive
 *     cumulative gain, shortest on ties, is applied.
 * Rounds stop after one that applies nothing, or after max_rounds.  Writes
 * host int64 info[4]: rounds run, moves applied, decrease of Eq. 1 (both
 * summed over the rounds), moves proposed in the last round.  Needs the
 * level's state.  Synchronous (reads sizes back between steps); its scratch
 * (about 150 bytes per pin) is the context's arena.
 */
int hg_refine(hg_ctx* ctx, const hg_level* lvl, int32_t* part, int32_t n_parts,
              const hg_limits* limits, int32_t max_rounds, int64_t* info);

/*
 * hg_connectivity with no allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation in their loop).  Same arguments, result and checks
 * as hg_connectivity; its kernels use a fixed device array of the library
 * (64 MiB per GPU, held until the process ends) instead of the context's
 * arena.  A level needing more than that (about 12 bytes per vertex plus 16
 * per hyperedge, e.g. 2.3M of each) fails with HG_ERR_CAPACITY before any
 * work.  All calls on one GPU share the array: calls that overlap on one GPU
 * (other streams or host threads) race, and the caller must serialise them.
 * With HG_VALIDATE=1 the level check also uses the fixed array.
 */
int hg_connectivity_static(hg_ctx* ctx, const hg_level* lvl, const int32_t* part,
                           int64_t* conn);

/*
 * Score-step tuning of a context.  The score step (Eq. 12) scores a vertex in
 * one pass over an on-chip table when its distinct-neighbour bound (its
 * expansion, the sum of the sizes of its incident hyperedges, capped by the
 * vertex count) is at most single_pass_load16/16 of the table's slots.
 * Neighbourhoods that visit at least one id in dense_ratio of the level's
 * ids (dense_ratio * expansion >= V; 0 disables it) and are larger than the
 * single-pass tables or have an expansion of at least 2^16 are scored in
 * dense windows of 2^14 ids, one packed (score, overlap) word per id, on
 * levels of at most 2^21 vertices.  Other large neighbourhoods are scored in
 * windows of neighbour ids with an on-chip bitmap of seen ids (at most 768
 * incident hyperedges), else in passes over a table, each range aimed at
 * pass_fill16/16 of it where the distinct-axon overlap of Section 3 can
 * bind.  On levels whose id windows are aligned (at most 16 windows of 2^19
 * ids) and whose pins are 16-byte aligned, wide_loads = 1 reads the long
 * slices of the windows 16 bytes per lane; 0 reads one pin per lane.
 * Results never depend on these values, only the speed does.
 * Defaults 8, 5, 8 and 1; accepted ranges 1..12, 1..10, 0..64 and 0..1
 * (HG_ERR_INVALID_ARG otherwise).
 */
typedef struct {
  int32_t single_pass_load16;
  int32_t pass_fill16;
  int32_t dense_ratio;
  int32_t wide_loads;
} hg_tuning;
int hg_set_tuning(hg_ctx* ctx, const hg_tuning* tuning);
int hg_get_tuning(hg_ctx* ctx, hg_tuning* tuning);

/*
 * Batches: many independent hypergraphs coarsened together (Section 4.1 per
 * graph, each with its own limits).  The graphs are laid side by side as one
 * level; they share no hyperedge, so every graph's hierarchy, partition and
 * level count are exactly those of a separate run (hg_coarsen_level +
 * hg_contract until no candidate).  A graph is finished after the first level
 * at which none of its vertices proposes a candidate.
 *
 * The batch owns all its device memory (hg_batch_create allocates it for the
 * given totals; hg_batch_bytes reports it) and works on the context's stream
 * with the context's tuning.  Graphs can be added between steps, also while
 * others are half-way through their hierarchy.
 *
 *   hg_batch_create    capacities are totals over the graphs held at once
 *                      (pins below 2^31); max_graphs is the number of slots
 *   hg_batch_add_graph copies a level with state (device arrays, e.g. from
 *                      hg_init_state) into a free slot; writes the slot
 *                      index; HG_ERR_CAPACITY when slots, vertices,
 *                      hyperedges or pins would exceed the capacities
 *   hg_batch_step      n_levels levels of every unfinished graph;
 *                      use_graph != 0 replays one HIP graph per level (the
 *                      level's kernels read all sizes from device memory)
 *   hg_batch_done      synchronous; writes up to `cap` slots finished since
 *                      the last call and the number still running
 *   hg_batch_result    synchronous; for a reported slot: part[v] (device
 *                      int32, one entry per vertex of the graph as added) =
 *                      its final super-node numbered 0..n_parts-1 inside the
 *                      graph, and the number of contractions performed; then
 *                      releases the slot
 *   hg_batch_compact   removes released graphs from the level (their slots
 *                      become free)
 *   hg_batch_sizes     synchronous; int64[4]: V, E, P of the current level
 *                      and the original vertices held for unreleased graphs
 */
typedef struct hg_batch hg_batch;
int hg_batch_create(hg_ctx* ctx, int32_t max_graphs, int32_t cap_vertices, int32_t cap_edges,
                    int64_t cap_pins, hg_batch** out);
int hg_batch_destroy(hg_batch* batch);
int64_t hg_batch_bytes(hg_batch* batch);
int hg_batch_add_graph(hg_batch* batch, const hg_level* level, const hg_limits* limits,
                       int32_t* slot);
int hg_batch_step(hg_batch* batch, int32_t n_levels, int32_t use_graph);
int hg_batch_done(hg_batch* batch, int32_t* slots, int32_t cap, int32_t* n_done,
                  int32_t* n_running);
int hg_batch_result(hg_batch* batch, int32_t slot, int32_t* part, int32_t* n_parts,
                    int32_t* n_levels);
int hg_batch_compact(hg_batch* batch);
int hg_batch_sizes(hg_batch* batch, int64_t* sizes);

/*
 * Census of the score step (Eq. 12) of the most recent hg_coarsen_level on
 * the context (synchronous): out[k] = vertices scored by work list k and
 * out[HG_SCORE_LISTS + k] = their neighbour visits (sum over incident
 * hyperedges of the hyperedge's size less one), for the lists of the bucket
 * rule described at hg_tuning: 0 single pass in the small table, 1 single
 * pass in the big table, 2 windows with a bitmap of seen ids, 3 passes over a
 * table; 4-7 the same where the distinct-axon overlap of Section 3 can bind;
 * 8 and 9 (without and with the overlap) dense windows, taken by the
 * neighbourhoods that visit at least one id in dense_ratio (hg_tuning,
 * default 8) of the level and are either large (lists 2, 3, 6, 7) or have an
 * expansion of at least 2^16, on levels of at most 2^21 vertices.  `out` is host
 * int64[2 * HG_SCORE_LISTS].
 */
#define HG_SCORE_LISTS 10
int hg_score_census(hg_ctx* ctx, int64_t* out);

/*
 * Placement of a partitioned hypergraph G_P on the cores of a lattice
 * (Section 4.2).  `gp` is the level whose vertices are the parts (nodes):
 * hg_contract of the level-0 hypergraph with the partition as its vertex
 * map gives it; only edge_offsets, pins (flags ignored) and edge_weight (the
 * spike rates eta) are read.  The lattice has width x height cores, 1 <=
 * width, height <= 64; core c sits at (x, y) = (c / height, c % height) and
 * distances are Manhattan (Section 2).  1 <= V <= width * height.
 *
 * Every call runs n_starts >= 1 placements together (the multi-start of
 * Section 4.2); per-start device arrays are start-major: core_of[s * V + p]
 * is the core of node p in start s.  All pointers are device memory owned
 * by the caller; the calls are asynchronous; an order that is not a
 * permutation, or a placement with a core outside the lattice or held by two
 * nodes, is reported by the next hg_sync (HG_ERR_INVALID_ARG) and leaves the
 * outputs undefined.
 *
 * hg_place_initial ("Initial Placement"): start s lays the nodes in the
 * order orders[s * V .. s * V + V) (a permutation of 0..V-1, the random
 * initial order), bisects the sequence recursively (a section of len nodes
 * into its first ceil(len/2) and last floor(len/2) positions) with up to
 * lp_rounds label-propagation rounds per section (gains of crossing to the
 * other half over the hyperedges cut inside the section, both halves sorted
 * by gain descending then node id, i-th pairs swapped while their gains sum
 * above 0, a section stopping after a round without swaps), folds the tree
 * (a non-root section flips, reversing its order, when its child facing
 * away from its sibling is the more connected one to that sibling; ties
 * keep the order) and places the i-th node of the result on the i-th core
 * of the lattice's Hilbert order (the curve of the smallest power-of-two
 * square holding the lattice, cores outside skipped).  Writes core_of.
 *
 * hg_place_refine ("Swap Proposals", "Placement Refinement"): rounds of
 * forces (Eq. 14) and tensions (Eq. 15) towards the four neighbour cores;
 * every occupied core proposes the neighbour of largest positive tension
 * (lowest core id on ties); proposals are matched by the rule of Eq. 13
 * over cores; the matched swaps are ordered by tension descending, then
 * lower core id; their tensions are recomputed as if the swaps before them
 * were applied, and the prefix of largest positive cumulative tension (the
 * shortest on ties) is applied.  A start stops after a round that applies
 * nothing, all after max_rounds.  core_of is updated in place (synchronous:
 * the host reads one counter per round); info (device int64[3 * n_starts])
 * = per start [rounds run, swaps applied, decrease of the residual distance].
 *
 * hg_place_residual: dist[s] (device int64[n_starts]) = sum over hyperedges
 * of eta times the Manhattan distances of all unordered pairs of their pins'
 * cores, the quantity each applied swap decreases by its recomputed tension;
 * best (device int32[1], may be NULL) = the start of least dist, lowest
 * index on ties (the multi-start choice of Section 4.2).
 */
int hg_place_initial(hg_ctx* ctx, const hg_level* gp, int32_t width, int32_t height,
                     int32_t n_starts, const int32_t* orders, int32_t lp_rounds,
                     int32_t* core_of);
int hg_place_refine(hg_ctx* ctx, const hg_level* gp, int32_t width, int32_t height,
                    int32_t n_starts, int32_t* core_of, int32_t max_rounds, int64_t* info);
int hg_place_residual(hg_ctx* ctx, const hg_level* gp, int32_t width, int32_t height,
                      int32_t n_starts, const int32_t* core_of, int64_t* dist, int32_t* best);

/*
 * Synchronous structural check of a level: offsets non-decreasing and within
 * P, ids < V and strictly ascending per hyperedge, weights and multiplicities
 * >= 1, total weight < 2^31, state values >= 0 when present (state pointers
 * may be NULL).  Returns HG_OK or HG_ERR_INVALID_LEVEL / HG_ERR_OVERFLOW.
 */
int hg_validate_level(hg_ctx* ctx, const hg_level* lvl);

#ifdef __cplusplus
}
#endif

#endif /* HG_H_ */
