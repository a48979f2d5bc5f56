#!/usr/bin/env python
"""Benchmark of one coarsening level on one MI355X.

Workload (default): the recurrent power-law SNN with 2,000,000 neurons
(out-degree ~ d^-2.1 on [20, 10000], uniform distinct targets, exponential
spike-rate weights of mean 50, 20% inhibitory neurons halved), level 0, core
limits 4096 neurons / 262,144 synapses / 16,384 axons.

A step is one pass of the whole hot path over the level resident in HBM:
hg_coarsen_level (incidence lists, scores and candidates, matching, coarse
vertex map) + hg_contract (coarse hypergraph) + hg_connectivity (Eq. 1 of
the level under the new vertex map).  `value` is pins of the level divided
by the wall time of a step.

Prints one JSON line.  See the design doc for the byte model behind `roofline`.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "pins coarsened/sec per level (1 GPU, % HBM roofline); batched vs plain; p99 ms"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "powerlaw2M": dict(
        desc=("recurrent power-law SNN: 2,000,000 neurons, out-degree d^-2.1 on [20, 10000], "
              "uniform distinct targets, exponential weights (mean 50), 20% inhibitory x0.5; "
              "limits 4096/262144/16384; level 0"),
        make=lambda synth, seed: synth.powerlaw(seed, n=2_000_000, dmin=20, dmax=10_000),
        limits="powerlaw"),
    "powerlaw200k": dict(
        desc=("recurrent power-law SNN: 200,000 neurons, out-degree d^-2.1 on [20, 10000], "
              "uniform distinct targets, exponential weights (mean 50), 20% inhibitory x0.5; "
              "limits 4096/262144/16384; level 0 (profiling size: same per-vertex work)"),
        make=lambda synth, seed: synth.powerlaw(seed, n=200_000, dmin=20, dmax=10_000),
        limits="powerlaw"),
    "conv": dict(
        desc=("convolutional SNN: 4 layers of 64x64x16, 3x3 window over all channels of the "
              "next layer; log-uniform weights 1..1000; limits 1024/65536/4096; level 0"),
        make=lambda synth, seed: synth.conv(seed),
        limits="conv"),
    "layered": dict(
        desc=("layered SNN: 4 x 1024 neurons, 64 uniform targets in the next layer; weights "
              "1..100; limits 256/16384/1024; level 0"),
        make=lambda synth, seed: synth.layered(seed),
        limits="layered"),
}


# The score kernel of each work list of the library's bucket rule (lists 4-7
# and 9 also count shared inbound axons); lists 2 and 6 use the aligned-window
# variants on levels of at most 16 windows of 2^19 ids (with 16-byte body
# loads unless the tuning's wide_loads is 0).
SCORE_KERNELS = (
    "score_block_kernel<256,4096>", "score_block_kernel<512,16384>",
    "score_window_kernel<1024>", "score_block_kernel<512,16384,multipass>",
    "score_block_kernel<256,4096,overlap>", "score_block_kernel<512,8192,overlap>",
    "score_stream_kernel<1024,8192,overlap>", "score_block_kernel<512,8192,multipass,overlap>",
    "score_dense_kernel<1024>", "score_dense_kernel<1024,overlap>",
)


def expansion_stats(g):
    """X = sum over hyperedges of |e| (|e| - 1): neighbour visits of the score step."""
    lens = np.diff(g.eoff).astype(np.int64)
    return int(np.sum(lens * (lens - 1)))


def s2_bytes(V, E, P, X):
    """Algorithmic bytes of the score/candidate step (one launch set):
    4 B per neighbour visit (pin re-read), 24 B per incidence entry (incidence
    word, offsets pair, weight, cursor), 48 B per vertex (offsets, expansion,
    state, work list, outputs)."""
    return 4 * X + 24 * P + 48 * V


def level_bytes(V, E, P, X):
    """Algorithmic bytes of a whole step (level + connectivity): the score
    step plus 48 B per pin (incidence build 8, score-side headers counted
    above, contraction 16, copy 4, connectivity 8, expansion 12), 40 B per
    hyperedge and 76 B per vertex."""
    return 4 * X + 72 * P + 40 * E + 124 * V


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(workload):
    """HBM traffic of the score kernel from committed rocprofv3 counter runs,
    if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_score_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    src = d.get("source_file", "paper_2609_07577_amd/csrc/hg_score.hip")
    cur = source_hash(os.path.join(ROOT, src))
    if d.get("source_hash") != cur:
        return None
    return d.get("bytes_per_launch")


def _edge_subset(OL, frac, rng):
    """The level restricted to a seeded fraction of its hyperedges (all
    vertices and their state kept): a sample for timing the contraction."""
    import oracle
    E = OL.E
    keep = np.sort(rng.choice(E, size=max(1, int(frac * E)), replace=False))
    lens = np.diff(OL.eoff)[keep]
    eoff = np.zeros(keep.shape[0] + 1, np.int64)
    np.cumsum(lens, out=eoff[1:])
    starts = OL.eoff[keep]
    idx = np.repeat(starts - eoff[:-1], lens) + np.arange(eoff[-1])
    return oracle.OLevel(OL.V, eoff, OL.pins[idx].copy(), OL.w[keep].copy(),
                         OL.mult[keep].copy(), OL.size, OL.syn, OL.soff, OL.sids)


def cpu_baseline(g, lim, X, P, seconds):
    """The oracle's time for the whole level, every step timed on a bounded
    sample and scaled to the level: candidates (Eq. 12) for a seeded vertex
    sample, scaled by neighbour visits; the incidence build in full;
    matching (Eq. 13) and the vertex map over all vertices, on the oracle's
    candidates of the sample (no candidate elsewhere: the step's cost is
    linear in the vertices); the contraction under that vertex map on two
    seeded hyperedge subsets (4% and 8% of the hyperedges, every vertex),
    scaled linearly in pins.  Every input is the oracle's own."""
    import oracle
    oracle.build(force=False)
    nthreads = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        nthreads = min(nthreads, int(omp))
    OL = oracle.level0(g)
    lens = np.diff(g.eoff).astype(np.int64)
    ids = (g.pins & 0x7FFFFFFF).astype(np.int64)
    edge_of_pin = np.repeat(np.arange(g.n_edges), lens)
    xn = np.bincount(ids, weights=(lens - 1)[edge_of_pin], minlength=g.n_vertices)
    del edge_of_pin, ids
    rng = np.random.default_rng(12345)
    # sample size from an a-priori cost of 14 ns per neighbour visit per thread
    # (measured on 16 host threads: 5.99e9 visits in 5.4 s)
    target_visits = seconds * nthreads / 14e-9
    n = int(min(g.n_vertices, max(64, target_visits / max(1.0, xn.mean()))))
    q = np.sort(rng.choice(g.n_vertices, n, replace=False)).astype(np.int32)
    secs = np.zeros(2, np.float64)
    t0 = time.perf_counter()
    qc, qs = oracle.candidates(OL, lim, query=q, nthreads=nthreads, seconds=secs)
    t_cand_wall = time.perf_counter() - t0
    t_setup, t_vert = float(secs[0]), max(float(secs[1]), 1e-6)
    xs = float(xn[q].sum())
    t_cand = t_vert * (X / xs)
    cand = np.full(g.n_vertices, -1, np.int32)
    cscore = np.zeros(g.n_vertices, np.int32)
    cand[q], cscore[q] = qc, qs
    t0 = time.perf_counter()
    m = oracle.match(cand, cscore)
    vmap, nc = oracle.vmap_from_match(m)
    t_match = time.perf_counter() - t0
    timed = []
    for frac in (0.04, 0.08):
        sub = _edge_subset(OL, frac, rng)
        t0 = time.perf_counter()
        oracle.contract(sub, vmap, nc)
        timed.append((sub.P, time.perf_counter() - t0))
    (p1, t1), (p2, t2) = timed
    slope = max(0.0, (t2 - t1) / max(1, p2 - p1))
    t_contract = max(t2, t2 + slope * (P - p2))
    t_level = t_setup + t_cand + t_match + t_contract
    return {
        "value": P / t_level, "unit": "pins/s", "cores": nthreads, "kind": "oracle",
        "seconds_per_level": t_level,
        "phases_s": {"incidence": t_setup, "candidates": t_cand, "match": t_match,
                     "contract": t_contract},
        "sample": (f"oracle level 0 scaled from samples: candidates of {n} seeded vertices "
                   f"({xs:.3g} of {X:.3g} neighbour visits, {t_cand_wall:.1f} s incl. "
                   f"{t_setup:.1f} s incidence build) scaled by visits to {t_cand:.0f} s; "
                   f"matching and vertex map over all vertices (on the sample's candidates) "
                   f"{t_match:.1f} s; contraction of "
                   f"{p1} and {p2} pins ({t1:.1f} s, {t2:.1f} s) scaled linearly to {P} pins: "
                   f"{t_contract:.0f} s; {t_level:.0f} s per level on {nthreads} threads "
                   f"(candidate step parallel, the rest sequential)"),
    }


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _pack(sizes, cap_pins, vsizes=None, cap_vertices=None):
    """Consecutive groups whose pin totals stay within cap_pins (and vertex
    totals within cap_vertices)."""
    groups, cur, tot, vtot = [], [], 0, 0
    for i, p in enumerate(sizes):
        v = vsizes[i] if vsizes is not None else 0
        if cur and (tot + p > cap_pins or (cap_vertices and vtot + v > cap_vertices)):
            groups.append(cur)
            cur, tot, vtot = [], 0, 0
        cur.append(i)
        tot += p
        vtot += v
    if cur:
        groups.append(cur)
    return groups


def run_batch(args):
    """The mixed batch: 256 graphs, feed-forward or recurrent by a fair coin,
    neuron count log-uniform in [10k, 500k), fan-out U{16..256}, weights
    U{1..100}, limits 512/32768/2048 per graph.

    (a) one level of every graph, batched (graphs packed into unions of at
    most 2^21 vertices and below 2^31 pins, one union step each) vs plain (hg_coarsen_level + hg_contract
    per graph); the score-step tuning is autotuned first and used by both;
    (b) whole hierarchies of two size-scaled copies of the distribution
    (neurons in [1k, 20k) with the full fan-out range, and [500, 5000) with
    fan-out 8..32), batched with the level step replayed from a HIP graph vs
    plain level-by-level runs, with every partition compared; (c) with
    --full-hier-graphs N, the same for N graphs of the mix at full size (a
    graph needs 100-260 contractions, so the whole batch of 256 is out of
    reach of one run)."""
    import torch
    from paper_2609_07577_amd import hg, hierarchy, synth, tune

    lim = synth.LIMITS["batch"]
    ctx = hg.Context(0)
    # ---- (a) full size, one level -------------------------------------------
    t0 = time.perf_counter()
    levels = []
    X_total = 0
    bytes_level = 0
    for k in range(args.graphs):
        g = synth.batch_graph(args.seed, k)
        xg = int(expansion_stats(g))
        X_total += xg
        bytes_level += level_bytes(g.n_vertices, g.n_edges, g.n_pins, xg)
        levels.append(ctx.upload(g))
        if k % 32 == 31:
            ctx.sync()
            _log(f"generated and uploaded {k + 1} graphs")
    ctx.sync()
    V = sum(L.V for L in levels)
    E = sum(L.E for L in levels)
    P = sum(L.P for L in levels)
    _log(f"{args.graphs} graphs: V={V} E={E} P={P} ({time.perf_counter() - t0:.1f} s)")
    sample = sorted(range(len(levels)), key=lambda i: levels[i].P)[:: max(1, len(levels) // 6)]
    tuned = tune.autotune(ctx, [levels[i] for i in sample], [lim] * len(sample), verbose=True)
    _log(f"tuning: {tuned['single_pass_load16']}/{tuned['pass_fill16']}/{tuned['dense_ratio']}")

    def plain_level():
        for L in levels:
            out = ctx.coarsen_level(L, lim, want_candidates=False)
            ctx.contract(L, out["vmap"], out["n_coarse"], trim=False)

    plain_level()  # warm-up
    ctx.sync()
    t0 = time.perf_counter()
    plain_level()
    ctx.sync()
    t_plain = time.perf_counter() - t0
    _log(f"plain: one level of {len(levels)} graphs in {t_plain:.3f} s")

    # unions of at most 2^21 vertices, the largest level the dense score
    # windows cover (and below 2^31 pins)
    groups = _pack([L.P for L in levels], (1 << 31) - 1, [L.V for L in levels], 1 << 21)
    capV = max(sum(levels[i].V for i in gr) for gr in groups)
    capE = max(sum(levels[i].E for i in gr) for gr in groups)
    capP = max(sum(levels[i].P for i in gr) for gr in groups)
    t_batch = 0.0
    for rep in range(2):  # first pass is the warm-up
        t_batch = 0.0
        for gr in groups:
            B = hg.Batch(ctx, len(gr), capV, capE, capP)
            ctx.sync()
            t0 = time.perf_counter()
            for i in gr:
                B.add(levels[i], lim)
            B.step(1, use_graph=False)
            ctx.sync()
            t_batch += time.perf_counter() - t0
            B.close()
    ctx.sync()
    _log(f"batched: one level in {len(groups)} unions in {t_batch:.3f} s")
    del levels
    torch.cuda.empty_cache()

    # ---- (b) size-scaled, whole hierarchies ----------------------------------
    def hierarchies(name, n_min, n_max, fan_min, fan_max, seed):
        levels_h = []
        for k in range(args.hier_graphs):
            g = synth.batch_graph(seed, k, n_min=n_min, n_max=n_max, fan_min=fan_min,
                                  fan_max=fan_max)
            levels_h.append(ctx.upload(g))
        ctx.sync()
        hP = sum(L.P for L in levels_h)
        t0 = time.perf_counter()
        plain_res = []
        for k, L in enumerate(levels_h):
            vmaps, nlev, last = hierarchy.plain_hierarchy(ctx, L, lim)
            plain_res.append((vmaps, nlev, last.V))
            if k % 16 == 15:
                _log(f"{name}: plain hierarchies {k + 1} done")
        ctx.sync()
        t_p = time.perf_counter() - t0
        hierarchy.batched_hierarchies(ctx, levels_h[:4], [lim] * 4)  # warm-up (capture)
        ctx.sync()
        t0 = time.perf_counter()
        batch_res = hierarchy.batched_hierarchies(ctx, levels_h, [lim] * len(levels_h))
        ctx.sync()
        t_b = time.perf_counter() - t0
        equal, total_levels = True, 0
        for (vmaps, nlev, nparts), (part, bparts, blev), L in zip(plain_res, batch_res, levels_h):
            ref = hierarchy.compose(vmaps, L.V, ctx.device)
            equal &= bool(torch.equal(ref, part)) and nparts == bparts and nlev == blev
            total_levels += nlev
        _log(f"{name}: {len(levels_h)} hierarchies, plain {t_p:.2f} s, batched {t_b:.2f} s, "
             f"identical={equal}")
        return {
            "workload": ("%d graphs of the mix with neurons log-uniform in [%d, %d), fan-out "
                         "U{%d..%d}, coarsened to the end" % (len(levels_h), n_min, n_max,
                                                              fan_min, fan_max)),
            "pins": hP, "contractions": total_levels,
            "plain_s": t_p, "batched_s": t_b, "batched_vs_plain": t_p / t_b,
            "plain_pins_per_s": hP / t_p, "batched_pins_per_s": hP / t_b,
            "identical_partitions": equal,
        }

    hier_mid = hierarchies("mid", 1000, 20000, 16, 256, args.seed + 1000)
    hier_small = hierarchies("small", 500, 5000, 8, 32, args.seed + 1100)
    hier_full = None
    if args.full_hier_graphs:
        saved = args.hier_graphs
        args.hier_graphs = args.full_hier_graphs
        hier_full = hierarchies("full", 10000, 500000, 16, 256, args.seed + 1200)
        args.hier_graphs = saved
    result = {
        "metric": METRIC,
        "value": P / t_batch,
        "unit": "pins/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": 1000.0 * t_batch,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": ("batch of %d SNN hypergraphs: feed-forward (4 layers) or "
                                "recurrent by a fair coin, neurons log-uniform in [10k, 500k), "
                                "fan-out U{16..256}, weights U{1..100}; limits 512/32768/2048; "
                                "level 0" % args.graphs),
                   "seed": args.seed, "vertices": V, "hyperedges": E, "pins": P,
                   "unions": len(groups)},
        "plain_pins_per_s": P / t_plain,
        "batched_vs_plain": t_plain / t_batch,
        "neighbour_visits": X_total,
        "level_algorithmic_bytes": bytes_level,
        "level_hbm_frac_batched": bytes_level / t_batch / 1e9 / HBM_PEAK_GBS,
        "level_hbm_frac_plain": bytes_level / t_plain / 1e9 / HBM_PEAK_GBS,
        "tuning": {k: tuned[k] for k in ("single_pass_load16", "pass_fill16", "dense_ratio")},
        "hierarchies_mid": hier_mid,
        "hierarchies_small": hier_small,
        "hierarchies_full_size": hier_full,
    }
    ctx.sync()
    print(json.dumps(result), flush=True)


def run_hierarchy(args):
    """The whole hierarchy of one workload (default: the 2M-neuron recurrent
    level): hg_coarsen_level + hg_contract until no vertex proposes a
    candidate (Section 4.1 stop rule).  At every level Eq. 1 is evaluated two
    ways and must agree: on the coarse level under the identity (closed form
    sum of w(e)(|e| - 1)) and on the original level under the composed
    vertex map (hg_connectivity over all original pins).  Reports the level
    count, levels/s, hierarchy pins/s (sum of P_in over the levels / total
    time of the coarsening steps) and a per-level table."""
    import torch
    from paper_2609_07577_amd import hg, synth

    wl = WORKLOADS[args.workload]
    lim = synth.LIMITS[wl["limits"]]
    g = wl["make"](synth, args.seed)
    ctx = hg.Context(0)
    L0 = ctx.upload(g)
    ctx.sync()
    _log(f"{args.workload}: V={g.n_vertices} E={g.n_edges} P={g.n_pins}; coarsening to the end")
    L = L0
    part = torch.arange(g.n_vertices, dtype=torch.int32, device="cuda")
    rows, t_total, pins_total, all_equal = [], 0.0, 0, True
    t_start = time.perf_counter()
    anyc = 1
    while True:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.coarsen_level(L, lim, want_candidates=False)
        anyc = int(out["any_candidate"].item())
        C = ctx.contract(L, out["vmap"], out["n_coarse"]) if anyc else None
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_total += dt
        pins_total += L.P
        row = {"level": len(rows), "V": L.V, "E": L.E, "P": L.P, "ms": 1000.0 * dt}
        if anyc:
            part = out["vmap"][part.long()].contiguous()
            lens = (C.eoff[1:] - C.eoff[:-1]).to(torch.int64)
            closed = int(torch.sum(C.w.to(torch.int64) * (lens - 1)).item())
            full = int(ctx.connectivity(L0, part).item())
            ctx.sync()
            row.update(conn=closed, conn_equal=closed == full)
            all_equal &= closed == full
        rows.append(row)
        if len(rows) % 10 == 1 or not anyc:
            _log(f"level {row['level']}: V={L.V} E={L.E} P={L.P} {row['ms']:.1f} ms "
                 f"conn={row.get('conn')} equal={row.get('conn_equal')}")
        if not anyc:
            break
        if args.time_limit and time.perf_counter() - t_start > args.time_limit:
            _log(f"time limit reached after {len(rows)} levels; reporting them")
            break
        L = C
    finished = not anyc
    n_contract = len(rows) - 1 if finished else len(rows)
    result = {
        "metric": METRIC,
        "value": pins_total / t_total,
        "unit": "pins/s",
        "n_gpus": 1, "steps": len(rows), "warmup": 0,
        "ms_per_step": 1000.0 * t_total / len(rows),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": wl["desc"].replace("; level 0", "") + "; whole hierarchy",
                   "seed": args.seed, "vertices": g.n_vertices, "hyperedges": g.n_edges,
                   "pins": g.n_pins},
        "contractions": n_contract,
        "finished": finished,
        "levels_per_s": len(rows) / t_total,
        "hierarchy_s": t_total,
        "final_parts": rows[-1]["V"],
        "conn_two_ways_equal_every_level": all_equal,
        "levels": rows,
    }
    print(json.dumps(result), flush=True)


def run_partition(args):
    """The whole partitioner on one workload (Section 4.1): the coarsening
    hierarchy with every level kept on the device, then the uncoarsening
    (projection of the final super-nodes and refinement rounds, level by
    level down to level 0), then the partition report of level 0 (Eq. 1 and
    the parts' totals against the limits).  Reports the time of both phases,
    Eq. 1 of the final super-nodes and after refinement, and per level the
    rounds and the decrease."""
    import torch
    from paper_2609_07577_amd import hg, hierarchy, synth

    wl = WORKLOADS[args.workload]
    lim = synth.LIMITS[wl["limits"]]
    g = wl["make"](synth, args.seed)
    ctx = hg.Context(0)
    L0 = ctx.upload(g)
    ctx.sync()
    _log(f"{args.workload}: V={g.n_vertices} E={g.n_edges} P={g.n_pins}; partitioning")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    levels, maps = hierarchy.hierarchy_levels(ctx, L0, lim)
    torch.cuda.synchronize()
    t_coarsen = time.perf_counter() - t0
    _log(f"coarsening: {len(maps)} contractions in {t_coarsen:.2f} s; {levels[-1].V} parts")
    t0 = time.perf_counter()
    part, n_parts, trace = hierarchy.uncoarsen(ctx, levels, maps, lim, args.rounds)
    torch.cuda.synchronize()
    t_uncoarsen = time.perf_counter() - t0
    rep = ctx.partition_report(L0, part, torch.tensor([n_parts], dtype=torch.int32,
                                                      device="cuda"), lim, per_part=False)
    _log(f"uncoarsening: {t_uncoarsen:.2f} s; Eq. 1 {trace[0][1]} -> {trace[-1][2]}")
    pins_total = sum(L.P for L in levels)
    result = {
        "metric": METRIC,
        "value": pins_total / (t_coarsen + t_uncoarsen),
        "unit": "pins/s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1000.0 * (t_coarsen + t_uncoarsen),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": wl["desc"].replace("; level 0", "") +
                   "; coarsening, uncoarsening and refinement",
                   "seed": args.seed, "vertices": g.n_vertices, "hyperedges": g.n_edges,
                   "pins": g.n_pins, "max_rounds": args.rounds},
        "contractions": len(maps),
        "parts": n_parts,
        "coarsen_s": t_coarsen,
        "uncoarsen_s": t_uncoarsen,
        "conn_final_supernodes": trace[0][1],
        "conn_refined": trace[-1][2],
        "refinement_gain_pct": 100.0 * (trace[0][1] - trace[-1][2]) / max(1, trace[0][1]),
        "level0_report": {k: rep[k] for k in ("conn", "max_size", "max_syn", "max_axons",
                                              "over_neurons", "over_synapses", "over_axons",
                                              "n_parts")},
        "levels": [{"level": li, "conn_projected": b, "conn_refined": a_, "rounds": r}
                   for li, b, a_, r in trace],
    }
    print(json.dumps(result), flush=True)


def run_place(args):
    """Multi-start placement (Section 4.2) of a partitioned network: G_P of
    --workload under a partition into --parts blocks of consecutive neuron
    ids (contracted on the device), placed on a --lattice x --lattice core
    lattice from --starts seeded random orders: initial placements,
    refinement to the end, residual distances and the best start.  Reports
    the time of each phase and per refinement round, and the residual
    distance before and after refinement."""
    import torch
    from paper_2609_07577_amd import hg, synth

    wl = WORKLOADS[args.workload]
    g = wl["make"](synth, args.seed)
    V0 = g.n_vertices
    ctx = hg.Context(0)
    L0 = ctx.upload(g)
    k = args.parts
    part = (torch.arange(V0, dtype=torch.int64, device="cuda") * k // V0).to(torch.int32)
    gp = ctx.contract(L0, part, torch.tensor([k], dtype=torch.int32, device="cuda"))
    ctx.sync()
    del L0
    W = H = args.lattice
    _log(f"{args.workload}: G_P of {k} parts: E={gp.E} P={gp.P}; {args.starts} starts on "
         f"{W} x {H}")
    orders = torch.from_numpy(synth.start_orders(args.seed + 1, k, args.starts)).cuda()
    for i in range(args.warmup):  # untimed: one whole placement
        core = ctx.place_initial(gp, W, H, orders, args.lp_rounds)
        ctx.place_refine(gp, W, H, core, args.max_place_rounds)
        ctx.place_residual(gp, W, H, core)
        ctx.sync()
        _log(f"warmup {i} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    core = ctx.place_initial(gp, W, H, orders, args.lp_rounds)
    ctx.sync()
    t1 = time.perf_counter()
    d0, _ = ctx.place_residual(gp, W, H, core)
    d0 = d0.cpu()
    t2 = time.perf_counter()
    info = ctx.place_refine(gp, W, H, core, args.max_place_rounds)
    ctx.sync()
    t3 = time.perf_counter()
    d1, best = ctx.place_residual(gp, W, H, core)
    ctx.sync()
    t4 = time.perf_counter()
    info = info.cpu().numpy()
    d1 = d1.cpu()
    b = int(best.item())
    rounds = int(info[:, 0].max())
    t_init, t_ref, t_res = t1 - t0, t3 - t2, (t2 - t1) + (t4 - t3)
    total = t_init + t_ref + (t4 - t3)
    _log(f"initial {t_init * 1e3:.1f} ms, refinement {t_ref * 1e3:.1f} ms in {rounds} rounds, "
         f"residual {t_res * 1e3:.1f} ms; best start {b}: D {int(d0[b])} -> {int(d1[b])}")
    result = {
        "metric": "multi-start placement time (initial placement, swap refinement to the end, "
                  "residual distances and choice)",
        "value": 1000.0 * total, "unit": "ms",
        "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": 1000.0 * total,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": wl["desc"].replace("; level 0", "") +
                   f"; G_P of {k} parts of consecutive neuron ids; {W} x {H} lattice; "
                   f"{args.starts} starts",
                   "seed": args.seed, "parts": k, "gp_hyperedges": gp.E, "gp_pins": gp.P,
                   "lattice": [W, H], "starts": args.starts, "lp_rounds": args.lp_rounds},
        "initial_ms": 1000.0 * t_init,
        "refine_ms": 1000.0 * t_ref,
        "residual_ms": 1000.0 * t_res,
        "rounds_max": rounds,
        "ms_per_round": 1000.0 * t_ref / max(1, rounds),
        "swaps_applied": int(info[:, 1].sum()),
        "best_start": b,
        "residual_initial_best": int(d0[b]),
        "residual_refined_best": int(d1[b]),
        "residual_refined_min_max": [int(d1.min()), int(d1.max())],
        "refinement_decrease_pct": 100.0 * float(d0[b] - d1[b]) / max(1, int(d0[b])),
    }
    print(json.dumps(result), flush=True)


def run_serve(args):
    """Served requests: Poisson arrivals at --rate per second for --duration
    seconds.  A request is one SNN hypergraph to coarsen to the end, drawn
    from a pool of 1024 graphs of the batch mix scaled down to neurons in
    [500, 5000) and fan-out 8..32 (98%) plus 2% such graphs of 20,000
    neurons, all resident on the device; with --mix full, from 64 graphs of
    the full-size mix (neurons in [10k, 500k), fan-out 16..256) plus 2%
    graphs of 2,000,000 neurons, served until --serve-wall seconds at most,
    the backlog then reported.  (A request of the full-size mix
    costs 0.3-40 GPU-seconds, so a 200/s stream of them cannot be served by
    one GPU; the scaled mix keeps the offered load below capacity.)  Requests are admitted by footprint into one
    batch (continuous batching) and stepped 4 levels per union step from a
    captured HIP graph.  Latency = finish - arrival.  Every served partition
    of a seeded sample is compared with a plain run of the same graph."""
    import numpy as np
    import torch
    from paper_2609_07577_amd import hg, hierarchy, serve, synth

    ctx = hg.Context(0)
    rng = np.random.default_rng(args.seed)
    pool, lims = [], []
    full = args.mix == "full"
    n_small, n_big = (64, 2) if full else (1024, 8)
    for k in range(n_small):
        if full:
            g = synth.batch_graph(args.seed + 2000, k)
        else:
            g = synth.batch_graph(args.seed + 2000, k, n_min=500, n_max=5000, fan_min=8,
                                  fan_max=32)
        pool.append(ctx.upload(g))
        lims.append(synth.LIMITS["batch"])
    for k in range(n_big):
        if full:
            g = synth.batch_graph(args.seed + 3000, k, n_min=2_000_000, n_max=2_000_001)
        else:
            g = synth.batch_graph(args.seed + 3000, k, n_min=20000, n_max=20001, fan_min=8,
                                  fan_max=32)
        pool.append(ctx.upload(g))
        lims.append(synth.LIMITS["batch"])
    ctx.sync()
    _log(f"request pool: {len(pool)} graphs on the device")
    n_req = int(rng.poisson(args.rate * args.duration))
    arrivals = np.sort(rng.uniform(0.0, args.duration, n_req))
    big = rng.random(n_req) < 0.02
    which = np.where(big, n_small + rng.integers(0, n_big, n_req),
                     rng.integers(0, n_small, n_req))
    if full:
        srv = serve.Server(ctx, max_graphs=256, cap_vertices=1 << 21, cap_edges=4_000_000,
                           cap_pins=640_000_000, levels_per_step=4, use_graph=True)
    else:
        srv = serve.Server(ctx, max_graphs=1024, cap_vertices=2_000_000, cap_edges=2_000_000,
                           cap_pins=64_000_000, levels_per_step=4, use_graph=True)
    # warm-up: capture and first launches
    srv.submit(-1, pool[0], lims[0], time.perf_counter())
    while not srv.idle():
        srv.step()
    ctx.sync()
    _log(f"serving {n_req} requests over {args.duration:.0f} s")
    lat, pins_done, served = [], 0, {}
    t0 = time.perf_counter()
    nxt = 0
    last_log = t0
    stopped = False
    while nxt < n_req or not srv.idle():
        now = time.perf_counter() - t0
        if args.serve_wall and now > args.serve_wall:
            stopped = True
            _log(f"wall limit: {len(lat)} served, {n_req - nxt} not yet arrived, "
                 f"{len(srv.queue)} queued, {len(srv.running)} running")
            break
        while nxt < n_req and arrivals[nxt] <= now:
            srv.submit(nxt, pool[which[nxt]], lims[which[nxt]], t0 + arrivals[nxt])
            nxt += 1
        for rid, arr, fin, part, n_parts, n_levels, pins in srv.step():
            lat.append(fin - arr)
            pins_done += pins
            if rid % 97 == 0:
                served[rid] = (part, n_parts, n_levels)
        if srv.idle() and nxt < n_req:
            time.sleep(max(0.0, min(0.005, arrivals[nxt] - (time.perf_counter() - t0))))
        if time.perf_counter() - last_log > 10:
            last_log = time.perf_counter()
            _log(f"t={last_log - t0:.0f} s: {len(lat)} served, {len(srv.queue)} queued, "
                 f"{len(srv.running)} running")
    wall = time.perf_counter() - t0
    backlog = {"not_arrived": int(n_req - nxt), "queued": len(srv.queue),
               "running": len(srv.running)}
    ctx.sync()
    # the same graphs alone, plain
    equal = True
    for rid, (part, n_parts, n_levels) in served.items():
        L = pool[which[rid]]
        vmaps, nlev, last = hierarchy.plain_hierarchy(ctx, L, lims[which[rid]])
        ref = hierarchy.compose(vmaps, L.V, ctx.device)
        equal &= bool(torch.equal(ref, part)) and nlev == n_levels and last.V == n_parts
    # plain service capacity on a sample of the stream (small requests only
    # for the full mix: one 2M-neuron request alone takes minutes)
    cand = np.flatnonzero(~big) if full else np.arange(n_req)
    sample = [int(x) for x in rng.choice(cand, size=min(24 if not full else 8, len(cand)),
                                         replace=False)]
    ctx.sync()
    t1 = time.perf_counter()
    for r in sample:
        hierarchy.plain_hierarchy(ctx, pool[which[r]], lims[which[r]], keep_maps=False)
    ctx.sync()
    t_plain_req = (time.perf_counter() - t1) / len(sample)
    lat_ms = np.array(lat) * 1000.0
    batch_bytes = srv.bytes()
    srv.close()
    result = {
        "metric": METRIC,
        "value": pins_done / wall,
        "unit": "pins/s",
        "n_gpus": 1,
        "steps": len(lat),
        "warmup": 1,
        "ms_per_step": 1000.0 * wall / max(1, len(lat)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": (("served mapping requests, Poisson %g/s for %.0f s: 98%% "
                                 "batch-mix graphs with neurons log-uniform in [10k, 500k) and "
                                 "fan-out U{16..256}, 2%% such graphs of 2,000,000 neurons; "
                                 "limits 512/32768/2048; each coarsened to the end"
                                 % (args.rate, args.duration)) if full else
                                ("served mapping requests, Poisson %g/s for %.0f s: 98%% "
                                 "batch-mix graphs with neurons log-uniform in [500, 5000) and "
                                 "fan-out U{8..32}, 2%% such graphs of 20,000 neurons; limits "
                                 "512/32768/2048; each coarsened to the end"
                                 % (args.rate, args.duration))),
                   "requests": n_req, "seed": args.seed, "batch_bytes": batch_bytes},
        "p50_ms": float(np.percentile(lat_ms, 50)) if len(lat_ms) else None,
        "p99_ms": float(np.percentile(lat_ms, 99)) if len(lat_ms) else None,
        "served_per_s": len(lat) / wall,
        "plain_mean_service_ms": 1000.0 * t_plain_req,
        "plain_capacity_per_s": 1.0 / t_plain_req,
        "served_equal_to_alone": equal,
        "checked": len(served),
        "stopped_at_wall_limit": stopped,
        "backlog_at_end": backlog,
        "big_requests": int(big.sum()),
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="powerlaw2M", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--start-level", type=int, default=0,
                    help="level mode: time this level of the hierarchy (the levels before it "
                         "are coarsened first, untimed)")
    ap.add_argument("--time-limit", type=float, default=0.0,
                    help="hierarchy mode: stop after this many seconds and report the levels "
                         "done (0: run to the stop rule)")
    ap.add_argument("--rounds", type=int, default=16,
                    help="partition mode: refinement rounds per level at most")
    ap.add_argument("--mode", default="level",
                    choices=("level", "hierarchy", "partition", "place", "batch", "serve"),
                    help="level: one coarsening level of one graph (default); hierarchy: the "
                         "whole hierarchy of --workload with Eq. 1 checked two ways per level; "
                         "partition: coarsening, uncoarsening and refinement of --workload; "
                         "place: multi-start placement of G_P of --workload; "
                         "batch: the 256-graph batch, batched vs plain; serve: continuous "
                         "batching of Poisson-arriving requests")
    ap.add_argument("--parts", type=int, default=4096, help="place mode: parts of G_P")
    ap.add_argument("--lattice", type=int, default=64, help="place mode: lattice side")
    ap.add_argument("--starts", type=int, default=64, help="place mode: multi-start count")
    ap.add_argument("--lp-rounds", type=int, default=4,
                    help="place mode: label-propagation rounds per section")
    ap.add_argument("--max-place-rounds", type=int, default=1000,
                    help="place mode: refinement rounds at most")
    ap.add_argument("--graphs", type=int, default=256, help="batch mode: graphs at full size")
    ap.add_argument("--hier-graphs", type=int, default=64,
                    help="batch mode: graphs of the size-scaled full-hierarchy comparison")
    ap.add_argument("--full-hier-graphs", type=int, default=0,
                    help="batch mode: graphs of the mix at full size coarsened to the end, "
                         "batched vs plain (0: skipped)")
    ap.add_argument("--rate", type=float, default=200.0, help="serve mode: requests per second")
    ap.add_argument("--mix", default="scaled", choices=("scaled", "full"),
                    help="serve mode: request sizes (scaled-down mix, or the full-size mix "
                         "with 2%% of 2M-neuron graphs)")
    ap.add_argument("--serve-wall", type=float, default=0.0,
                    help="serve mode: stop serving after this many seconds and report the "
                         "backlog (0: serve every request)")
    ap.add_argument("--duration", type=float, default=60.0, help="serve mode: seconds of arrivals")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (5 times), the "
                         "reference kernel for scaling the FETCH_SIZE/WRITE_SIZE counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.arange(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "launches": 5}), flush=True)
        return

    if args.mode == "batch":
        run_batch(args)
        return
    if args.mode == "serve":
        run_serve(args)
        return
    if args.mode == "hierarchy":
        run_hierarchy(args)
        return
    if args.mode == "partition":
        run_partition(args)
        return
    if args.mode == "place":
        run_place(args)
        return

    from paper_2609_07577_amd import hg, synth

    wl = WORKLOADS[args.workload]
    lim = synth.LIMITS[wl["limits"]]
    t0 = time.perf_counter()
    g = wl["make"](synth, args.seed)
    t_gen = time.perf_counter() - t0
    V, E, P = g.n_vertices, g.n_edges, g.n_pins
    X = expansion_stats(g)
    print(f"[bench] {args.workload}: V={V} E={E} P={P} X={X:.4g} (generated in {t_gen:.1f} s)",
          file=sys.stderr, flush=True)

    ctx = hg.Context(0)
    L = ctx.upload(g)
    ctx.sync()
    for k in range(args.start_level):  # coarser levels of the same hierarchy
        out = ctx.coarsen_level(L, lim, want_candidates=False)
        L = ctx.contract(L, out["vmap"], out["n_coarse"])
        print(f"[bench] level {k + 1}: V={L.V} E={L.E} P={L.P}", file=sys.stderr, flush=True)
    if args.start_level:
        V, E, P = L.V, L.E, L.P
        h = L.to_host()
        lens = np.diff(h["eoff"]).astype(np.int64)
        X = int(np.sum(lens * (lens - 1)))
        del h
    ctx.enable_timing(True)

    def step():
        out = ctx.coarsen_level(L, lim, want_candidates=False)
        ctx.contract(L, out["vmap"], out["n_coarse"], trim=False)
        conn = ctx.connectivity(L, out["vmap"])
        return out, conn

    for i in range(args.warmup):
        step()
        ctx.sync()
        ctx.phase_times()
        print(f"[bench] warmup step {i} done", file=sys.stderr, flush=True)

    phases = {k: 0.0 for k in hg.PHASES}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out, conn = step()
        pt = ctx.phase_times()  # synchronises the stream
        for k, v in pt.items():
            phases[k] += v
        print(f"[bench] step {i}: " + " ".join(f"{k}={v:.1f}ms" for k, v in pt.items()),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()  # raises if any kernel reached an internal bound
    ms_step = 1000.0 * wall / args.steps
    for k in phases:
        phases[k] /= args.steps
    print(f"[bench] {args.steps} steps, {ms_step:.1f} ms/step, phases {phases}",
          file=sys.stderr, flush=True)

    # invariant check on the last step: Eq. (1) of level 0 under the new map
    # equals the closed form on the coarse level
    C = ctx.contract(L, out["vmap"], out["n_coarse"], trim=True)
    lens = (C.eoff[1:] - C.eoff[:-1]).to(torch.int64)
    conn_coarse = int(torch.sum(C.w.to(torch.int64) * (lens - 1)).item())
    conn_ok = conn_coarse == int(conn.item())

    # the score kernel that carried most neighbour visits on this level (from
    # the library's census of its work lists)
    n_by_list, visits_by_list = ctx.score_census()
    top = int(np.argmax(visits_by_list))
    kernel = SCORE_KERNELS[top]
    if top in (2, 6) and V <= (16 << 19):  # aligned windows (pins of torch tensors: 16-byte aligned)
        wide = ctx.get_tuning()["wide_loads"]
        kernel = "%s<1024%s>" % ("score_wide_kernel" if wide else "score_window2_kernel",
                                 ",overlap" if top == 6 else "")
    value = P / (ms_step / 1000.0)
    b_s2 = s2_bytes(V, E, P, X)
    t_s2 = phases["score"] / 1000.0
    achieved = b_s2 / t_s2 / 1e9 if t_s2 > 0 else 0.0
    traffic = read_traffic(args.workload)
    b_level = level_bytes(V, E, P, X)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "pins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wl["desc"].replace("level 0", f"level {args.start_level}"),
                   "seed": args.seed, "vertices": V, "hyperedges": E,
                   "pins": P, "neighbour_visits": X, "coarse_vertices": C.V,
                   "coarse_hyperedges": C.E, "coarse_pins": C.P},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel + " (Eq. 12 scores and candidates)",
                     "kernel_visit_share": visits_by_list[top] / max(1, sum(visits_by_list)),
                     "algorithmic_bytes": b_s2, "ms_per_launch": phases["score"]},
        "score_work_lists": {"vertices": n_by_list, "visits": visits_by_list},
        "level_hbm_frac": b_level / (ms_step / 1000.0) / 1e9 / HBM_PEAK_GBS,
        "phases_ms": phases,
        "levels_per_s": 1000.0 / ms_step,
        "scratch_bytes": ctx.scratch_bytes(),
        "conn_invariant_ok": conn_ok,
    }
    if not args.no_cpu_baseline and args.start_level == 0:
        print("[bench] timing the CPU oracle on samples of every step", file=sys.stderr,
              flush=True)
        result["cpu_baseline"] = cpu_baseline(g, lim, X, P, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
