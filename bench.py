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
    cur = source_hash(os.path.join(ROOT, "paper_2609_07577_amd", "csrc", "hg_score.hip"))
    if d.get("source_hash") != cur:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(g, lim, X, P, seconds):
    """The oracle's candidate step (the whole level's dominant cost) on a
    seeded vertex sample, extrapolated to the level by neighbour visits."""
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
    rng = np.random.default_rng(12345)
    # sample size from an a-priori cost of 14 ns per neighbour visit per thread
    # (measured on 16 host threads: 5.99e9 visits in 5.4 s)
    target_visits = seconds * nthreads / 14e-9
    n = int(min(g.n_vertices, max(64, target_visits / max(1.0, xn.mean()))))
    q = np.sort(rng.choice(g.n_vertices, n, replace=False)).astype(np.int32)
    secs = np.zeros(2, np.float64)
    t0 = time.perf_counter()
    oracle.candidates(OL, lim, query=q, nthreads=nthreads, seconds=secs)
    t = time.perf_counter() - t0
    t_setup, t_vert = float(secs[0]), max(float(secs[1]), 1e-6)
    xs = float(xn[q].sum())
    t_level = t_setup + t_vert * (X / xs)
    return {
        "value": P / t_level, "unit": "pins/s", "cores": nthreads, "kind": "oracle",
        "sample": (f"oracle candidate step for {n} seeded level-0 vertices "
                   f"({xs:.3g} of {X:.3g} neighbour visits) in {t:.1f} s incl. "
                   f"{t_setup:.1f} s incidence build, extrapolated by visits to "
                   f"{t_level:.0f} s per level; matching/contraction (O(P)) not timed"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="powerlaw2M", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
        "config": {"workload": wl["desc"], "seed": args.seed, "vertices": V, "hyperedges": E,
                   "pins": P, "neighbour_visits": X, "coarse_vertices": C.V,
                   "coarse_hyperedges": C.E, "coarse_pins": C.P},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "score_stream_kernel<1024,16384,false> (Eq. 12 scores and candidates)",
                     "algorithmic_bytes": b_s2, "ms_per_launch": phases["score"]},
        "level_hbm_frac": b_level / (ms_step / 1000.0) / 1e9 / HBM_PEAK_GBS,
        "phases_ms": phases,
        "levels_per_s": 1000.0 / ms_step,
        "scratch_bytes": ctx.scratch_bytes(),
        "conn_invariant_ok": conn_ok,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a vertex sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(g, lim, X, P, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
