"""Autotuner of the score-step settings (``hg_tuning``).

The score step (Eq. 12) scores a vertex in one pass over an on-chip table
when its distinct-neighbour bound is at most ``single_pass_load16``/16 of
the table, in dense windows when its visits cover at least one id in
``dense_ratio`` of the level, and in windows of neighbour ids otherwise (in
passes over a table aimed at ``pass_fill16``/16 of it where the
distinct-axon overlap can bind); on levels with aligned windows the long
slices are read 16 bytes per lane unless ``wide_loads`` is 0.
Results never depend on these settings; the best ones depend on the degree
and hyperedge-size mix of the workload.
``autotune`` times one coarsening level of sample levels under each
candidate setting and keeps the fastest.
"""
from __future__ import annotations

import itertools
import sys
import time

import torch

LOADS = (4, 8, 12)
FILLS = (3, 5, 8)
DENSE = (4, 8, 16)


def time_levels(ctx, levels, limits, repeats: int = 1) -> float:
    """Seconds for one hg_coarsen_level of every level in ``levels``."""
    best = float("inf")
    for _ in range(repeats):
        ctx.sync()
        t0 = time.perf_counter()
        for L, lim in zip(levels, limits):
            ctx.coarsen_level(L, lim, want_candidates=False)
        ctx.sync()
        best = min(best, time.perf_counter() - t0)
    return best


def autotune(ctx, levels, limits, loads=LOADS, fills=FILLS, dense=DENSE,
             verbose=False) -> dict:
    """Set and return the fastest tuning for ``levels`` (device levels with
    state) under ``limits`` (one per level)."""
    results = []
    for load, fill, dr in itertools.product(loads, fills, dense):
        ctx.set_tuning(load, fill, dr)
        time_levels(ctx, levels, limits)  # warm-up (first launch, caches)
        t = time_levels(ctx, levels, limits, repeats=2)
        results.append((t, load, fill, dr))
        if verbose:
            print(f"[tune] load16={load} fill16={fill} dense={dr}: {1e3 * t:.2f} ms",
                  file=sys.stderr, flush=True)
    t, load, fill, dr = min(results)
    # the width of the window loads, at the best setting
    wide = 1
    ctx.set_tuning(load, fill, dr, 0)
    time_levels(ctx, levels, limits)
    t0 = time_levels(ctx, levels, limits, repeats=2)
    if verbose:
        print(f"[tune] load16={load} fill16={fill} dense={dr} wide_loads=0: {1e3 * t0:.2f} ms",
              file=sys.stderr, flush=True)
    if t0 < t:
        t, wide = t0, 0
    ctx.set_tuning(load, fill, dr, wide)
    torch.cuda.synchronize()
    return dict(single_pass_load16=load, pass_fill16=fill, dense_ratio=dr, wide_loads=wide,
                seconds=t,
                table=[dict(single_pass_load16=l, pass_fill16=f, dense_ratio=d, seconds=s)
                       for s, l, f, d in results] +
                [dict(single_pass_load16=load, pass_fill16=fill, dense_ratio=dr, wide_loads=0,
                      seconds=t0)])
