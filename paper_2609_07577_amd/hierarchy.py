"""Whole coarsening hierarchies (Section 4.1: repeat the level until no vertex
proposes a candidate), plain or batched.

``plain_hierarchy`` drives one graph level by level through the C ABI
(hg_coarsen_level + hg_contract), reading the stop flag after every level.
``batched_hierarchies`` runs many graphs through one hg_batch, which steps
every unfinished graph one level per union step and replays the captured
level graph.  Both return, per graph, the partition of the original
vertices into final super-nodes and the number of contractions; the two
are identical by construction (the graphs of a batch share no hyperedge).
"""
from __future__ import annotations

import torch

from . import hg


def plain_hierarchy(ctx: hg.Context, L: hg.DeviceLevel, limits, max_levels: int = 100000,
                    keep_maps: bool = True):
    """Coarsen one graph to the end.  Returns (vmaps, n_levels, final level);
    ``vmaps`` are the device vertex maps of the contractions (if kept)."""
    vmaps = []
    n = 0
    while n < max_levels:
        out = ctx.coarsen_level(L, limits, want_candidates=False)
        if not int(out["any_candidate"].item()):  # one synchronisation per level
            break
        C = ctx.contract(L, out["vmap"], out["n_coarse"])
        if keep_maps:
            vmaps.append(out["vmap"])
        L = C
        n += 1
    return vmaps, n, L


def compose(vmaps, V0: int, device) -> torch.Tensor:
    """Partition of the original vertices: the composition of the level maps."""
    part = torch.arange(V0, dtype=torch.int64, device=device)
    for vm in vmaps:
        part = vm.to(torch.int64)[part]
    return part.to(torch.int32)


def batched_hierarchies(ctx: hg.Context, levels, limits, use_graph: bool = True,
                        levels_per_step: int = 4, max_steps: int = 1000000, cap=None):
    """Coarsen every level in ``levels`` to the end in one batch.  Returns a
    list of (part, n_parts, n_levels) in the order of ``levels``."""
    V = sum(L.V for L in levels)
    E = sum(L.E for L in levels)
    P = sum(L.P for L in levels)
    if cap is not None:
        V, E, P = cap
    B = hg.Batch(ctx, len(levels), V, E, P)
    pending = {B.add(L, lim): i for i, (L, lim) in enumerate(zip(levels, limits))}
    results = [None] * len(levels)
    steps = 0
    while pending and steps < max_steps:
        B.step(levels_per_step, use_graph)
        steps += 1
        done, _ = B.done()
        for s in done:
            results[pending.pop(s)] = B.result(s)
    B.close()
    if pending:
        raise RuntimeError("batched hierarchies did not finish")
    return results
