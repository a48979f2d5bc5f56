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


def uncoarsen(ctx: hg.Context, levels, maps, limits, max_rounds: int = 16):
    """The uncoarsening (Section 4.1): the final super-nodes of a hierarchy
    as initial parts, then level by level down to level 0, the partition
    projected through the level's vertex map (hg_project) and refined
    (hg_refine).  ``levels``: the device levels of the hierarchy, level 0
    first; ``maps``: their (vmap, n_coarse) pairs, one fewer.  Returns the
    level-0 partition (device int32), the number of parts and a per-level
    list of (level, Eq. 1 after projection, Eq. 1 after refinement, rounds)."""
    top = levels[-1]
    n_parts = top.V
    part = torch.arange(n_parts, dtype=torch.int32, device=ctx.device)
    trace = []
    for li in range(len(levels) - 1, -1, -1):
        L = levels[li]
        if li < len(levels) - 1:
            vmap, nc = maps[li]
            part = ctx.project(vmap, nc, part)
        before = int(ctx.connectivity(L, part).item())
        info = ctx.refine(L, part, n_parts, limits, max_rounds)
        trace.append((li, before, before - info[2], info[0]))
    return part, n_parts, trace


def hierarchy_levels(ctx: hg.Context, L: hg.DeviceLevel, limits, max_levels: int = 100000):
    """The plain hierarchy with every level kept on the device: (levels,
    maps) as uncoarsen() takes them."""
    levels, maps = [L], []
    while len(maps) < max_levels:
        out = ctx.coarsen_level(L, limits, want_candidates=False)
        if not int(out["any_candidate"].item()):
            break
        maps.append((out["vmap"], out["n_coarse"]))
        L = ctx.contract(L, out["vmap"], out["n_coarse"])
        levels.append(L)
    return levels, maps
