"""Refinement in the uncoarsening (hg_refine) against the oracle, through the
C ABI: single rounds on partitions of every level of small hierarchies (the
new partition and the counts must be the oracle's), then whole
uncoarsenings (projection and rounds down to level 0), level by level."""
import numpy as np
import pytest

import oracle
from paper_2609_07577_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_07577_amd import hg
    oracle.build(force=False)
    return hg.Context(0)


def _round(ctx, L, part, n_parts, lim):
    t = torch.from_numpy(np.ascontiguousarray(part, dtype=np.int32)).cuda()
    info = ctx.refine(L, t, n_parts, lim, max_rounds=1)
    ctx.sync()
    return t.cpu().numpy(), info


GRAPHS = [
    ("tiny", lambda s: synth.tiny_random(s, 30, max_fan=6, w_max=4), synth.Limits(5, 40, 10)),
    ("uniform", lambda s: synth.uniform(s, 800, 1, 14), synth.Limits(16, 300, 40)),
    ("layered", lambda s: synth.layered(s, width=128, fanout=12), synth.Limits(24, 600, 80)),
]


@pytest.mark.parametrize("name,make,lim", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_single_rounds(ctx, name, make, lim):
    from paper_2609_07577_amd import hierarchy
    rng = np.random.default_rng(17)
    moved = 0
    for seed in range(4):
        g = make(seed)
        oh = oracle.hierarchy(g, lim)
        levels, _ = hierarchy.hierarchy_levels(ctx, ctx.upload(g), lim)
        assert len(levels) == len(oh.levels)
        top = oh.levels[-1].level.V
        proj = np.arange(top, dtype=np.int32)
        for li in range(len(levels) - 1, -1, -1):
            OL = oh.levels[li].level
            if li < len(levels) - 1:
                proj = oracle.project(oh.levels[li].vmap, proj)
            k = int(rng.integers(1, OL.V + 1))
            for part, n_parts in ((proj, top), (rng.integers(0, k, OL.V).astype(np.int32), k)):
                exp, einfo = oracle.refine_round(OL, part, n_parts, lim)
                got, info = _round(ctx, levels[li], part, n_parts, lim)
                where = f"{name} seed {seed} level {li} parts {n_parts}"
                np.testing.assert_array_equal(got, exp, err_msg=where)
                assert info[1:3] == [int(einfo[1]), int(einfo[2])], (where, info, einfo)
                assert info[3] == int(einfo[0]), (where, info, einfo)
                moved += int(einfo[1]) > 0
    print(f"  {name}: {moved} rounds with moves", flush=True)
    assert moved > 0


@pytest.mark.parametrize("name,make,lim", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_whole_uncoarsening(ctx, name, make, lim):
    from paper_2609_07577_amd import hierarchy
    for seed in range(3):
        g = make(100 + seed)
        oh = oracle.hierarchy(g, lim)
        epart, en, etrace = oracle.uncoarsen(oh, lim)
        levels, maps = hierarchy.hierarchy_levels(ctx, ctx.upload(g), lim)
        part, n_parts, trace = hierarchy.uncoarsen(ctx, levels, maps, lim)
        ctx.sync()
        assert n_parts == en
        assert trace == [tuple(int(x) for x in t) for t in etrace], (name, seed)
        np.testing.assert_array_equal(part.cpu().numpy(), epart)
        print(f"  {name} seed {seed}: Eq. 1 {etrace[0][1]} -> {etrace[-1][2]}", flush=True)
