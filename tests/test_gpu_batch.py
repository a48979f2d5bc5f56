"""Batched and continuously batched coarsening (hg_batch_*) vs the CPU oracle.

Every graph of a batch must end with exactly the partition and the number of
contractions of its own oracle hierarchy, whatever else shares the batch,
whenever it was added, and whether the level steps run eagerly or as
replays of a captured HIP graph (with host work and synchronisation between
the replays).
"""
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


def mixed_graphs():
    """Uneven graphs with different limits (feed-forward and recurrent)."""
    gs = []
    for k in range(6):
        gs.append((synth.batch_graph(7, k, n_min=500, n_max=4000, fan_min=4, fan_max=24),
                   synth.LIMITS["batch"]))
    gs.append((synth.uniform(3, 3000, 1, 30), synth.Limits(64, 4096, 128)))
    gs.append((synth.tiny_random(5, 40), synth.Limits(4, 100, 8)))
    gs.append((synth.layered(2, width=256, fanout=16), synth.Limits(32, 2048, 128)))
    gs.append((synth.uniform(4, 2000, 2, 12), synth.Limits(16, 200, 40)))
    return gs


_expected = {}


def expected(i, g, lim):
    if i not in _expected:
        h = oracle.hierarchy(g, lim)
        _expected[i] = (h.final_partition(), h.n_levels)
    return _expected[i]


def caps(graphs):
    V = sum(g.n_vertices for g, _ in graphs)
    E = sum(g.n_edges for g, _ in graphs)
    P = sum(g.n_pins for g, _ in graphs)
    return V, E, P


def check_result(i, g, lim, res):
    part, n_parts, n_levels = res
    exp_part, exp_levels = expected(i, g, lim)
    got = part.cpu().numpy()
    np.testing.assert_array_equal(got, exp_part, err_msg=f"partition of graph {i} ({g.name})")
    assert n_parts == int(exp_part.max()) + 1 if exp_part.size else n_parts == 0, g.name
    assert n_levels == exp_levels, (g.name, n_levels, exp_levels)


def drain(B, pending, results, use_graph, levels_per_step=2, max_steps=400):
    for _ in range(max_steps):
        if not pending:
            return
        B.step(levels_per_step, use_graph)
        done, _live = B.done()
        for s in done:
            results[pending.pop(s)] = B.result(s)
    raise AssertionError("batch did not finish")


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_all_at_once(ctx, use_graph):
    from paper_2609_07577_amd import hg
    graphs = mixed_graphs()
    V, E, P = caps(graphs)
    B = hg.Batch(ctx, len(graphs), V, E, P)
    pending, results = {}, {}
    for i, (g, lim) in enumerate(graphs):
        print(f"  add {i}: {g.name} V={g.n_vertices} P={g.n_pins}", flush=True)
        pending[B.add(ctx.upload(g), lim)] = i
    drain(B, pending, results, use_graph)
    ctx.sync()
    for i, (g, lim) in enumerate(graphs):
        check_result(i, g, lim, results[i])
    B.close()


def test_batch_continuous_admission(ctx):
    """Graphs arrive while others are half-way through their hierarchy; slots
    and memory are reused after release and compaction."""
    from paper_2609_07577_amd import hg
    graphs = mixed_graphs()
    # room for about half of the graphs at once
    V, E, P = caps(graphs)
    B = hg.Batch(ctx, 5, V // 2 + 4000, E // 2 + 4000, P // 2 + 200000)
    queue = list(range(len(graphs)))
    pending, results = {}, {}
    uploaded = {}
    steps = 0
    while queue or pending:
        # admit what fits (the library reports a full batch as HG_ERR_CAPACITY)
        while queue:
            i = queue[0]
            g, lim = graphs[i]
            if i not in uploaded:
                uploaded[i] = ctx.upload(g)
            try:
                slot = B.add(uploaded[i], lim)
            except hg.HgError as e:
                assert e.code == 3, e
                break
            pending[slot] = i
            queue.pop(0)
            print(f"  step {steps}: admitted {i} into slot {slot}", flush=True)
        B.step(1, use_graph=True)
        steps += 1
        done, _ = B.done()
        for s in done:
            results[pending.pop(s)] = B.result(s)
        if done:
            B.compact()
        assert steps < 2000
    ctx.sync()
    for i, (g, lim) in enumerate(graphs):
        check_result(i, g, lim, results[i])
    B.close()


def test_batch_same_graph_alone_and_mixed(ctx):
    """One graph run alone and inside a mix gives the identical result."""
    from paper_2609_07577_amd import hg
    graphs = mixed_graphs()
    g, lim = graphs[2]
    alone = hg.Batch(ctx, 1, g.n_vertices, g.n_edges, g.n_pins)
    s = alone.add(ctx.upload(g), lim)
    res_alone = {}
    drain(alone, {s: 0}, res_alone, use_graph=True)
    V, E, P = caps(graphs)
    mixed = hg.Batch(ctx, len(graphs), V, E, P)
    pending = {}
    for i, (gg, ll) in enumerate(graphs):
        pending[mixed.add(ctx.upload(gg), ll)] = i
    res_mixed = {}
    drain(mixed, pending, res_mixed, use_graph=True)
    ctx.sync()
    pa, na, la = res_alone[0]
    pm, nm, lm = res_mixed[2]
    np.testing.assert_array_equal(pa.cpu().numpy(), pm.cpu().numpy())
    assert (na, la) == (nm, lm)
    check_result(2, g, lim, res_mixed[2])


def test_server_admits_compacts_and_matches_oracle(ctx):
    """The request loop of the served mode: a capacity for only a few graphs
    at a time forces refused admissions and compactions; every request's
    result must still be its own oracle hierarchy."""
    import time
    from paper_2609_07577_amd import serve
    graphs = mixed_graphs()
    biggest = max(g.n_pins for g, _ in graphs)
    srv = serve.Server(ctx, max_graphs=4, cap_vertices=9000, cap_edges=9000,
                       cap_pins=2 * biggest + 1000, levels_per_step=3, use_graph=True,
                       compact_every=2)
    levels = [ctx.upload(g) for g, _ in graphs]
    for i, (g, lim) in enumerate(graphs):
        srv.submit(i, levels[i], lim, time.perf_counter())
    results = {}
    steps = 0
    while not srv.idle():
        for rid, arr, fin, part, n_parts, n_levels, pins in srv.step():
            results[rid] = (part, n_parts, n_levels)
        steps += 1
        assert steps < 5000
    ctx.sync()
    srv.close()
    assert sorted(results) == list(range(len(graphs)))
    for i, (g, lim) in enumerate(graphs):
        check_result(i, g, lim, results[i])
