"""Pins of the CPU oracle against the paper's definitions (no GPU).

* hand-derived cases H1-H6 (tests/golden/hand_cases.json, each citing the
  definition it follows);
* brute-force enumeration on hundreds of tiny random SNNs, including tight
  limits and many ties (tests/brute.py evaluates every constraint on the
  original neurons of each super-node);
* the paper's walk procedure, simulated sequentially, against Eq. (13);
* closed forms of Eq. (1).
"""
import numpy as np
import pytest

import brute
import hgcheck
import oracle
from paper_2609_07577_amd import synth


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


CASES = hgcheck.load_hand_cases()


def _run_level(case, lim):
    g = hgcheck.level_from_case(case)
    L = oracle.level0(g)
    return L, oracle.coarsen_level(L, lim)


@pytest.mark.parametrize("name", ["H1_path_increasing", "H2_path_ties", "H3_neuron_limit",
                                  "H4_axon_overlap"])
def test_hand_case_level0(name):
    case = CASES[name]
    lim = hgcheck.limits_of(case["limits"])
    L, r = _run_level(case, lim)
    assert r.cand.tolist() == case["cand"]
    if "cscore" in case:
        assert r.cscore.tolist() == case["cscore"]
    assert r.match.tolist() == case["match"]
    if "vmap" in case:
        assert r.vmap.tolist() == case["vmap"]
    if "coarse_edges" in case:
        c = r.coarse
        assert hgcheck.edge_lists(c.eoff, c.pins) == case["coarse_edges"]
        assert c.w.tolist() == case["coarse_w"]
    if "coarse_mult" in case:
        assert r.coarse.mult.tolist() == case["coarse_mult"]
    if "coarse_size" in case:
        assert r.coarse.size.tolist() == case["coarse_size"]
        assert r.coarse.syn.tolist() == case["coarse_syn"]
        assert r.coarse.ax.tolist() == case["coarse_ax"]
    if "conn_vmap" in case:
        assert oracle.connectivity(L.eoff, L.pins, L.w, r.vmap) == case["conn_vmap"]


@pytest.mark.parametrize("name", ["H1_path_increasing", "H3_neuron_limit"])
def test_hand_case_hierarchy(name):
    case = CASES[name]
    lim = hgcheck.limits_of(case["limits"])
    g = hgcheck.level_from_case(case)
    h = oracle.hierarchy(g, lim)
    assert h.n_levels == case["levels_until_stop"]
    if "level1_cand" in case:
        assert h.levels[1].cand.tolist() == case["level1_cand"]
    if "final_conn" in case:
        L0 = h.levels[0].level
        assert oracle.connectivity(L0.eoff, L0.pins, L0.w, h.final_partition()) == case["final_conn"]


def test_hand_case_destination_flags():
    case = CASES["H5_destination_flags"]
    g = hgcheck.level_from_case(case)
    L = oracle.level0(g)
    c = oracle.contract(L, np.array(case["vmap"], np.int32), case["n_coarse"])
    assert hgcheck.edge_lists(c.eoff, c.pins) == case["coarse_edges"]
    assert c.w.tolist() == case["coarse_w"]
    assert c.mult.tolist() == case["coarse_mult"]
    assert c.ax.tolist() == case["coarse_ax"]
    c2 = oracle.contract(c, np.array([0, 0], np.int32), 1)
    assert c2.ax.tolist() == [case["merged_ax_after_second_contraction"]]
    assert c2.E == 0


def test_hand_case_connectivity():
    case = CASES["H6_connectivity"]
    g = hgcheck.level_from_case(case)
    n = case["n"]
    assert oracle.connectivity(g.eoff, g.pins, g.weight, np.array(case["part"], np.int32)) == case["conn"]
    assert oracle.connectivity(g.eoff, g.pins, g.weight, np.arange(n, dtype=np.int32)) == case["conn_singletons"]
    assert oracle.connectivity(g.eoff, g.pins, g.weight, np.zeros(n, np.int32)) == case["conn_one_block"]


def _tiny_limits(rng):
    kind = rng.integers(0, 4)
    if kind == 0:
        return hgcheck.BIG
    return synth.Limits(int(rng.integers(2, 6)), int(rng.integers(1, 10)), int(rng.integers(1, 8)))


def _compare_with_brute(g, lim):
    bl, orig = brute.hierarchy(g.n_vertices, g.eoff, g.pins, g.weight, lim)
    h = oracle.hierarchy(g, lim)
    assert len(h.levels) == len(bl)
    for r, b in zip(h.levels, bl):
        L = r.level
        assert L.V == b["V"]
        assert hgcheck.edge_lists(L.eoff, L.pins) == [[[v, int(d)] for v, d in pl] for pl in b["edges"]]
        assert L.w.tolist() == b["w"]
        assert L.mult.tolist() == b["mult"]
        mem = b["members"]
        assert L.size.tolist() == [orig.size(s) for s in mem]
        assert L.syn.tolist() == [orig.synapses(s) for s in mem]
        assert L.ax.tolist() == [orig.axons(s) for s in mem]
        assert r.cand.tolist() == b["cand"]
        assert r.cscore.tolist() == b["cscore"]
        assert r.match.tolist() == b["match"]
        assert b["match_walk"] == b["match"]
        if "vmap" in b:
            assert r.vmap.tolist() == b["vmap"]
            assert r.n_coarse == b["n_coarse"]
        # every super-node is within limits at every level
        for s in mem:
            if len(s) > 1:
                assert orig.feasible(s, lim)


@pytest.mark.parametrize("block", range(6))
def test_oracle_matches_brute_force_tiny(block):
    rng = np.random.default_rng(1000 + block)
    for i in range(60):
        seed = int(rng.integers(0, 1 << 30))
        n = int(rng.integers(1, 13))
        g = synth.tiny_random(seed, n, p_axon=float(rng.uniform(0.3, 1.0)),
                              max_fan=int(rng.integers(1, 6)), w_max=int(rng.integers(1, 4)))
        _compare_with_brute(g, _tiny_limits(rng))


def test_oracle_matches_brute_force_dense_ties():
    # every weight 1 and full fan-out: ties decide every candidate
    for seed in range(20):
        g = synth.tiny_random(seed, 9, p_axon=1.0, max_fan=8, w_max=1)
        _compare_with_brute(g, hgcheck.BIG)
        _compare_with_brute(g, synth.Limits(3, 100, 100))


def test_score_symmetry_and_candidates_subset():
    g = synth.uniform(7, 300, 3, 12)
    L = oracle.level0(g)
    lim = synth.LIMITS["layered"]
    cand, cscore = oracle.candidates(L, lim)
    q = np.array([5, 17, 299, 0, 123], np.int32)
    c2, s2 = oracle.candidates(L, lim, query=q)
    assert np.array_equal(c2, cand[q]) and np.array_equal(s2, cscore[q])
    edges = brute.edges_of(L.eoff, L.pins)
    for n in q.tolist():
        m = int(cand[n])
        if m >= 0:
            assert brute.score(edges, L.w, n, m) == brute.score(edges, L.w, m, n) == cscore[n]


def test_connectivity_closed_forms():
    g = synth.uniform(3, 500, 2, 20)
    L = oracle.level0(g)
    lens = np.diff(L.eoff)
    singletons = int(np.sum(L.w.astype(np.int64) * (lens - 1)))
    assert oracle.connectivity(L.eoff, L.pins, L.w, np.arange(g.n_vertices, dtype=np.int32)) == singletons
    assert oracle.connectivity(L.eoff, L.pins, L.w, np.zeros(g.n_vertices, np.int32)) == 0
    rng = np.random.default_rng(0)
    part = rng.integers(0, 37, g.n_vertices).astype(np.int32)
    assert oracle.connectivity(L.eoff, L.pins, L.w, part) == hgcheck.connectivity_numpy(
        L.eoff, L.pins, L.w, part)
    edges = brute.edges_of(L.eoff, L.pins)
    assert oracle.connectivity(L.eoff, L.pins, L.w, part) == brute.connectivity(edges, L.w, part)


def test_contract_general_partition_vs_brute():
    rng = np.random.default_rng(5)
    for seed in range(40):
        g = synth.tiny_random(seed, int(rng.integers(2, 14)), max_fan=5, w_max=9)
        L = oracle.level0(g)
        k = int(rng.integers(1, g.n_vertices + 1))
        part = rng.integers(0, k, g.n_vertices)
        # compact to [0, nc)
        uniq = np.unique(part)
        vmap = np.searchsorted(uniq, part).astype(np.int32)
        c = oracle.contract(L, vmap, len(uniq))
        be, bw, bm = brute.contract(brute.edges_of(L.eoff, L.pins), L.w, L.mult, vmap.tolist())
        assert hgcheck.edge_lists(c.eoff, c.pins) == [[[v, int(d)] for v, d in pl] for pl in be]
        assert c.w.tolist() == bw and c.mult.tolist() == bm
        orig = brute.Orig(g.n_vertices, g.eoff, g.pins)
        for b in range(len(uniq)):
            mem = set(np.nonzero(vmap == b)[0].tolist())
            assert c.size[b] == orig.size(mem)
            assert c.syn[b] == orig.synapses(mem)
            assert c.ax[b] == orig.axons(mem)


def _union(graphs):
    """Graphs side by side: vertex ids and pin offsets shifted, flags kept."""
    eoff, pins, w = [np.zeros(1, np.int64)], [], []
    V = P = 0
    for g in graphs:
        eoff.append(np.asarray(g.eoff[1:], np.int64) + P)
        p = np.asarray(g.pins, np.uint32)
        pins.append(((p & 0x7FFFFFFF) + V) | (p & 0x80000000))
        w.append(np.asarray(g.weight, np.int32))
        V += g.n_vertices
        P += g.n_pins
    return synth.Level0(V, np.concatenate(eoff), np.concatenate(pins).astype(np.uint32),
                        np.concatenate(w), "union")


def test_union_of_disjoint_graphs_is_separate_runs():
    """Graphs that share no hyperedge never interact (Eq. 12 scores only
    pairs inside a hyperedge; Eq. 13 only follows candidate arcs; G_P keeps
    vertex and hyperedge order), so coarsening their union gives every graph
    the partition of its own hierarchy, and the union needs as many levels
    as its deepest graph.  This is what a batch of graphs relies on."""
    lim = synth.Limits(24, 400, 60)
    graphs = [synth.uniform(s, n, 1, 9) for s, n in ((1, 150), (2, 90), (3, 200))]
    graphs.append(synth.tiny_random(4, 30))
    alone = [oracle.hierarchy(g, lim) for g in graphs]
    u = oracle.hierarchy(_union(graphs), lim)
    assert u.n_levels == max(h.n_levels for h in alone)
    part = u.final_partition()
    base = 0
    for g, h in zip(graphs, alone):
        mine = part[base:base + g.n_vertices]
        # the union numbers the graph's super-nodes after those of earlier graphs
        np.testing.assert_array_equal(mine - mine.min(), h.final_partition())
        base += g.n_vertices


def _original_members(h, li, n_parts, part):
    """Original neurons of every part of a partition of level ``li``."""
    up = np.arange(h.levels[0].level.V)
    for r in h.levels[:li]:
        up = r.vmap[up]
    members = [set() for _ in range(n_parts)]
    for v0, v in enumerate(up.tolist()):
        members[int(part[v])].add(v0)
    return members


def test_partition_report_vs_brute_force():
    """The oracle's partition report (Section 3) against first principles:
    every part's size, inbound synapses and distinct inbound axons counted
    on the ORIGINAL neurons it holds, and Eq. (1) by enumeration, for random
    partitions of every level of tiny hierarchies."""
    rng = np.random.default_rng(31)
    for seed in range(40):
        g = synth.tiny_random(seed, int(rng.integers(2, 14)), max_fan=5, w_max=7)
        lim = synth.Limits(int(rng.integers(2, 6)), 30, int(rng.integers(2, 8)))
        h = oracle.hierarchy(g, lim)
        orig = brute.Orig(g.n_vertices, g.eoff, g.pins)
        for li, r in enumerate(h.levels):
            L = r.level
            k = int(rng.integers(1, L.V + 1))
            part = rng.integers(0, k, L.V).astype(np.int32)
            rep = oracle.partition_report(L, part, k, lim)
            mem = _original_members(h, li, k, part)
            assert rep.size.tolist() == [orig.size(m) for m in mem]
            assert rep.syn.tolist() == [orig.synapses(m) for m in mem]
            assert rep.ax.tolist() == [orig.axons(m) for m in mem]
            assert rep.conn == brute.connectivity(brute.edges_of(L.eoff, L.pins), L.w, part)
            assert rep.summary[4] == sum(orig.size(m) > lim.max_neurons for m in mem)
            assert rep.summary[6] == sum(orig.axons(m) > lim.max_axons for m in mem)


def test_projection_down_the_hierarchy():
    """The final super-nodes as parts (Section 4.1), projected level by level
    down to level 0, give every original neuron its final super-node (the
    composition of the level maps, taken upwards); Eq. (1) of each level
    under its projected partition is the same number; every part is within
    the limits, except a single neuron that already breaks one."""
    for seed in range(12):
        g = synth.uniform(seed, 300, 1, 10)
        lim = synth.Limits(12, 200, 30)
        h = oracle.hierarchy(g, lim)
        top = h.levels[-1].level
        part = np.arange(top.V, dtype=np.int32)
        conns = []
        for li in range(len(h.levels) - 1, -1, -1):
            L = h.levels[li].level
            rep = oracle.partition_report(L, part, top.V, lim)
            conns.append(rep.conn)
            bad = (rep.size > lim.max_neurons) | (rep.syn > lim.max_synapses) | \
                  (rep.ax > lim.max_axons)
            assert np.all(rep.size[bad] == 1)
            if li > 0:
                part = oracle.project(h.levels[li - 1].vmap, part)
        assert len(set(conns)) == 1
        np.testing.assert_array_equal(part, h.final_partition())


def _level_members(h, li):
    """Original neurons of every vertex of level ``li``."""
    up = np.arange(h.levels[0].level.V)
    for r in h.levels[:li]:
        up = r.vmap[up]
    mem = [set() for _ in range(h.levels[li].level.V)]
    for v0, v in enumerate(up.tolist()):
        mem[int(v)].add(v0)
    return mem


@pytest.mark.parametrize("block", range(4))
def test_refine_round_vs_brute_force(block):
    """The oracle's refinement round against enumeration: every proposal's
    gain is the drop of Eq. (1) recomputed from scratch, every limit is
    checked on the original neurons of a part, every prefix is applied and
    evaluated from scratch; the chosen prefix and the new partition must be
    the same.  Tiny hierarchies at every level, with the projected partition
    of the final super-nodes and with random partitions."""
    rng = np.random.default_rng(400 + block)
    for it in range(40):
        g = synth.tiny_random(int(rng.integers(0, 1 << 30)), int(rng.integers(2, 13)),
                              p_axon=float(rng.uniform(0.4, 1.0)), max_fan=5,
                              w_max=int(rng.integers(1, 6)))
        lim = synth.Limits(int(rng.integers(2, 6)), int(rng.integers(2, 25)),
                           int(rng.integers(1, 8)))
        h = oracle.hierarchy(g, lim)
        orig = brute.Orig(g.n_vertices, g.eoff, g.pins)
        top = h.levels[-1].level.V
        proj = np.arange(top, dtype=np.int32)
        for li in range(len(h.levels) - 1, -1, -1):
            L = h.levels[li].level
            if li < len(h.levels) - 1:
                proj = oracle.project(h.levels[li].vmap, proj)
            mem = _level_members(h, li)
            edges = brute.edges_of(L.eoff, L.pins)
            k = int(rng.integers(1, L.V + 1))
            for part, n_parts in ((proj, top), (rng.integers(0, k, L.V).astype(np.int32), k)):
                got, info = oracle.refine_round(L, part, n_parts, lim)
                exp, einfo = brute.refine_round(edges, L.w, part, n_parts, mem, orig, lim)
                assert got.tolist() == exp, (it, li)
                assert info.tolist() == einfo, (it, li)


def test_refinement_never_worsens_and_keeps_limits():
    """Whole uncoarsening (projection and refinement rounds down to level 0):
    Eq. (1) never rises, the level-0 result is at most that of the final
    super-nodes, and every part that was within the limits stays so."""
    for seed in range(6):
        g = synth.uniform(seed, 400, 1, 12)
        lim = synth.Limits(16, 300, 40)
        h = oracle.hierarchy(g, lim)
        part, n_parts, trace = oracle.uncoarsen(h, lim)
        for li, before, after, rounds in trace:
            assert after <= before
        L0 = h.levels[0].level
        assert trace[-1][2] == oracle.connectivity(L0.eoff, L0.pins, L0.w, part)
        assert trace[-1][2] <= trace[0][1]
        rep = oracle.partition_report(L0, part, n_parts, lim)
        bad = (rep.size > lim.max_neurons) | (rep.syn > lim.max_synapses) | \
              (rep.ax > lim.max_axons)
        assert np.all(rep.size[bad] <= 1)


def test_hilbert_order():
    """Every core once; on a power-of-two square consecutive cores are
    neighbours (the curve's locality)."""
    for w, h in ((1, 1), (2, 2), (8, 8), (64, 64), (5, 3), (6, 11)):
        hc = oracle.hilbert_cores(w, h)
        assert sorted(hc.tolist()) == list(range(w * h))
    hc = oracle.hilbert_cores(16, 16)
    steps = [brute.manhattan(int(a), int(b), 16) for a, b in zip(hc[:-1], hc[1:])]
    assert set(steps) == {1}
    assert oracle.hilbert_cores(2, 2).tolist() == [0, 1, 3, 2]  # (0,0) (0,1) (1,1) (1,0)


def _gp(seed, n, lim):
    """A small partitioned hypergraph G_P (final super-nodes as nodes)."""
    g = synth.uniform(seed, n, 1, 8)
    h = oracle.hierarchy(g, lim)
    return h.levels[-1].level


@pytest.mark.parametrize("block", range(3))
def test_swap_round_vs_brute_force(block):
    """A swap-refinement round (Eq. 14, 15 and the matching and prefix of
    Section 4.2) against enumeration, where every tension and every prefix
    is the decrease of the residual distance recomputed from scratch."""
    rng = np.random.default_rng(900 + block)
    applied = 0
    for it in range(8):
        L = _gp(int(rng.integers(0, 1 << 20)), int(rng.integers(30, 90)), synth.Limits(6, 60, 20))
        w, h = (int(x) for x in rng.integers(2, 7, 2))
        if L.V > w * h:
            w = h = int(np.ceil(np.sqrt(L.V))) + 1
        core = rng.permutation(w * h)[:L.V].astype(np.int32)
        got, info = oracle.place_refine(L, w, h, core, max_rounds=1)
        exp, n_app, dec = brute.place_refine_round(brute.edges_of(L.eoff, L.pins), L.w,
                                                   core.tolist(), w, h)
        assert got.tolist() == exp, it
        assert (int(info[1]), int(info[2])) == (n_app, dec), it
        applied += n_app > 0
    assert applied > 0


@pytest.mark.parametrize("block", range(3))
def test_initial_placement_vs_brute_force(block):
    """Initial placement (Hilbert order, recursive bisection with label
    propagation, folding) against enumeration, where every gain is the drop
    of a section's cut recomputed from scratch and every folding decision
    compares connection weights counted from scratch."""
    rng = np.random.default_rng(700 + block)
    for it in range(6):
        L = _gp(int(rng.integers(0, 1 << 20)), int(rng.integers(40, 120)), synth.Limits(5, 60, 20))
        w = h = int(np.ceil(np.sqrt(L.V))) + int(rng.integers(0, 3))
        order0 = rng.permutation(L.V).astype(np.int32)
        got = oracle.initial_placement(L, w, h, order0, lp_rounds=3)
        exp = brute.initial_placement(brute.edges_of(L.eoff, L.pins), L.w, L.V,
                                      oracle.hilbert_cores(w, h), order0, 3)
        assert got.tolist() == exp, it
        assert len(set(got.tolist())) == L.V


def test_placement_improves_residual_distance():
    """Multi-start placement: refinement never raises a start's residual
    distance, and the chosen start has the least."""
    L = _gp(3, 400, synth.Limits(8, 100, 30))
    orders = synth.start_orders(5, L.V, 4)
    core, best, dists = oracle.place(L, 16, 16, orders)
    for k, o in enumerate(orders):
        c0 = oracle.initial_placement(L, 16, 16, o)
        assert dists[k] <= oracle.residual_distance(L, 16, c0)
    assert dists[best] == dists.min() and best == int(np.argmin(dists))
    assert oracle.residual_distance(L, 16, core) == dists[best]
