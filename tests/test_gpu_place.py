"""Placement (hg_place_initial, hg_place_refine, hg_place_residual) against
the oracle, through the C ABI: the Hilbert order of lattices of every shape,
initial placements (bisection, label propagation, folding) of every start,
swap refinement round by round and to the end, residual distances and the
multi-start choice; element by element."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _no_edges(n):
    return synth.Level0(n, np.zeros(1, np.int64), np.zeros(0, np.uint32),
                        np.zeros(0, np.int32), "empty")


@pytest.mark.parametrize("width,height", [(1, 1), (1, 7), (5, 1), (3, 7), (8, 8), (13, 64),
                                          (64, 64), (64, 33)])
def test_hilbert_order(ctx, width, height):
    """With no hyperedges nothing moves: node order[i] lands on the i-th
    core of the Hilbert order, which must be the oracle's."""
    C = width * height
    hc = oracle.hilbert_cores(width, height)
    assert sorted(hc.tolist()) == list(range(C))
    V = max(1, C - C // 5)
    orders = synth.start_orders(3, V, 2)
    gp = ctx.upload(_no_edges(V))
    core = ctx.place_initial(gp, width, height, _dev(orders), lp_rounds=4)
    ctx.sync()
    got = core.cpu().numpy()
    for s in range(2):
        exp = np.empty(V, np.int32)
        exp[orders[s]] = hc[:V]
        np.testing.assert_array_equal(got[s], exp, err_msg=f"start {s}")


CASES = [
    ("tiny", 12, 20, 4, 4, dict(fan_max=4)),
    ("small", 60, 150, 8, 8, {}),
    ("sparse-lattice", 50, 200, 9, 11, {}),
    ("medium", 400, 1600, 20, 20, {}),
    ("wide-edges", 300, 200, 16, 20, dict(fan_min=40, fan_max=200)),
    ("full", 1024, 4000, 32, 32, {}),
    ("max", 4096, 12000, 64, 64, {}),
]


@pytest.mark.parametrize("name,V,E,W,H,kw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("lp_rounds", [0, 1, 4])
def test_initial_placement(ctx, name, V, E, W, H, kw, lp_rounds):
    g = synth.gp_graph(5, V, E, **kw)
    L = oracle.level0(g)
    S = 3
    orders = synth.start_orders(7, V, S)
    gp = ctx.upload(g)
    core = ctx.place_initial(gp, W, H, _dev(orders), lp_rounds=lp_rounds)
    ctx.sync()
    got = core.cpu().numpy()
    for s in range(S):
        exp = oracle.initial_placement(L, W, H, orders[s], lp_rounds)
        np.testing.assert_array_equal(got[s], exp, err_msg=f"{name} start {s}")
    assert len(np.unique(got[0])) == V and got.min() >= 0 and got.max() < W * H


@pytest.mark.parametrize("name,V,E,W,H,kw", CASES, ids=[c[0] for c in CASES])
def test_residual_distance(ctx, name, V, E, W, H, kw):
    g = synth.gp_graph(9, V, E, **kw)
    L = oracle.level0(g)
    rng = np.random.default_rng(1)
    S = 4
    core = np.stack([rng.permutation(W * H)[:V] for _ in range(S)]).astype(np.int32)
    gp = ctx.upload(g)
    dist, best = ctx.place_residual(gp, W, H, _dev(core))
    ctx.sync()
    exp = [oracle.residual_distance(L, H, core[s]) for s in range(S)]
    assert dist.cpu().tolist() == exp
    assert int(best.item()) == int(np.argmin(exp))


def _refine_case(ctx, g, W, H, S, max_rounds, seed):
    L = oracle.level0(g)
    V = g.n_vertices
    orders = synth.start_orders(seed, V, S)
    gp = ctx.upload(g)
    core = ctx.place_initial(gp, W, H, _dev(orders), lp_rounds=2)
    ctx.sync()
    init = core.cpu().numpy().copy()
    info = ctx.place_refine(gp, W, H, core, max_rounds=max_rounds)
    ctx.sync()
    got, ginfo = core.cpu().numpy(), info.cpu().numpy()
    for s in range(S):
        exp, einfo = oracle.place_refine(L, W, H, init[s], max_rounds)
        np.testing.assert_array_equal(got[s], exp, err_msg=f"start {s}")
        assert ginfo[s].tolist() == einfo.tolist(), (s, ginfo[s], einfo)
    return ginfo


@pytest.mark.parametrize("name,V,E,W,H,kw", CASES[:5], ids=[c[0] for c in CASES[:5]])
def test_refine_single_rounds(ctx, name, V, E, W, H, kw):
    """One round at a time from several starts: the swaps applied (the
    prefix of recomputed tensions) must be the oracle's exactly."""
    g = synth.gp_graph(11, V, E, **kw)
    for seed in range(3):
        _refine_case(ctx, g, W, H, 4, 1, seed)


@pytest.mark.parametrize("name,V,E,W,H,kw", CASES[:5], ids=[c[0] for c in CASES[:5]])
def test_refine_to_the_end(ctx, name, V, E, W, H, kw):
    g = synth.gp_graph(13, V, E, **kw)
    info = _refine_case(ctx, g, W, H, 3, 1000, 3)
    print(f"  {name}: rounds / swaps / decrease per start {info.tolist()}", flush=True)
    assert (info[:, 1] > 0).any(), "no swap applied: the case tests nothing"


def test_refine_full_lattice_rounds(ctx):
    """1,024 nodes on 32 x 32 (no empty core) and 4,096 on 64 x 64, a few
    rounds from two starts."""
    for V, E, W, H, rounds in ((1024, 4000, 32, 32, 6), (4096, 12000, 64, 64, 2)):
        g = synth.gp_graph(17, V, E)
        _refine_case(ctx, g, W, H, 2, rounds, 5)


def test_multistart_choice(ctx):
    """Eight starts to the end; the residual distances after refinement and
    the chosen start must be the oracle's multi-start result."""
    V, E, W, H = 150, 600, 14, 12
    g = synth.gp_graph(19, V, E)
    L = oracle.level0(g)
    orders = synth.start_orders(23, V, 8)
    gp = ctx.upload(g)
    core, info, dist, best = ctx.place(gp, W, H, _dev(orders), lp_rounds=4)
    ctx.sync()
    exp_core, exp_best, exp_dist = oracle.place(L, W, H, orders, lp_rounds=4)
    assert dist.cpu().tolist() == exp_dist.tolist()
    assert int(best.item()) == exp_best
    np.testing.assert_array_equal(core.cpu().numpy()[exp_best], exp_core)


def test_degenerate_inputs(ctx):
    """One node; singleton hyperedges only; a 1 x n strip."""
    g1 = synth.from_axons(1, [(0, [], 5)])
    gp = ctx.upload(g1)
    core = ctx.place_initial(gp, 1, 1, _dev(np.zeros((2, 1))))
    info = ctx.place_refine(gp, 1, 1, core)
    dist, best = ctx.place_residual(gp, 1, 1, core)
    ctx.sync()
    assert core.cpu().tolist() == [[0], [0]] and dist.cpu().tolist() == [0, 0]
    assert info.cpu().tolist() == [[1, 0, 0], [1, 0, 0]]
    g = synth.gp_graph(29, 20, 40, fan_min=3, fan_max=8)
    L = oracle.level0(g)
    orders = synth.start_orders(31, 20, 2)
    gp = ctx.upload(g)
    core = ctx.place_initial(gp, 1, 23, _dev(orders))
    ctx.sync()
    init = core.cpu().numpy().copy()
    for s in range(2):
        np.testing.assert_array_equal(init[s], oracle.initial_placement(L, 1, 23, orders[s]))
    info = ctx.place_refine(gp, 1, 23, core)
    ctx.sync()
    for s in range(2):
        exp, einfo = oracle.place_refine(L, 1, 23, init[s])
        np.testing.assert_array_equal(core.cpu().numpy()[s], exp)
        assert info.cpu().numpy()[s].tolist() == einfo.tolist()


def test_bad_arguments_are_rejected(ctx):
    from paper_2609_07577_amd import hg
    g = synth.gp_graph(37, 10, 20)
    gp = ctx.upload(g)
    with pytest.raises(hg.HgError):
        ctx.place_initial(gp, 3, 3, _dev(synth.start_orders(1, 10, 1)))  # 10 nodes, 9 cores
    with pytest.raises(hg.HgError):
        ctx.place_initial(gp, 65, 1, _dev(synth.start_orders(1, 10, 1)))
    bad = synth.start_orders(1, 10, 1)
    bad[0, 3] = bad[0, 4]  # not a permutation
    ctx.place_initial(gp, 4, 4, _dev(bad))
    with pytest.raises(hg.HgError):
        ctx.sync()
    dup = np.array([[0, 1, 2, 3, 4, 5, 6, 7, 8, 8]], np.int32)  # two nodes on core 8
    ctx.place_refine(gp, 4, 4, _dev(dup), max_rounds=1)
    with pytest.raises(hg.HgError):
        ctx.sync()
    ctx.place_initial(gp, 4, 4, _dev(synth.start_orders(1, 10, 1)))
    ctx.sync()  # the context works after the errors
