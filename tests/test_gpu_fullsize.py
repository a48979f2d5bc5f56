"""Parity at full workload sizes, through the C ABI, in the configuration the
benchmark times.

* The 2,000,000-neuron power-law level: the candidates of a seeded vertex
  sample are compared with the oracle computed one by one; the matching and
  the vertex map are compared in full with the oracle's Eq. 13 applied to the
  GPU candidates; the contraction is checked by its conservation laws and by
  Eq. 1 evaluated two ways (and by the oracle) on the fine level.
* The convolutional level (262,144 neurons, 27.9M pins): the whole level,
  every array, against the oracle; and the whole convolutional hierarchy
  (409 contractions) to the stop rule, every level against the oracle.
"""
import numpy as np
import pytest

import hgcheck
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


def _np(t):
    return t.cpu().numpy()


def test_powerlaw2M_level_sampled_and_invariants(ctx):
    g = synth.powerlaw(1, n=2_000_000, dmin=20, dmax=10_000)
    lim = synth.LIMITS["powerlaw"]
    print(f"  powerlaw2M: V={g.n_vertices} P={g.n_pins}", flush=True)
    L = ctx.upload(g)
    out = ctx.coarsen_level(L, lim)
    ctx.sync()
    cand, cscore, match, vmap = (_np(out[k]) for k in ("cand", "cscore", "match", "vmap"))
    n_coarse = int(out["n_coarse"].item())

    print("  oracle candidates of a sample", flush=True)
    OL = oracle.level0(g)
    rng = np.random.default_rng(20260)
    q = np.sort(rng.choice(g.n_vertices, 256, replace=False)).astype(np.int32)
    oc, ocs = oracle.candidates(OL, lim, query=q)
    np.testing.assert_array_equal(cand[q], oc)
    np.testing.assert_array_equal(cscore[q], ocs)

    print("  Eq. 13 and the vertex map over all vertices", flush=True)
    hgcheck.check_matching(g.n_vertices, cand, cscore, match)
    np.testing.assert_array_equal(match, oracle.match(cand, cscore))
    ovmap, onc = oracle.vmap_from_match(match)
    np.testing.assert_array_equal(vmap, ovmap)
    assert n_coarse == onc

    print("  contraction invariants and Eq. 1", flush=True)
    C = ctx.contract(L, out["vmap"], out["n_coarse"])
    ch = C.to_host()
    assert ch["V"] == n_coarse
    assert int(ch["size"].astype(np.int64).sum()) == g.n_vertices
    assert int(ch["syn"].astype(np.int64).sum()) == int(OL.syn.astype(np.int64).sum())
    assert np.all(ch["size"] <= lim.max_neurons)
    assert np.all(ch["syn"].astype(np.int64) <= lim.max_synapses)
    assert np.all(ch["ax"].astype(np.int64) <= lim.max_axons)
    lens = np.diff(ch["eoff"])
    assert np.all(lens >= 2)
    conn_fine = int(ctx.connectivity(L, out["vmap"]).item())
    conn_coarse = int((ch["w"].astype(np.int64) * (lens - 1)).sum())
    assert conn_fine == conn_coarse
    assert conn_fine == oracle.connectivity(OL.eoff, OL.pins, OL.w, vmap)


def test_conv_level0_full(ctx):
    g = synth.conv(1)
    lim = synth.LIMITS["conv"]
    print(f"  conv: V={g.n_vertices} P={g.n_pins}", flush=True)
    OL = oracle.level0(g)
    ores = oracle.coarsen_level(OL, lim)
    L = ctx.upload(g)
    out = ctx.coarsen_level(L, lim)
    ctx.sync()
    np.testing.assert_array_equal(_np(out["cand"]), ores.cand)
    np.testing.assert_array_equal(_np(out["cscore"]), ores.cscore)
    np.testing.assert_array_equal(_np(out["match"]), ores.match)
    np.testing.assert_array_equal(_np(out["vmap"]), ores.vmap)
    C = ctx.contract(L, out["vmap"], out["n_coarse"])
    ch = C.to_host()
    oc = ores.coarse
    assert ch["V"] == oc.V
    for k, ov in (("eoff", oc.eoff), ("pins", oc.pins), ("w", oc.w), ("mult", oc.mult),
                  ("size", oc.size), ("syn", oc.syn), ("ax", oc.ax)):
        np.testing.assert_array_equal(ch[k], ov, err_msg=k)
    conn = int(ctx.connectivity(L, out["vmap"]).item())
    assert conn == oracle.connectivity(OL.eoff, OL.pins, OL.w, ores.vmap)


@pytest.mark.timeout(900)
def test_conv_full_hierarchy(ctx):
    """The convolutional workload (4 layers of 64 x 64 x 16, limits
    1024 / 65536 / 4096) coarsened to the stop rule: every level's
    candidates, scores, matching, vertex map, coarse level and Eq. 1 value
    equal the oracle's, and both stop at the same level."""
    import test_gpu_parity as tp
    g = synth.conv(1)
    oh = tp.run_hierarchy_parity(ctx, g, synth.LIMITS["conv"], verbose=True)
    print(f"  conv: {oh.n_levels} contractions to the stop rule", flush=True)
