"""The boundary's checks and switches, through the C ABI.

* hg_validate_level on malformed levels (HG_ERR_INVALID_LEVEL) and on levels
  whose weights sum to 2^31 or more (HG_ERR_OVERFLOW);
* the device-side weight check of hg_coarsen_level (weights >= 1, sum below
  2^31, needed because scores are exact int32 sums packed next to ids),
  reported by hg_sync, after which the context works normally;
* HG_VALIDATE=1 (every input level checked first), HG_SCRATCH_CAP (a call
  needing a larger arena fails with HG_ERR_NO_MEMORY) and HG_TEST_FP_BITS
  (fingerprints cut to a few bits, so that the exact grouping of unequal
  coarse hyperedges that share a fingerprint decides every contraction; the
  results must still be the oracle's).
"""
import contextlib
import os

import numpy as np
import pytest

import hgcheck
import oracle
from paper_2609_07577_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

INVALID_ARG, OVERFLOW, NO_MEMORY, INVALID_LEVEL = 1, 2, 4, 7


@pytest.fixture(scope="module")
def hg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_07577_amd import hg as _hg
    oracle.build(force=False)
    return _hg


@contextlib.contextmanager
def env(**kw):
    old = {k: os.environ.get(k) for k in kw}
    os.environ.update({k: str(v) for k, v in kw.items()})
    try:
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _host(g):
    """Level-0 arrays with state (oracle level 0) as a dict for level_from_host."""
    L = oracle.level0(g)
    return dict(V=L.V, eoff=L.eoff.copy(), pins=L.pins.copy(), w=L.w.copy(), mult=L.mult.copy(),
                size=L.size.copy(), syn=L.syn.copy(), ax=L.ax.copy())


def _check_level(ctx, g, lim):
    """One level of ``g`` on the GPU equals the oracle's (the context works)."""
    L = ctx.upload(g)
    out = ctx.coarsen_level(L, lim)
    ctx.sync()
    r = oracle.coarsen_level(oracle.level0(g), lim)
    np.testing.assert_array_equal(out["cand"].cpu().numpy(), r.cand)
    np.testing.assert_array_equal(out["match"].cpu().numpy(), r.match)


def test_validate_level(hg):
    ctx = hg.Context(0)
    g = synth.uniform(3, 400, 2, 20)
    good = _host(g)
    ctx.validate(ctx.level_from_host(good))
    cases = []
    d = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in good.items()}
    s, t = int(d["eoff"][5]), int(d["eoff"][6])
    d["pins"][s:t] = d["pins"][s:t][::-1].copy()  # ids descending inside a hyperedge
    cases.append(("unsorted pins", d, INVALID_LEVEL))
    d = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in good.items()}
    d["pins"][int(d["eoff"][7])] = np.uint32(400)  # id == V
    cases.append(("pin id out of range", d, INVALID_LEVEL))
    d = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in good.items()}
    d["w"][11] = 0
    cases.append(("zero weight", d, INVALID_LEVEL))
    d = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in good.items()}
    d["mult"][2] = 0
    cases.append(("zero multiplicity", d, INVALID_LEVEL))
    d = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in good.items()}
    d["w"][:] = (1 << 31) // len(d["w"]) + 1
    cases.append(("weights summing to 2^31", d, OVERFLOW))
    for what, dd, code in cases:
        print(f"  validate: {what}", flush=True)
        with pytest.raises(hg.HgError) as ei:
            ctx.validate(ctx.level_from_host(dd))
        assert ei.value.code == code, (what, ei.value)
    ctx.validate(ctx.level_from_host(good))


def test_coarsen_checks_weights_on_device(hg):
    """A zero weight would let the score step pick a neighbour of score 0
    (the oracle never does), and weights summing to 2^31 would wrap the
    packed scores: both are caught on the device before the scores and
    reported by hg_sync; the next level is computed normally."""
    ctx = hg.Context(0)
    lim = synth.Limits(64, 4096, 256)
    g = synth.uniform(4, 600, 2, 16)
    good = _host(g)
    zero = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in good.items()}
    zero["w"][[3, 50]] = 0
    heavy = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in good.items()}
    heavy["w"][:] = (1 << 31) // len(heavy["w"]) + 1
    for what, d, code in (("zero weight", zero, INVALID_LEVEL), ("sum >= 2^31", heavy, OVERFLOW)):
        print(f"  coarsen: {what}", flush=True)
        L = ctx.level_from_host(d)
        out = ctx.coarsen_level(L, lim)
        with pytest.raises(hg.HgError) as ei:
            ctx.sync()
        assert ei.value.code == code, (what, ei.value)
        # hg_contract runs the same check
        ctx.contract(L, out["vmap"], out["n_coarse"], trim=False)
        with pytest.raises(hg.HgError) as ei:
            ctx.sync()
        assert ei.value.code == code, (what, ei.value)
        _check_level(ctx, g, lim)


def test_validate_switch(hg):
    """HG_VALIDATE=1: a malformed level is refused by the call itself."""
    g = synth.uniform(5, 300, 2, 12)
    bad = _host(g)
    s, t = int(bad["eoff"][1]), int(bad["eoff"][2])
    bad["pins"][s:t] = bad["pins"][s:t][::-1].copy()
    lim = synth.Limits(64, 4096, 256)
    with env(HG_VALIDATE=1):
        ctx = hg.Context(0)
    L = ctx.level_from_host(bad)
    with pytest.raises(hg.HgError) as ei:
        ctx.coarsen_level(L, lim)
    assert ei.value.code == INVALID_LEVEL
    with pytest.raises(hg.HgError) as ei:
        ctx.connectivity(L, torch.zeros(300, dtype=torch.int32, device="cuda"))
    assert ei.value.code == INVALID_LEVEL
    _check_level(ctx, g, lim)


def test_scratch_cap(hg):
    """HG_SCRATCH_CAP: a level whose scratch exceeds the cap fails with
    HG_ERR_NO_MEMORY and leaves the context usable for smaller levels."""
    lim = synth.Limits(64, 4096, 256)
    with env(HG_SCRATCH_CAP=4 << 20):
        ctx = hg.Context(0)
    big = synth.uniform(6, 20000, 20, 40)
    L = ctx.upload(big)
    with pytest.raises(hg.HgError) as ei:
        ctx.coarsen_level(L, lim)
    assert ei.value.code == NO_MEMORY
    _check_level(ctx, synth.uniform(7, 500, 2, 10), lim)
    assert ctx.scratch_bytes() <= 4 << 20


@pytest.mark.parametrize("bits", [3, 6])
def test_fingerprint_collisions(hg, bits):
    """With the fingerprints of coarse hyperedges cut to a few bits almost
    every hyperedge shares its fingerprint with unequal ones, so grouping
    rests on the exact comparison of colliding lists; contractions under
    general partitions and three coarsening levels must equal the oracle."""
    with env(HG_TEST_FP_BITS=bits):
        ctx = hg.Context(0)
    rng = np.random.default_rng(bits)
    g = synth.uniform(8, 1200, 1, 12)
    OL = oracle.level0(g)
    L = ctx.upload(g)
    for k in (3, 40, 600):
        part = rng.integers(0, k, g.n_vertices)
        uniq = np.unique(part)
        vmap = np.searchsorted(uniq, part).astype(np.int32)
        C = ctx.contract(L, torch.from_numpy(vmap).cuda(),
                         torch.tensor([len(uniq)], dtype=torch.int32, device="cuda"))
        exp = oracle.contract(OL, vmap, len(uniq))
        h = C.to_host()
        for key, ov in (("eoff", exp.eoff), ("pins", exp.pins), ("w", exp.w), ("mult", exp.mult),
                        ("size", exp.size), ("syn", exp.syn), ("ax", exp.ax)):
            np.testing.assert_array_equal(h[key], ov, err_msg=f"{key} k={k} bits={bits}")
    oh = oracle.hierarchy(g, synth.Limits(16, 400, 40), max_levels=3)
    for r in oh.levels:
        out = ctx.coarsen_level(L, synth.Limits(16, 400, 40))
        np.testing.assert_array_equal(out["vmap"].cpu().numpy(), r.vmap)
        if not r.any_candidate:
            break
        L = ctx.contract(L, out["vmap"], out["n_coarse"])
        h = L.to_host()
        np.testing.assert_array_equal(h["pins"], r.coarse.pins)
        np.testing.assert_array_equal(h["w"], r.coarse.w)
        np.testing.assert_array_equal(h["mult"], r.coarse.mult)
    ctx.sync()
