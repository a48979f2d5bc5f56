"""hg_connectivity_static (no allocation in the call) against hg_connectivity.

Both compute Eq. (1) of Section 3 with the same kernels; the first keeps its
scratch in the library's fixed device array.  Two calls in a row, the second
on a smaller level, must give exactly the values of hg_connectivity (and of
the oracle); a level above the fixed maximum is refused before any work.
"""
import numpy as np
import pytest

import oracle
from paper_2609_07577_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _partitions(rng, V):
    for k in (1, 2, 1000, max(V // 3, 1), V):
        part = rng.integers(0, k, V)
        yield k, np.searchsorted(np.unique(part), part).astype(np.int32)


def test_static_connectivity_equals_arena_version():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_07577_amd import hg
    oracle.build(force=False)
    ctx = hg.Context(0)
    rng = np.random.default_rng(2026)
    big = synth.powerlaw(1, n=2_000_000, dmin=20, dmax=10_000)  # the 2M-neuron level
    small = synth.powerlaw(2, n=50_000, dmin=8, dmax=20_000)    # hyperedges above 16384 pins
    for g in (big, small):
        print(f"  {g.name}: V={g.n_vertices} E={g.n_edges} P={g.n_pins}", flush=True)
        L = ctx.upload(g)
        for k, part in _partitions(rng, g.n_vertices):
            tp = torch.from_numpy(part).cuda()
            a = ctx.connectivity(L, tp)
            b = ctx.connectivity_static(L, tp)
            ctx.sync()
            va, vb = int(a.item()), int(b.item())
            print(f"    k={k}: {va} {vb}", flush=True)
            assert va == vb, (g.name, k)
            if g is small:
                assert vb == oracle.connectivity(g.eoff, g.pins, g.weight, part)
        del L
    # above the fixed maximum: refused on the host, nothing launched
    V = 6_000_000
    eoff = torch.zeros(1, dtype=torch.int64, device="cuda")
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    z = torch.zeros(V, dtype=torch.int32, device="cuda")
    L = hg.DeviceLevel(V, 0, 0, eoff, empty, empty, empty, z, z, z)
    with pytest.raises(hg.HgError) as ei:
        ctx.connectivity_static(L, z)
    assert ei.value.code == 3
    # and the context still works
    L = ctx.upload(small)
    part = np.zeros(small.n_vertices, np.int32)
    assert int(ctx.connectivity_static(L, torch.from_numpy(part).cuda()).item()) == 0
