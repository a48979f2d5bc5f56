"""Property checks on coarsening results (test helper).

These hold for any correct level whatever its size, so they apply to the
oracle's output and to the GPU library's output alike.  They compute nothing
of the method beyond the properties themselves.
"""
from __future__ import annotations

import json
import os

import numpy as np

from paper_2609_07577_amd import synth

MASK = np.uint32(0x7FFFFFFF)
HERE = os.path.dirname(os.path.abspath(__file__))


def load_hand_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        d = json.load(f)
    d.pop("_about")
    return d


BIG = synth.Limits(1 << 30, 1 << 30, 1 << 30)


def limits_of(spec):
    if spec == "big":
        return BIG
    return synth.Limits(*spec)


def level_from_case(case):
    return synth.from_axons(case["n"], [(a[0], a[1], a[2]) for a in case["axons"]])


def edge_lists(eoff, pins):
    """Hyperedges as lists of [vertex, flag] pairs (for comparisons)."""
    out = []
    for e in range(len(eoff) - 1):
        seg = pins[eoff[e]:eoff[e + 1]]
        out.append([[int(p & 0x7FFFFFFF), int(p >> 31)] for p in seg])
    return out


def per_edge_min_max(eoff, ids):
    """Min and max of ``ids`` over each hyperedge (empty hyperedges excluded)."""
    eoff = np.asarray(eoff)
    lens = np.diff(eoff)
    nz = lens > 0
    starts = eoff[:-1][nz]
    mn = np.full(lens.shape[0], -1, dtype=np.int64)
    mx = np.full(lens.shape[0], -1, dtype=np.int64)
    if starts.size:
        mn[nz] = np.minimum.reduceat(ids, starts)
        mx[nz] = np.maximum.reduceat(ids, starts)
    return mn, mx


def connectivity_numpy(eoff, pins, w, part):
    """Eq. (1) by sorting (block, edge) pairs: an independent implementation
    used to cross-check the oracle's and the GPU's values on big inputs."""
    eoff = np.asarray(eoff, dtype=np.int64)
    E = eoff.shape[0] - 1
    if E == 0:
        return 0
    lens = np.diff(eoff)
    edge = np.repeat(np.arange(E, dtype=np.int64), lens)
    blk = np.asarray(part, dtype=np.int64)[(np.asarray(pins) & MASK).astype(np.int64)]
    key = edge * (int(blk.max(initial=0)) + 1) + blk
    key = np.unique(key)
    e_of = key // (int(blk.max(initial=0)) + 1)
    lam = np.bincount(e_of, minlength=E)
    return int(np.sum(np.asarray(w, dtype=np.int64) * np.maximum(lam - 1, 0)))


def check_matching(V, cand, cscore, match):
    """Properties of Eq. (13): involution, pairs are candidate arcs, every
    two-cycle matched, no free vertex keeps a proposing child."""
    cand = np.asarray(cand)
    match = np.asarray(match)
    idx = np.arange(V)
    m = match >= 0
    assert np.all(match[m] != idx[m]), "self match"
    assert np.all(match[match[m]] == idx[m]), "match is not an involution"
    arcs = (cand[idx[m]] == match[m]) | (cand[match[m]] == idx[m])
    assert np.all(arcs), "matched pair is not a candidate arc"
    has = cand >= 0
    two = np.zeros(V, bool)
    two[has] = cand[cand[has]] == idx[has]
    assert np.all(match[two] == cand[two]), "two-cycle not matched"
    # an unmatched vertex has no child (otherwise it would take its best child)
    children = np.zeros(V, bool)
    children[cand[has]] = True
    assert not np.any(children & ~m), "free vertex with a proposing child"
    # a vertex without candidate has no child either (validity is symmetric)
    assert not np.any(children & ~has), "vertex with children but no candidate"
    assert np.all(np.asarray(cscore)[has] >= 1)


def check_vmap(match, vmap, n_coarse):
    match = np.asarray(match)
    V = match.shape[0]
    idx = np.arange(V)
    rep = (match < 0) | (idx < match)
    assert int(rep.sum()) == n_coarse
    assert np.array_equal(vmap[rep], np.arange(n_coarse))
    nr = ~rep
    assert np.array_equal(vmap[nr], vmap[match[nr]])


def check_contraction(fine, coarse, vmap):
    """Conservation across a contraction.  ``fine``/``coarse`` are dicts with
    eoff, pins, w, mult, size, syn, ax (numpy arrays)."""
    vmap = np.asarray(vmap, dtype=np.int64)
    assert coarse["size"].sum() == fine["size"].sum()
    assert coarse["syn"].sum() == fine["syn"].sum()
    ids = vmap[(fine["pins"] & MASK).astype(np.int64)]
    mn, mx = per_edge_min_max(fine["eoff"], ids)
    dropped = mn == mx
    w64 = fine["w"].astype(np.int64)
    assert int(coarse["w"].astype(np.int64).sum()) == int(w64[~dropped].sum())
    assert int(coarse["mult"].astype(np.int64).sum()) == int(
        fine["mult"].astype(np.int64)[~dropped].sum())
    # Eq. (1) is invariant under contraction
    c_coarse = int(np.sum(coarse["w"].astype(np.int64) * (np.diff(coarse["eoff"]) - 1)))
    c_fine = connectivity_numpy(fine["eoff"], fine["pins"], fine["w"], vmap)
    assert c_coarse == c_fine
    # canonical pins: strictly ascending ids inside every coarse hyperedge
    cid = (coarse["pins"] & MASK).astype(np.int64)
    if cid.size > 1:
        d = np.diff(cid)
        starts = np.zeros(cid.size, bool)
        starts[coarse["eoff"][1:-1]] = True
        assert np.all((d > 0) | starts[1:]), "coarse pins not strictly ascending"
    assert np.all(np.diff(coarse["eoff"]) >= 2)


def score_buckets(level, limits, load16=8, small=4096, big=16384, big_ov=8192, win_deg=768,
                  dense_ratio=8, dense_min_visits=1 << 16):
    """Work list of every vertex in the score step, by the rule the library
    applies before scoring (a host copy of that rule, used to show which
    scoring kernels an input reaches; results never depend on it).

    ``level`` is an oracle level (eoff, pins, ax, V).  Returns int array
    [V]: -1 for vertices without neighbours, else 0..7: single pass in the
    small table, single pass in the big table, windows (at most ``win_deg``
    incident hyperedges), passes over a table; +4 when the distinct-axon
    bound can bind for the vertex (its ax plus the level's largest ax above
    the limit), which makes the step also count shared inbound axons; 8 or 9
    (without or with that count) for neighbourhoods that visit at least one id
    in ``dense_ratio`` of the level (0: never) and are large (2, 3, 6, 7) or
    have an expansion of at least ``dense_min_visits``, on levels of at most
    2^21 vertices."""
    eoff = np.asarray(level.eoff, dtype=np.int64)
    lens = np.diff(eoff)
    ids = (np.asarray(level.pins) & MASK).astype(np.int64)
    V = int(level.V)
    edge_of_pin = np.repeat(np.arange(lens.shape[0]), lens)
    xn = np.bincount(ids, weights=(lens - 1)[edge_of_pin], minlength=V).astype(np.int64)
    deg = np.bincount(ids, minlength=V)
    ax = np.asarray(level.ax, dtype=np.int64)
    max_ax = int(ax.max(initial=0))
    ov = ax + max_ax > limits.max_axons
    dist = np.minimum(xn, V - 1)
    b = np.where(dist <= small * load16 // 16, 0,
                 np.where(dist <= np.where(ov, big_ov, big) * load16 // 16, 1,
                          np.where(deg <= win_deg, 2, 3)))
    b = b + 4 * ov
    # dense windows: large or often visited neighbourhoods visiting at least
    # one id in dense_ratio, on levels of at most 2^21 vertices
    if dense_ratio > 0 and 0 < V <= (1 << 21):
        big_or_hot = ((b & 3) >= 2) | (xn >= dense_min_visits)
        b = np.where(big_or_hot & (xn * dense_ratio >= V), 8 + ov, b)
    return np.where(xn > 0, b, -1)
