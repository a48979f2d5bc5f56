"""CPU oracle (TEST INFRASTRUCTURE ONLY).

Plain, slow reference for one coarsening level of an SNN hypergraph and for
the (lambda - 1) connectivity objective, after Ronzani & Silvano, "GPU-Accelerated
Hypergraph Partitioning and Placement to Map SNNs on Neuromorphic Hardware".
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2609_07577_amd``); the only common input is the seeded generator in
``paper_2609_07577_amd.synth``, which holds none of the method's arithmetic.

The arithmetic lives in ``oracle.cpp`` (plain C++17); this module is ctypes
marshalling plus the level loop.  See that file's header for the paper passage
each function follows and for the readings R1-R7 of points the paper leaves
open.

Parity status: every function here is pinned by the tests in
``tests/test_oracle_*.py`` (hand-derived cases, brute force on tiny inputs,
closed forms and invariants).  Absolute level counts, match counts and
connectivity values at the full workload sizes have no printed value in the
paper; there they are pinned only through those invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_P = ctypes.c_void_p
_i32 = ctypes.c_int32


def build(force: bool = True) -> str:
    """Compile the oracle shared library in place (g++, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_level0_state.argtypes = [_i32, _i32, _P, _P, _P, _P, _P, _P, _P]
        lib.oracle_candidates.argtypes = [_i32, _i32, _P, _P, _P, _P, _P, _P, _P,
                                          _i32, _i32, _i32, _i32, _P, _P, _P, _i32, _P]
        lib.oracle_match.argtypes = [_i32, _P, _P, _P]
        lib.oracle_vmap_from_match.argtypes = [_i32, _P, _P]
        lib.oracle_vmap_from_match.restype = _i32
        lib.oracle_contract.argtypes = [_i32, _i32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _i32,
                                        _P, _P, _P, _P, _P, _P, _P, _P, _P]
        lib.oracle_connectivity.argtypes = [_i32, _P, _P, _P, _P]
        lib.oracle_connectivity.restype = ctypes.c_int64
        lib.oracle_partition_report.argtypes = [_i32, _i32, _P, _P, _P, _P, _P, _P, _P, _P,
                                                _i32, _i32, _i32, _i32, _P, _P, _P, _P]
        lib.oracle_refine_round.argtypes = [_i32, _i32, _P, _P, _P, _P, _P, _P, _P, _P, _i32,
                                            _i32, _i32, _i32, _P]
        lib.oracle_hilbert_cores.argtypes = [_i32, _i32, _P]
        lib.oracle_hilbert_cores.restype = _i32
        lib.oracle_initial_placement.argtypes = [_i32, _i32, _P, _P, _P, _i32, _i32, _P, _i32,
                                                 _P]
        lib.oracle_residual_distance.argtypes = [_i32, _i32, _P, _P, _P, _i32, _P]
        lib.oracle_residual_distance.restype = ctypes.c_int64
        lib.oracle_place_refine.argtypes = [_i32, _i32, _P, _P, _P, _i32, _i32, _P, _i32, _P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


@dataclass
class OLevel:
    """One level as the oracle holds it (host arrays).

    ``soff``/``sids`` is the explicit inbound-axon set of every super-node
    (CSR); its lengths are the ``ax`` values the GPU library carries.
    """
    V: int
    eoff: np.ndarray   # int64 [E+1]
    pins: np.ndarray   # uint32 [P]
    w: np.ndarray      # int32 [E]
    mult: np.ndarray   # int32 [E]
    size: np.ndarray   # int32 [V]
    syn: np.ndarray    # int32 [V]
    soff: np.ndarray   # int64 [V+1]
    sids: np.ndarray   # int32 [sum ax]

    @property
    def E(self) -> int:
        return int(self.eoff.shape[0] - 1)

    @property
    def P(self) -> int:
        return int(self.pins.shape[0])

    @property
    def ax(self) -> np.ndarray:
        return np.diff(self.soff).astype(np.int32)


def level0(g) -> OLevel:
    """Level-0 state of a generated SNN (size 1, syn = ax = in-degree, mult 1)."""
    lib = _load()
    V, E = g.n_vertices, g.n_edges
    eoff = np.ascontiguousarray(g.eoff, dtype=np.int64)
    pins = np.ascontiguousarray(g.pins, dtype=np.uint32)
    ndst = int(np.count_nonzero(pins >> 31))
    size = np.empty(V, np.int32)
    syn = np.empty(V, np.int32)
    mult = np.empty(E, np.int32)
    soff = np.empty(V + 1, np.int64)
    sids = np.empty(ndst, np.int32)
    lib.oracle_level0_state(V, E, _ptr(eoff), _ptr(pins), _ptr(size), _ptr(syn), _ptr(mult),
                            _ptr(soff), _ptr(sids))
    return OLevel(V, eoff, pins, np.ascontiguousarray(g.weight, dtype=np.int32), mult, size,
                  syn, soff, sids)


def candidates(L: OLevel, limits, query=None, nthreads: int = 0, seconds=None):
    """cand[n], cscore[n] per Eq. (12) for all vertices, or for ``query``.
    ``seconds``: optional float64 array of 2 receiving the wall time of the
    incidence build and of the per-vertex loop."""
    lib = _load()
    if query is None:
        nq, qp = L.V, None
    else:
        query = np.ascontiguousarray(query, dtype=np.int32)
        nq, qp = int(query.shape[0]), _ptr(query)
    cand = np.empty(nq, np.int32)
    cscore = np.empty(nq, np.int32)
    lib.oracle_candidates(L.V, L.E, _ptr(L.eoff), _ptr(L.pins), _ptr(L.w), _ptr(L.size),
                          _ptr(L.syn), _ptr(L.soff), _ptr(L.sids), limits.max_neurons,
                          limits.max_synapses, limits.max_axons, nq, qp, _ptr(cand),
                          _ptr(cscore), nthreads, None if seconds is None else _ptr(seconds))
    return cand, cscore


def match(cand: np.ndarray, cscore: np.ndarray) -> np.ndarray:
    """match[n] per Eq. (13)."""
    lib = _load()
    V = int(cand.shape[0])
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    cscore = np.ascontiguousarray(cscore, dtype=np.int32)
    out = np.empty(V, np.int32)
    rc = lib.oracle_match(V, _ptr(cand), _ptr(cscore), _ptr(out))
    if rc != 0:
        raise RuntimeError("candidate graph has a cycle longer than two")
    return out


def vmap_from_match(m: np.ndarray):
    lib = _load()
    m = np.ascontiguousarray(m, dtype=np.int32)
    vmap = np.empty(m.shape[0], np.int32)
    nc = lib.oracle_vmap_from_match(int(m.shape[0]), _ptr(m), _ptr(vmap))
    return vmap, int(nc)


def contract(L: OLevel, vmap: np.ndarray, n_coarse: int) -> OLevel:
    """Coarse level G_P for the vertex map ``vmap`` (any partition)."""
    lib = _load()
    vmap = np.ascontiguousarray(vmap, dtype=np.int32)
    E, P = L.E, L.P
    o_eoff = np.empty(E + 1, np.int64)
    o_pins = np.empty(max(P, 1), np.uint32)
    o_w = np.empty(max(E, 1), np.int32)
    o_mult = np.empty(max(E, 1), np.int32)
    o_size = np.empty(max(n_coarse, 1), np.int32)
    o_syn = np.empty(max(n_coarse, 1), np.int32)
    o_soff = np.empty(n_coarse + 1, np.int64)
    o_sids = np.empty(max(L.sids.shape[0], 1), np.int32)
    sizes = np.zeros(3, np.int64)
    rc = lib.oracle_contract(L.V, E, _ptr(L.eoff), _ptr(L.pins), _ptr(L.w), _ptr(L.mult),
                             _ptr(L.size), _ptr(L.syn), _ptr(L.soff), _ptr(L.sids), _ptr(vmap),
                             n_coarse, _ptr(o_eoff), _ptr(o_pins), _ptr(o_w), _ptr(o_mult),
                             _ptr(o_size), _ptr(o_syn), _ptr(o_soff), _ptr(o_sids), _ptr(sizes))
    if rc != 0:
        raise ValueError("vmap value out of range")
    e2, p2, s2 = (int(x) for x in sizes)
    return OLevel(n_coarse, o_eoff[: e2 + 1].copy(), o_pins[:p2].copy(), o_w[:e2].copy(),
                  o_mult[:e2].copy(), o_size[:n_coarse].copy(), o_syn[:n_coarse].copy(),
                  o_soff, o_sids[:s2].copy())


def connectivity(eoff: np.ndarray, pins: np.ndarray, w: np.ndarray, part: np.ndarray) -> int:
    """Eq. (1): sum_e w(e) * (number of distinct part values over e's pins - 1)."""
    lib = _load()
    eoff = np.ascontiguousarray(eoff, dtype=np.int64)
    pins = np.ascontiguousarray(pins, dtype=np.uint32)
    w = np.ascontiguousarray(w, dtype=np.int32)
    part = np.ascontiguousarray(part, dtype=np.int32)
    return int(lib.oracle_connectivity(int(eoff.shape[0] - 1), _ptr(eoff), _ptr(pins), _ptr(w),
                                       _ptr(part)))


def project(vmap: np.ndarray, part_coarse: np.ndarray) -> np.ndarray:
    """A partition of the coarser level seen on the finer one (Section 4.1,
    uncoarsening: a super-node's members start in the super-node's part):
    part_fine[v] = part_coarse[vmap[v]]."""
    return np.asarray(part_coarse, dtype=np.int32)[np.asarray(vmap, dtype=np.int64)]


@dataclass
class Report:
    """Eq. (1) and the Section 3 totals of every part of a partition."""
    conn: int
    size: np.ndarray
    syn: np.ndarray
    ax: np.ndarray
    summary: np.ndarray  # conn, max size, max syn, max ax, over Omega, Phi, Delta, parts


def partition_report(L: OLevel, part: np.ndarray, n_parts: int, limits) -> Report:
    lib = _load()
    part = np.ascontiguousarray(part, dtype=np.int32)
    summary = np.zeros(8, np.int64)
    size = np.empty(max(n_parts, 1), np.int32)
    syn = np.empty(max(n_parts, 1), np.int32)
    ax = np.empty(max(n_parts, 1), np.int32)
    rc = lib.oracle_partition_report(L.V, L.E, _ptr(L.eoff), _ptr(L.pins), _ptr(L.w),
                                     _ptr(L.size), _ptr(L.syn), _ptr(L.soff), _ptr(L.sids),
                                     _ptr(part), n_parts, limits.max_neurons,
                                     limits.max_synapses, limits.max_axons, _ptr(summary),
                                     _ptr(size), _ptr(syn), _ptr(ax))
    if rc != 0:
        raise ValueError("part value out of range")
    return Report(int(summary[0]), size[:n_parts], syn[:n_parts], ax[:n_parts], summary)


def refine_round(L: OLevel, part: np.ndarray, n_parts: int, limits):
    """One refinement round (Section 4.1, "Uncoarsening and Refinement") on a
    copy of ``part``.  Returns (new part, [proposals, moves applied, Eq. (1)
    decrease])."""
    lib = _load()
    out = np.array(part, dtype=np.int32, copy=True)
    ax = np.ascontiguousarray(L.ax, dtype=np.int32)
    info = np.zeros(3, np.int64)
    rc = lib.oracle_refine_round(L.V, L.E, _ptr(L.eoff), _ptr(L.pins), _ptr(L.w), _ptr(L.mult),
                                 _ptr(L.size), _ptr(L.syn), _ptr(ax), _ptr(out), n_parts,
                                 limits.max_neurons, limits.max_synapses, limits.max_axons,
                                 _ptr(info))
    if rc != 0:
        raise ValueError("part value out of range")
    return out, info


def refine(L: OLevel, part: np.ndarray, n_parts: int, limits, max_rounds: int = 16):
    """Refinement rounds on one level until a round moves nothing (at most
    ``max_rounds``).  Returns (part, rounds run, total Eq. (1) decrease)."""
    total, rounds = 0, 0
    for _ in range(max_rounds):
        part, info = refine_round(L, part, n_parts, limits)
        rounds += 1
        total += int(info[2])
        if info[1] == 0:
            break
    return part, rounds, total


def uncoarsen(h: "Hierarchy", limits, max_rounds: int = 16):
    """The uncoarsening of a hierarchy: the final super-nodes as initial
    parts, then level by level down to level 0, projection and refinement.
    Returns (level-0 partition, number of parts, per-level list of
    (level, Eq. (1) after projection, Eq. (1) after refinement, rounds))."""
    top = h.levels[-1].level
    n_parts = top.V
    part = np.arange(n_parts, dtype=np.int32)
    trace = []
    for li in range(len(h.levels) - 1, -1, -1):
        L = h.levels[li].level
        if li < len(h.levels) - 1:
            part = project(h.levels[li].vmap, part)
        before = connectivity(L.eoff, L.pins, L.w, part)
        part, rounds, dec = refine(L, part, n_parts, limits, max_rounds)
        trace.append((li, before, before - dec, rounds))
    return part, n_parts, trace


def hilbert_cores(width: int, height: int) -> np.ndarray:
    """Cores of the width x height lattice (core = x * height + y) in Hilbert
    order (Section 4.2, "Initial Placement")."""
    lib = _load()
    out = np.empty(width * height, np.int32)
    n = lib.oracle_hilbert_cores(width, height, _ptr(out))
    return out[:n]


def initial_placement(L: OLevel, width: int, height: int, order0: np.ndarray,
                      lp_rounds: int = 4) -> np.ndarray:
    """One start of the initial placement of a partitioned hypergraph G_P
    (its nodes are the parts): core of every node."""
    lib = _load()
    order0 = np.ascontiguousarray(order0, dtype=np.int32)
    core = np.empty(max(L.V, 1), np.int32)
    rc = lib.oracle_initial_placement(L.V, L.E, _ptr(L.eoff), _ptr(L.pins), _ptr(L.w), width,
                                      height, _ptr(order0), lp_rounds, _ptr(core))
    if rc != 0:
        raise ValueError("more nodes than cores")
    return core[:L.V]


def residual_distance(L: OLevel, height: int, core: np.ndarray) -> int:
    """Sum over hyperedges of eta(a) times the Manhattan distances of all
    unordered pairs of its pins' cores."""
    lib = _load()
    core = np.ascontiguousarray(core, dtype=np.int32)
    return int(lib.oracle_residual_distance(L.V, L.E, _ptr(L.eoff), _ptr(L.pins), _ptr(L.w),
                                            height, _ptr(core)))


def place_refine(L: OLevel, width: int, height: int, core: np.ndarray, max_rounds: int = 1000):
    """Swap refinement (Section 4.2) on a copy of ``core``.  Returns (core,
    [rounds, swaps applied, decrease of the residual distance])."""
    lib = _load()
    out = np.array(core, dtype=np.int32, copy=True)
    info = np.zeros(3, np.int64)
    lib.oracle_place_refine(L.V, L.E, _ptr(L.eoff), _ptr(L.pins), _ptr(L.w), width, height,
                            _ptr(out), max_rounds, _ptr(info))
    return out, info


def place(L: OLevel, width: int, height: int, orders: np.ndarray, lp_rounds: int = 4,
          max_rounds: int = 1000):
    """Multi-start placement: every start's initial placement and swap
    refinement; the start of least residual distance (lowest index on
    ties) is chosen.  ``orders`` [starts, V]: the random initial orders.
    Returns (core of every node, chosen start, residual distance of every
    start after refinement)."""
    finals, dists = [], []
    for order0 in orders:
        c0 = initial_placement(L, width, height, order0, lp_rounds)
        c1, _ = place_refine(L, width, height, c0, max_rounds)
        finals.append(c1)
        dists.append(residual_distance(L, height, c1))
    best = int(np.argmin(dists))
    return finals[best], best, np.array(dists, np.int64)


@dataclass
class LevelResult:
    level: OLevel
    cand: np.ndarray
    cscore: np.ndarray
    match: np.ndarray
    vmap: np.ndarray
    n_coarse: int
    any_candidate: bool
    coarse: OLevel | None = None


def coarsen_level(L: OLevel, limits, nthreads: int = 0) -> LevelResult:
    """One coarsening level: Eq. (12) candidates, Eq. (13) matching, G_P."""
    cand, cscore = candidates(L, limits, nthreads=nthreads)
    m = match(cand, cscore)
    vmap, nc = vmap_from_match(m)
    anyc = bool((cand >= 0).any())
    res = LevelResult(L, cand, cscore, m, vmap, nc, anyc)
    if anyc:
        res.coarse = contract(L, vmap, nc)
    return res


@dataclass
class Hierarchy:
    levels: list = field(default_factory=list)  # LevelResult per level, last has no candidate

    @property
    def n_levels(self) -> int:
        """Number of contractions performed."""
        return len(self.levels) - 1

    def final_partition(self) -> np.ndarray:
        """Composed vertex map from level 0 to the final level."""
        part = np.arange(self.levels[0].level.V, dtype=np.int32)
        for r in self.levels[:-1]:
            part = r.vmap[part]
        return part


def hierarchy(g_or_level, limits, max_levels: int = 1000, nthreads: int = 0) -> Hierarchy:
    """Coarsen until no vertex proposes a candidate (Section 4.1: when constraints
    forbid further merging the super-nodes form the initial partitions)."""
    L = g_or_level if isinstance(g_or_level, OLevel) else level0(g_or_level)
    h = Hierarchy()
    for _ in range(max_levels):
        r = coarsen_level(L, limits, nthreads=nthreads)
        h.levels.append(r)
        if not r.any_candidate:
            break
        L = r.coarse
    return h
