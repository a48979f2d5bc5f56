"""Seeded synthetic SNN hypergraphs (level-0 inputs).

A spiking network becomes a hypergraph with one hyperedge per axon: the source
neuron plus its synapse targets (paper, Section 2, "SNN and Hardware Models").
This module only draws random numbers and lays out arrays.  It holds none of the
coarsening arithmetic and is the one input source that both the CPU oracle and
the GPU library consume.

Layout of a generated level (host numpy arrays):

* ``eoff``   int64  [E+1]  hyperedge offsets into ``pins``
* ``pins``   uint32 [P]    ``vertex_id | (is_destination << 31)``, ascending id
* ``weight`` int32  [E]    spike rate (>= 1)

The big generators are C++ (``synth.cpp``) with counter-based SplitMix64 draws,
so outputs do not depend on the thread count.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.cpp")
_LIB = os.path.join(_HERE, "libhgsynth.so")

K_LAYERED, K_CONV, K_POWERLAW, K_BATCHGRAPH, K_UNIFORM = 1, 2, 3, 4, 5


class _Params(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("layers", ctypes.c_int32), ("width", ctypes.c_int32),
        ("height", ctypes.c_int32), ("channels", ctypes.c_int32),
        ("fan_min", ctypes.c_int32), ("fan_max", ctypes.c_int32),
        ("n", ctypes.c_int32), ("dmin", ctypes.c_int32), ("dmax", ctypes.c_int32),
        ("w_min", ctypes.c_int32), ("w_max", ctypes.c_int32), ("w_mode", ctypes.c_int32),
        ("n_max", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("graph", ctypes.c_uint64),
        ("alpha", ctypes.c_double), ("inhib_frac", ctypes.c_double),
        ("w_mean", ctypes.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile the generator shared library in place."""
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
        lib.synth_sizes.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
        lib.synth_fill.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class Level0:
    """A generated level-0 hypergraph (host arrays)."""
    n_vertices: int
    eoff: np.ndarray
    pins: np.ndarray
    weight: np.ndarray
    name: str = ""

    @property
    def n_edges(self) -> int:
        return int(self.eoff.shape[0] - 1)

    @property
    def n_pins(self) -> int:
        return int(self.pins.shape[0])


def _generate(name: str, **kw) -> Level0:
    p = _Params()
    p.kind = kw.get("kind")
    for k, v in kw.items():
        if k != "kind":
            setattr(p, k, v)
    lib = _load()
    V, E, P = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    lib.synth_sizes(ctypes.byref(p), ctypes.byref(V), ctypes.byref(E), ctypes.byref(P))
    eoff = np.empty(E.value + 1, dtype=np.int64)
    pins = np.empty(P.value, dtype=np.uint32)
    w = np.empty(E.value, dtype=np.int32)
    lib.synth_fill(ctypes.byref(p), eoff.ctypes.data, pins.ctypes.data, w.ctypes.data)
    return Level0(V.value, eoff, pins, w, name)


def layered(seed: int, layers: int = 4, width: int = 1024, fanout: int = 64,
            w_min: int = 1, w_max: int = 100) -> Level0:
    """Feed-forward layers; each non-final neuron targets ``fanout`` distinct
    uniform neurons of the next layer; weight uniform in [w_min, w_max]."""
    return _generate(f"layered{layers}x{width}f{fanout}s{seed}", kind=K_LAYERED,
                     layers=layers, width=width, fan_min=fanout, fan_max=fanout,
                     w_min=w_min, w_max=w_max, w_mode=0, seed=seed)


def conv(seed: int, layers: int = 4, height: int = 64, width: int = 64, channels: int = 16,
         w_max: int = 1000) -> Level0:
    """Convolutional layers; each non-final neuron targets the 3x3 window (clipped
    at borders) over all channels of the next layer; weight log-uniform 1..w_max."""
    return _generate(f"conv{layers}x{height}x{width}x{channels}s{seed}", kind=K_CONV,
                     layers=layers, width=width, height=height, channels=channels,
                     w_max=w_max, w_mode=1, seed=seed)


def powerlaw(seed: int, n: int = 2_000_000, dmin: int = 20, dmax: int = 10_000,
             alpha: float = 2.1, inhib_frac: float = 0.2, w_mean: float = 50.0) -> Level0:
    """Recurrent network: out-degree from a discrete power law d^-alpha on
    [dmin, dmax], distinct uniform targets among the other neurons, exponential
    weight with mean ``w_mean`` (rounded up), a fraction ``inhib_frac`` of the
    neurons halved (rounding up)."""
    return _generate(f"powerlaw{n}d{dmin}-{dmax}s{seed}", kind=K_POWERLAW, n=n,
                     dmin=dmin, dmax=dmax, alpha=alpha, inhib_frac=inhib_frac,
                     w_mean=w_mean, w_mode=2, seed=seed)


def batch_graph(seed: int, g: int, n_min: int = 10_000, n_max: int = 500_000,
                fan_min: int = 16, fan_max: int = 256, w_min: int = 1,
                w_max: int = 100) -> Level0:
    """Graph ``g`` of the mixed batch: feed-forward (4 equal layers) or recurrent
    by a fair coin, neuron count log-uniform in [n_min, n_max), per-neuron fan-out
    uniform in [fan_min, fan_max], weight uniform in [w_min, w_max]."""
    return _generate(f"batch{seed}g{g}", kind=K_BATCHGRAPH, n=n_min, n_max=n_max,
                     fan_min=fan_min, fan_max=fan_max, w_min=w_min, w_max=w_max,
                     w_mode=0, seed=seed, graph=g)


def uniform(seed: int, n: int, fan_min: int, fan_max: int, w_min: int = 1,
            w_max: int = 100, graph: int = 0) -> Level0:
    """Small recurrent network with uniform out-degree (test sizes)."""
    return _generate(f"uniform{n}f{fan_min}-{fan_max}s{seed}", kind=K_UNIFORM, n=n,
                     fan_min=fan_min, fan_max=fan_max, w_min=w_min, w_max=w_max,
                     w_mode=0, seed=seed, graph=graph)


def tiny_random(seed: int, n: int, p_axon: float = 0.8, max_fan: int = 4,
                w_max: int = 5) -> Level0:
    """Tiny irregular SNN for exhaustive checks: each neuron has an axon with
    probability ``p_axon``; the axon has 0..max_fan distinct targets; weights
    are small so that ties are frequent."""
    rng = np.random.default_rng(seed)
    eoff = [0]
    pins: list[int] = []
    w: list[int] = []
    for src in range(n):
        if rng.random() >= p_axon:
            continue
        others = [v for v in range(n) if v != src]
        k = int(rng.integers(0, min(max_fan, len(others)) + 1))
        tg = sorted(rng.choice(others, size=k, replace=False).tolist()) if k else []
        members = sorted([(src, 0)] + [(t, 1) for t in tg])
        pins.extend(v | (d << 31) for v, d in members)
        eoff.append(len(pins))
        w.append(int(rng.integers(1, w_max + 1)))
    return Level0(n, np.array(eoff, dtype=np.int64), np.array(pins, dtype=np.uint32),
                  np.array(w, dtype=np.int32), f"tiny{n}s{seed}")


def from_axons(n: int, axons: list[tuple[int, list[int], int]]) -> Level0:
    """Hand-written hypergraph: ``axons`` is a list of (source, targets, weight)."""
    eoff = [0]
    pins: list[int] = []
    w = []
    for src, tg, wt in axons:
        members = sorted([(src, 0)] + [(t, 1) for t in tg])
        pins.extend(v | (d << 31) for v, d in members)
        eoff.append(len(pins))
        w.append(wt)
    return Level0(n, np.array(eoff, dtype=np.int64), np.array(pins, dtype=np.uint32),
                  np.array(w, dtype=np.int32), "hand")


@dataclass(frozen=True)
class Limits:
    """Per-core limits: neurons (Omega), synapses (Phi), distinct input axons (Delta)."""
    max_neurons: int
    max_synapses: int
    max_axons: int


# The workloads this project is measured on.
LIMITS = {
    "layered": Limits(256, 16_384, 1_024),
    "conv": Limits(1_024, 65_536, 4_096),
    "powerlaw": Limits(4_096, 262_144, 16_384),
    "batch": Limits(512, 32_768, 2_048),
}


def hub_graph(seed: int, n: int, fan: int, n_hubs: int, hub_p: float, w_max: int = 100,
              skew: float = 0.0) -> Level0:
    """Recurrent network with a few hub neurons (test sizes).

    Every neuron's axon reaches ``fan`` distinct other neurons, drawn with
    probability proportional to (id + 1)^-skew (uniform for skew 0), and in
    addition each of ``n_hubs`` hub neurons with probability ``hub_p``, so
    that the hubs have about ``hub_p * n`` inbound axons.  Weights uniform in
    [1, w_max]."""
    rng = np.random.default_rng(seed)
    hubs = np.arange(n_hubs, dtype=np.int64) * (n // max(n_hubs, 1)) + 7
    cdf = None
    if skew > 0:
        cdf = np.cumsum((np.arange(n, dtype=np.float64) + 1.0) ** -skew)
        cdf /= cdf[-1]
    eoff = [0]
    pins = []
    w = np.empty(n, dtype=np.int32)
    for s in range(n):
        if cdf is None:
            t = rng.choice(n - 1, size=fan, replace=False)
            t = t + (t >= s)
        else:
            # draws with replacement until fan distinct others are found,
            # kept in the order they were drawn
            t = np.empty(0, dtype=np.int64)
            while t.shape[0] < fan:
                d = np.searchsorted(cdf, rng.random(4 * fan), side="right")
                d = np.minimum(d, n - 1)
                d = np.concatenate([t, d[d != s]])
                _, first = np.unique(d, return_index=True)
                t = d[np.sort(first)]
            t = t[:fan]
        extra = hubs[rng.random(n_hubs) < hub_p]
        ids = np.union1d(np.union1d(t, extra[extra != s]), [s]).astype(np.uint32)
        flag = (ids != s).astype(np.uint32) << np.uint32(31)
        pins.append(ids | flag)
        eoff.append(eoff[-1] + ids.shape[0])
        w[s] = int(rng.integers(1, w_max + 1))
    return Level0(n, np.array(eoff, dtype=np.int64), np.concatenate(pins).astype(np.uint32), w,
                  f"hub{n}f{fan}h{n_hubs}s{seed}")


def start_orders(seed: int, n_nodes: int, n_starts: int) -> np.ndarray:
    """Random initial node orders of the multi-start placement: n_starts
    seeded permutations of 0..n_nodes-1 (int32 [n_starts, n_nodes])."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(n_nodes) for _ in range(n_starts)]).astype(np.int32) \
        if n_starts > 0 else np.zeros((0, n_nodes), np.int32)


def gp_graph(seed: int, n_nodes: int, n_edges: int, fan_min: int = 2, fan_max: int = 24,
             w_max: int = 100, local: float = 0.7, span: int = 32) -> Level0:
    """A partitioned hypergraph G_P for placement: n_nodes parts, n_edges
    hyperedges, each from a uniform source part to fan targets (fan uniform
    in [fan_min, fan_max], capped at n_nodes - 1), a target within ``span``
    ids of the source with probability ``local`` (the id locality of parts
    cut from layered networks) and uniform otherwise; distinct pins;
    weights (spike rates) uniform in [1, w_max]."""
    rng = np.random.default_rng(seed)
    eoff = [0]
    pins: list[np.ndarray] = []
    w = rng.integers(1, w_max + 1, size=n_edges).astype(np.int32)
    for _ in range(n_edges):
        src = int(rng.integers(0, n_nodes))
        fan = int(rng.integers(fan_min, fan_max + 1))
        fan = max(0, min(fan, n_nodes - 1))
        tg: set[int] = set()
        while len(tg) < fan:
            if rng.random() < local:
                t = src + int(rng.integers(-span, span + 1))
                if t < 0 or t >= n_nodes:
                    continue
            else:
                t = int(rng.integers(0, n_nodes))
            if t != src:
                tg.add(t)
        ids = np.array(sorted(tg | {src}), dtype=np.int64)
        flags = (ids != src).astype(np.int64) << 31
        pins.append((ids | flags).astype(np.uint32))
        eoff.append(eoff[-1] + len(ids))
    P = np.concatenate(pins) if pins else np.zeros(0, np.uint32)
    return Level0(n_nodes, np.array(eoff, dtype=np.int64), P, w, f"gp{n_nodes}s{seed}")
