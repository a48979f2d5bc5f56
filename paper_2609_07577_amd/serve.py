"""Serving mapping requests with continuous batching.

A request is one hypergraph (a level with state, resident on the device) to
be coarsened to the end (Section 4.1).  The server keeps one hg_batch: a
request is admitted as soon as the batch has room for it (slots, vertices,
hyperedges, pins: the batch's HBM footprint is fixed at creation, so the
room is what is left of it), requests that arrive while others are on the
GPU join the next union step, finished ones are read out and their space is
reclaimed by compaction.  Every request's result is the same as a run on
its own (the graphs of a batch share no hyperedge).
"""
from __future__ import annotations

import collections
import time

from . import hg


class Server:
    def __init__(self, ctx: hg.Context, max_graphs: int, cap_vertices: int, cap_edges: int,
                 cap_pins: int, levels_per_step: int = 4, use_graph: bool = True,
                 compact_every: int = 16):
        self.ctx = ctx
        self.batch = hg.Batch(ctx, max_graphs, cap_vertices, cap_edges, cap_pins)
        self.cap = (max_graphs, cap_vertices, cap_edges, cap_pins)
        self.levels_per_step = levels_per_step
        self.use_graph = use_graph
        self.compact_every = compact_every
        self.queue = collections.deque()  # (request id, level, limits, arrival time)
        self.running = {}                  # slot -> (request id, arrival time, pins)
        self.released = 0                  # read out since the last compaction

    def bytes(self) -> int:
        return self.batch.bytes()

    def submit(self, rid, level: hg.DeviceLevel, limits, arrival: float):
        self.queue.append((rid, level, limits, arrival))

    def _admit(self):
        """Admit queued requests in arrival order while the batch has room
        (the library checks slots, vertices, hyperedges and pins against the
        footprint fixed at creation and reports HG_ERR_CAPACITY)."""
        admitted = 0
        while self.queue:
            rid, L, lim, arr = self.queue[0]
            try:
                slot = self.batch.add(L, lim)
            except hg.HgError as e:
                if e.code != 3:
                    raise
                if self.released:
                    self._compact()
                    continue
                if not self.running:
                    raise ValueError(f"request {rid} is larger than the server's capacity")
                break
            self.queue.popleft()
            self.running[slot] = (rid, arr, L.P)
            admitted += 1
        return admitted

    def _compact(self):
        self.batch.compact()
        self.released = 0

    def step(self):
        """Admit what fits, run one union step, collect finished requests.
        Returns [(request id, arrival, finish time, part, n_parts, n_levels, pins)]."""
        self._admit()
        if not self.running:
            return []
        self.batch.step(self.levels_per_step, self.use_graph)
        done, _ = self.batch.done()
        now = time.perf_counter()
        out = []
        for s in done:
            rid, arr, pins = self.running.pop(s)
            part, n_parts, n_levels = self.batch.result(s)
            out.append((rid, arr, now, part, n_parts, n_levels, pins))
            self.released += 1
        if self.released >= self.compact_every:
            self._compact()
        return out

    def idle(self) -> bool:
        return not self.queue and not self.running

    def close(self):
        self.batch.close()
