"""Brute-force definitions for tiny hypergraphs (test helper).

Every quantity is computed straight from its definition in Ronzani & Silvano,
"GPU-Accelerated Hypergraph Partitioning and Placement to Map SNNs on
Neuromorphic Hardware", by enumeration, with no data structure shared with the
C++ oracle.  Super-nodes are tracked as explicit sets of ORIGINAL neurons, and
every constraint is evaluated on the original hypergraph, so the propagated
state of the oracle (sizes, inbound sets) is checked against first principles.

Intended for inputs with at most a few dozen vertices.
"""
from __future__ import annotations

DST = 1 << 31


def edges_of(eoff, pins):
    """List of hyperedges as lists of (vertex, is_destination)."""
    out = []
    for e in range(len(eoff) - 1):
        out.append([(int(p) & (DST - 1), bool(int(p) & DST)) for p in pins[eoff[e]:eoff[e + 1]]])
    return out


class Orig:
    """The original (level-0) SNN: in(n) and the Section 3 constraints."""

    def __init__(self, n_vertices, eoff, pins):
        self.V = n_vertices
        self.edges = edges_of(eoff, pins)
        self.inb = [set() for _ in range(n_vertices)]  # in(n): axons with n as destination
        for e, pl in enumerate(self.edges):
            for v, d in pl:
                if d:
                    self.inb[v].add(e)

    def size(self, members):
        return len(members)

    def synapses(self, members):
        """sum over n in p of |in(n)| (inbound pins)."""
        return sum(len(self.inb[n]) for n in members)

    def axons(self, members):
        """|U_{n in p} in(n)| (distinct inbound hyperedges)."""
        s = set()
        for n in members:
            s |= self.inb[n]
        return len(s)

    def feasible(self, members, lim):
        return (self.size(members) <= lim.max_neurons
                and self.synapses(members) <= lim.max_synapses
                and self.axons(members) <= lim.max_axons)


def score(edges, w, n, m):
    """Eq. (12): sum of w(e) over e incident to n with m in e."""
    s = 0
    for e, pl in enumerate(edges):
        vs = {v for v, _ in pl}
        if n in vs and m in vs:
            s += int(w[e])
    return s


def neighbours(edges, n):
    out = set()
    for pl in edges:
        vs = {v for v, _ in pl}
        if n in vs:
            out |= vs
    out.discard(n)
    return out


def candidates(V, edges, w, members, orig, lim):
    """cand(n): valid neighbour of largest score, lowest id on ties."""
    cand = [-1] * V
    cs = [0] * V
    for n in range(V):
        best, bs = -1, 0
        for m in sorted(neighbours(edges, n)):
            if not orig.feasible(members[n] | members[m], lim):
                continue
            s = score(edges, w, n, m)
            if s > bs or (s == bs and m < best):
                best, bs = m, s
        cand[n], cs[n] = best, bs
    return cand, cs


def best_child(V, cand, edges, w, n):
    best, bs = -1, 0
    for m in range(V):
        if cand[m] == n:
            s = score(edges, w, n, m)
            if best < 0 or s > bs or (s == bs and m < best):
                best, bs = m, s
    return best


def match_eq13(V, cand, edges, w):
    """Eq. (13) by literal memoised recursion (first case takes precedence)."""
    memo = {}

    def match(n):
        if n in memo:
            return memo[n]
        c = cand[n]
        if c >= 0 and (cand[c] == n or match(c) == n):
            r = c
        else:
            r = best_child(V, cand, edges, w, n)
        memo[n] = r
        return r

    return [match(n) for n in range(V)]


def match_walk(V, cand, edges, w):
    """Sequential simulation of the walk procedure of Section 4.1: each node
    acquires its candidate (a contested candidate keeps the acquirer of best
    score, lowest id on ties), two-cycles are matched first, then the forest is
    walked downward from the roots, matching a node with its acquirer when
    both are still free."""
    acq = [best_child(V, cand, edges, w, n) for n in range(V)]
    m = [-1] * V
    roots = [n for n in range(V) if cand[n] >= 0 and cand[cand[n]] == n]
    for n in roots:
        m[n] = cand[n]
    frontier = list(roots)
    seen = set(frontier)
    while frontier:
        nxt = []
        for c in frontier:
            children = sorted(x for x in range(V) if cand[x] == c and x not in seen)
            if m[c] < 0 and acq[c] >= 0 and m[acq[c]] < 0:
                m[c] = acq[c]
                m[acq[c]] = c
            for x in children:
                seen.add(x)
                nxt.append(x)
        frontier = nxt
    return m


def vmap_from_match(V, m):
    reps = [n for n in range(V) if m[n] < 0 or n < m[n]]
    rank = {r: i for i, r in enumerate(reps)}
    return [rank[n if (m[n] < 0 or n < m[n]) else m[n]] for n in range(V)], len(reps)


def contract(edges, w, mult, vmap):
    """Coarse hyperedges: distinct coarse vertices with OR-ed destination flags,
    fewer than two dropped, identical (vertex, flag) lists merged (weights and
    multiplicities summed), ordered by smallest fine hyperedge."""
    order, agg = [], {}
    for e, pl in enumerate(edges):
        flags = {}
        for v, d in pl:
            c = vmap[v]
            flags[c] = flags.get(c, False) or d
        if len(flags) < 2:
            continue
        key = tuple(sorted(flags.items()))
        if key not in agg:
            agg[key] = [0, 0]
            order.append(key)
        agg[key][0] += int(w[e])
        agg[key][1] += int(mult[e])
    new_edges = [list(k) for k in order]
    return new_edges, [agg[k][0] for k in order], [agg[k][1] for k in order]


def connectivity(edges, w, part):
    """Eq. (1)."""
    return sum(int(w[e]) * (len({part[v] for v, _ in pl}) - 1) for e, pl in enumerate(edges))


def hierarchy(n_vertices, eoff, pins, weight, lim, max_levels=64):
    """Full coarsening loop by brute force.  Returns a list of per-level dicts."""
    orig = Orig(n_vertices, eoff, pins)
    edges = orig.edges
    w = [int(x) for x in weight]
    mult = [1] * len(edges)
    members = [frozenset([n]) for n in range(n_vertices)]
    V = n_vertices
    out = []
    for _ in range(max_levels):
        cand, cs = candidates(V, edges, w, members, orig, lim)
        m = match_eq13(V, cand, edges, w)
        rec = dict(V=V, edges=edges, w=w, mult=mult, members=members, cand=cand, cscore=cs,
                   match=m, match_walk=match_walk(V, cand, edges, w))
        out.append(rec)
        if all(c < 0 for c in cand):
            break
        vmap, nc = vmap_from_match(V, m)
        rec["vmap"], rec["n_coarse"] = vmap, nc
        new_members = [set() for _ in range(nc)]
        for n in range(V):
            new_members[vmap[n]] |= members[n]
        members = [frozenset(s) for s in new_members]
        edges, w, mult = contract(edges, w, mult, vmap)
        V = nc
    return out, orig


def refine_round(level_edges, w, part, n_parts, members, orig, lim):
    """One refinement round (Section 4.1, "Uncoarsening and Refinement") by
    enumeration.  ``level_edges``: the level's hyperedges (vertex, flag)
    lists; ``members``: the original neurons of every level vertex; every
    limit is evaluated on original neurons (``orig``).  Each gain is the
    drop of Eq. (1) recomputed from scratch.  Returns (new part, [proposals,
    moves applied, Eq. (1) decrease])."""
    V = len(members)
    part = [int(x) for x in part]

    def conn(pt):
        return connectivity(level_edges, w, pt)

    def orig_members(pt):
        mem = [set() for _ in range(n_parts)]
        for v in range(V):
            mem[pt[v]] |= members[v]
        return mem

    base = conn(part)
    mem0 = orig_members(part)
    within0 = [(orig.size(m) <= lim.max_neurons, orig.synapses(m) <= lim.max_synapses,
                orig.axons(m) <= lim.max_axons) for m in mem0]
    moves = []
    for n in range(V):
        a = part[n]
        adj = set()
        for pl in level_edges:
            vs = [v for v, _ in pl]
            if n in vs:
                adj |= {part[v] for v in vs}
        adj.discard(a)
        best = None
        for p in sorted(adj):
            if not orig.feasible(mem0[p] | members[n], lim):
                continue
            pt = list(part)
            pt[n] = p
            gain = base - conn(pt)
            if best is None or gain > best[0]:
                best = (gain, n, a, p)
        if best is not None:
            moves.append(best)
    moves.sort(key=lambda m: (-m[0], m[1]))
    best_cum, best_len = 0, 0
    pt = list(part)
    for i, (_, n, a, p) in enumerate(moves):
        pt[n] = p
        cum = base - conn(pt)
        mem = orig_members(pt)
        ok = all(not (within0[q][0] and orig.size(mem[q]) > lim.max_neurons)
                 and not (within0[q][1] and orig.synapses(mem[q]) > lim.max_synapses)
                 and not (within0[q][2] and orig.axons(mem[q]) > lim.max_axons)
                 for q in range(n_parts))
        if ok and cum > 0 and cum > best_cum:
            best_cum, best_len = cum, i + 1
    out = list(part)
    for _, n, a, p in moves[:best_len]:
        out[n] = p
    return out, [len(moves), best_len, best_cum]


def manhattan(a, b, height):
    return abs(a // height - b // height) + abs(a % height - b % height)


def residual_distance(level_edges, w, core, height):
    """Sum over hyperedges of w(e) times the distances of all unordered pin
    pairs (the placement objective)."""
    d = 0
    for e, pl in enumerate(level_edges):
        vs = [v for v, _ in pl]
        s = 0
        for i in range(len(vs)):
            for j in range(i + 1, len(vs)):
                s += manhattan(core[vs[i]], core[vs[j]], height)
        d += int(w[e]) * s
    return d


def place_refine_round(level_edges, w, core, width, height):
    """One swap-refinement round (Section 4.2) by enumeration: each tension is
    the decrease of the residual distance of a swap computed from scratch;
    the matching is Eq. 13 by literal recursion over cores; each prefix is
    applied and evaluated from scratch.  Returns (new core, applied)."""
    V = len(core)
    C = width * height
    occ = [-1] * C
    for p in range(V):
        occ[core[p]] = p
    base = residual_distance(level_edges, w, core, height)

    def swapped(cr, oc, a, b):
        cr = list(cr)
        pa, pb = oc[a], oc[b]
        if pa >= 0:
            cr[pa] = b
        if pb >= 0:
            cr[pb] = a
        return cr

    def tension(a, b):
        return base - residual_distance(level_edges, w, swapped(core, occ, a, b), height)

    cand, score = [-1] * C, [0] * C
    for h in range(C):
        if occ[h] < 0:
            continue
        x, y = divmod(h, height)
        best, bk = 0, -1
        for nx, ny in ((x - 1, y), (x, y - 1), (x, y + 1), (x + 1, y)):
            if 0 <= nx < width and 0 <= ny < height:
                k = nx * height + ny
                t = tension(h, k)
                if t > best:
                    best, bk = t, k
        cand[h], score[h] = bk, best
    m = match_eq13_scores(cand, score)
    swaps = sorted(((tension(h, m[h]), h, m[h]) for h in range(C) if m[h] > h),
                   key=lambda s: (-s[0], s[1]))
    cur = list(core)
    best_cum, best_len = 0, 0
    for i in range(len(swaps)):
        trial = list(core)
        oc = list(occ)
        for _, a, b in swaps[:i + 1]:
            trial = swapped(trial, oc, a, b)
            oc[a], oc[b] = oc[b], oc[a]
        cum = base - residual_distance(level_edges, w, trial, height)
        if cum > best_cum:
            best_cum, best_len = cum, i + 1
    oc = list(occ)
    for _, a, b in swaps[:best_len]:
        cur = swapped(cur, oc, a, b)
        oc[a], oc[b] = oc[b], oc[a]
    return cur, best_len, best_cum


def match_eq13_scores(cand, score):
    """Eq. (13) by literal memoised recursion, for given candidates and the
    score of each candidate arc (best child: largest score, lowest id)."""
    n_items = len(cand)
    memo = {}

    def best_child(n):
        kids = [m for m in range(n_items) if cand[m] == n]
        if not kids:
            return -1
        return min(kids, key=lambda m: (-score[m], m))

    def match(n):
        if n in memo:
            return memo[n]
        c = cand[n]
        r = c if c >= 0 and (cand[c] == n or match(c) == n) else best_child(n)
        memo[n] = r
        return r

    return [match(n) for n in range(n_items)]


def initial_placement(level_edges, w, V, hilbert, order0, lp_rounds):
    """Initial placement (Section 4.2) by enumeration: recursive bisection
    where each node's gain is the drop of the section's cut recomputed from
    scratch after moving it alone, label-propagation swaps of the best pairs,
    then folding by connection weights counted from scratch; the i-th node of
    the result on core hilbert[i]."""
    seq = [int(x) for x in order0]
    pins = [{v for v, _ in pl} for pl in level_edges]

    def cut(A, Bs):
        return sum(int(w[e]) for e, ps in enumerate(pins) if ps & A and ps & Bs)

    sections = [(0, V)]
    while sections:
        nxt = []
        for st, ln in sections:
            if ln < 2:
                continue
            nl = ln - ln // 2
            for _ in range(lp_rounds):
                L, R = set(seq[st:st + nl]), set(seq[st + nl:st + ln])
                base = cut(L, R)
                gl = sorted((-(base - cut(L - {u}, R | {u})), u) for u in L)
                gr = sorted((-(base - cut(L | {u}, R - {u})), u) for u in R)
                pos = {seq[i]: i for i in range(st, st + ln)}
                done = 0
                for (a, u), (b, v) in zip(gl, gr):
                    if -a - b <= 0:
                        break
                    seq[pos[u]], seq[pos[v]] = seq[pos[v]], seq[pos[u]]
                    done += 1
                if not done:
                    break
            nxt += [(st, nl), (st + nl, ln - nl)]
        sections = nxt

    def fold(st, ln, side, us, ul):
        if ln == 1:
            return [seq[st]]
        nl = ln - ln // 2
        c0 = fold(st, nl, 0, st + nl, ln - nl)
        c1 = fold(st + nl, ln - nl, 1, st, nl)
        out = c0 + c1
        if side >= 0:
            u = set(seq[us:us + ul])
            k0, k1 = cut(set(seq[st:st + nl]), u), cut(set(seq[st + nl:st + ln]), u)
            if (side == 0 and k0 > k1) or (side == 1 and k1 > k0):
                out = out[::-1]
        return out

    order = fold(0, V, -1, 0, 0) if V else []
    core = [0] * V
    for i, v in enumerate(order):
        core[v] = int(hilbert[i])
    return core
