"""MS-complex graph and persistence-driven simplification, serial and plain
-- TEST INFRASTRUCTURE ONLY (tests and the smoke check; never the product).

Graph (Section 3.5, "Data structure"): the critical points as nodes, numbered
in the order of the critical list (index, cell id), and for every node its
arcs down (to index - 1) and up (to index + 1) with multiplicities, taken
from the oracle's M10, M32 and P = M21^T.

Simplification (Section 2.1: cancellation of critical pairs joined by a
single arc, ordered by the difference of their function values; Section 4:
pairs joined by several arcs would strangle and are not cancelled).  A
cancellation of (p, q), index(p) = index(q) + 1, removes p, q and their arcs
and reroutes the descending arcs of p to the destinations of the ascending
arcs of q: each other upper neighbour s of q gains m(s, q) * m(p, r) paths to
each other lower neighbour r of p (counts saturate at 2^64 - 1, like every
path count here).

Serial order: while some live arc (p, q) has multiplicity 1 and persistence
|f(p) - f(q)| (float64) below the threshold, cancel the least such arc in the
order (persistence, p, q).  The heap below only finds that least arc faster:
persistence never changes, multiplicities only grow and nodes only die, so
every valid arc is in the heap and an entry that is no longer valid is
dropped when it comes up.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass, field

U64_MAX = (1 << 64) - 1


@dataclass
class Graph:
    index: list        # per node
    value: list        # per node (float32 values as Python floats)
    cell: list
    alive: list
    down: list = field(default_factory=list)   # per node: dict nbr -> multiplicity
    up: list = field(default_factory=list)
    log: list = field(default_factory=list)    # (upper, lower, persistence)

    def pers(self, a, b):
        return abs(float(self.value[a]) - float(self.value[b]))

    def live_arcs(self, node, direction):
        if not self.alive[node]:
            return {}
        d = self.down[node] if direction == "down" else self.up[node]
        return {n: m for n, m in d.items() if self.alive[n]}


def from_complex(cx) -> Graph:
    """Graph of an oracle.Complex (crit, m10, m32, p)."""
    cnt = [int(c) for c in cx.crit.count]
    first = [0, cnt[0], cnt[0] + cnt[1], cnt[0] + cnt[1] + cnt[2]]
    n = sum(cnt)
    g = Graph(index=[int(i) for i in cx.crit.index], value=[float(v) for v in cx.crit.value],
              cell=[int(c) for c in cx.crit.id], alive=[True] * n,
              down=[{} for _ in range(n)], up=[{} for _ in range(n)])
    # M10: rows 1-saddles, cols minima; P: rows 1-saddles, cols 2-saddles;
    # M32: rows maxima, cols 2-saddles
    for (rows, cols, vals, upper_k, lower_k, upper_is_row) in (
            (cx.m10.row, cx.m10.col, cx.m10.val, 1, 0, True),
            (cx.p.row, cx.p.col, cx.p.val, 2, 1, False),
            (cx.m32.row, cx.m32.col, cx.m32.val, 3, 2, True)):
        for r, c, v in zip(rows, cols, vals):
            u, l = (int(r), int(c)) if upper_is_row else (int(c), int(r))
            u += first[upper_k]
            l += first[lower_k]
            g.down[u][l] = int(v)
            g.up[l][u] = int(v)
    return g


def cancel(g: Graph, u: int, l: int):
    """Cancels the pair (u upper, l lower); returns the arcs it creates or
    changes as (upper, lower) pairs."""
    U = [(s, m) for s, m in g.up[l].items() if g.alive[s] and s != u]
    D = [(r, m) for r, m in g.down[u].items() if g.alive[r] and r != l]
    touched = []
    for s, a in U:
        for r, b in D:
            m = min(g.down[s].get(r, 0) + min(a * b, U64_MAX), U64_MAX)
            g.down[s][r] = m
            g.up[r][s] = m
            touched.append((s, r))
    g.alive[u] = False
    g.alive[l] = False
    g.log.append((u, l, g.pers(u, l)))
    return touched


def valid(g: Graph, u: int, l: int, threshold: float) -> bool:
    return g.alive[u] and g.alive[l] and g.down[u].get(l, 0) == 1 and g.pers(u, l) < threshold


def simplify(g: Graph, threshold: float) -> Graph:
    """Serial persistence-ordered cancellation (module docstring)."""
    heap = []
    for u in range(len(g.index)):
        for l in g.down[u]:
            if valid(g, u, l, threshold):
                heap.append((g.pers(u, l), u, l))
    heapq.heapify(heap)
    while heap:
        p, u, l = heapq.heappop(heap)
        if not valid(g, u, l, threshold):
            continue
        for s, r in cancel(g, u, l):
            if valid(g, s, r, threshold):
                heapq.heappush(heap, (g.pers(s, r), s, r))
    return g


def live_graph(g: Graph):
    """Canonical form of the live part: {node: (index, {down nbr: mult})}."""
    return {i: (g.index[i], g.live_arcs(i, "down")) for i in range(len(g.index)) if g.alive[i]}
