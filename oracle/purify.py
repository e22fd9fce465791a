"""Purification of a transport plan to a basic (acyclic) one -- CPU oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 2.2 recalls that the bipartite graph of any vertex of the transport
polytope, zero flows removed, is acyclic, so an optimal plan exists with at most
m+n-1 nonzeros.  The interior-point iterates converge to a point of the optimal
face, which need not be a vertex when the LP is degenerate.  This module walks
from such a plan to a vertex without increasing the cost: every cycle of the
support is cancelled by pushing flow around it in the direction that does not
increase the cost, until one edge of the cycle reaches zero.  Pushing flow
around a cycle of the bipartite graph leaves every row and column sum unchanged.

The steps are written plainly:

1. Kruskal: scan the edges by decreasing flow (ties: lower variable index
   first) and keep those that join two different trees; this is a
   maximum-flow spanning forest F.  Every other edge e closes exactly one cycle
   with F.
2. For each non-forest edge e = (i, j), walk the forest path from column node j
   back to row node i.  Along the cycle "e, path" the signs alternate: raising
   the flow on e by t lowers the 1st, 3rd, ... path edges and raises the 2nd,
   4th, ... ones by t.  The cost changes by t * (c_e + sum c_plus - sum c_minus),
   an exact integer for integer costs (a correctly rounded sum otherwise).
3. If that change is < 0 push t > 0 ("+" direction), else, on a tie too, push
   in the "-" direction (e decreases: on a tie either direction keeps the cost,
   and e, the smallest flow on its cycle of the maximum-flow forest, then
   usually leaves, so the forest stays); t is the smallest flow among the edges
   that decrease (ties: lowest variable index).  That bottleneck edge is set to
   exactly 0 and leaves; if it was a forest edge, e takes its place in F.
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np


class _DSU:
    def __init__(self, n):
        self.p = list(range(n))

    def find(self, x):
        p = self.p
        while p[x] != x:
            p[x] = p[p[x]]
            x = p[x]
        return x

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra == rb:
            return False
        self.p[ra] = rb
        return True


def is_forest(rows, cols, m, n) -> bool:
    """True when the bipartite graph with edges (rows[k], cols[k]) has no cycle."""
    d = _DSU(m + n)
    for i, j in zip(np.asarray(rows).tolist(), np.asarray(cols).tolist()):
        if not d.union(int(i), m + int(j)):
            return False
    return True


def _forest_path(adj, src, dst):
    """Edges of the unique forest path src -> dst, in walking order."""
    prev = {src: (-1, -1)}
    q = deque([src])
    while q:
        u = q.popleft()
        if u == dst:
            break
        for v, e in adj[u].items():
            if v not in prev:
                prev[v] = (u, e)
                q.append(v)
    if dst not in prev:
        raise RuntimeError("purify: endpoints not connected in the forest")
    path = []
    v = dst
    while v != src:
        u, e = prev[v]
        path.append(e)
        v = u
    path.reverse()
    return path


def purify_to_forest(rows, cols, flows, costs, m, n):
    """Cancel every cycle of the plan's support; returns (rows, cols, flows).

    rows, cols: int arrays (0-based source / target of each edge), flows >= 0,
    costs: the cost of each edge (doubles, exact for integer costs).  Edges with
    zero flow are dropped.
    """
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    flows = np.asarray(flows, np.float64).copy()
    costs = np.asarray(costs, np.float64)
    keep = flows > 0.0
    rows, cols, flows, costs = rows[keep], cols[keep], flows[keep], costs[keep]
    E = flows.shape[0]
    vidx = rows + cols * m
    order = np.lexsort((vidx, -flows))

    dsu = _DSU(m + n)
    adj = [dict() for _ in range(m + n)]
    nonforest = []
    for e in order.tolist():
        u, v = int(rows[e]), m + int(cols[e])
        if dsu.union(u, v):
            adj[u][v] = e
            adj[v][u] = e
        else:
            nonforest.append(e)

    alive = np.ones(E, dtype=bool)
    fl = flows.tolist()
    cs = costs.tolist()
    vi = vidx.tolist()
    for e in nonforest:
        u, v = int(rows[e]), m + int(cols[e])
        path = _forest_path(adj, v, u)
        minus = path[0::2]
        plus = path[1::2]
        dcost = math.fsum([cs[e]] + [cs[k] for k in plus] + [-cs[k] for k in minus])
        if dcost < 0:
            dec, inc = minus, [e] + plus
        else:
            dec, inc = [e] + plus, minus
        bott = min(dec, key=lambda k: (fl[k], vi[k]))
        t = fl[bott]
        for k in dec:
            fl[k] -= t
        for k in inc:
            fl[k] += t
        fl[bott] = 0.0
        alive[bott] = False
        if bott != e:
            bu, bv = int(rows[bott]), m + int(cols[bott])
            del adj[bu][bv]
            del adj[bv][bu]
            adj[u][v] = e
            adj[v][u] = e
    fl = np.asarray(fl)
    out = alive & (fl > 0.0)
    return rows[out], cols[out], fl[out]


def forest_flows(rows, cols, a, b):
    """Flows on an acyclic support determined by the marginals alone (a basic
    solution, Section 2.2): repeatedly take a leaf node -- a row or column with a
    single remaining edge -- send its remaining mass along that edge and remove
    it.  Leaves are taken in increasing node order (rows 0..m-1 then columns).
    Returns (flows, imbalance) where imbalance is the mass left at the last node
    of each tree (zero for an exactly balanced tree)."""
    m, n = len(a), len(b)
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    E = rows.shape[0]
    rem = np.concatenate([np.asarray(a, np.float64), np.asarray(b, np.float64)]).tolist()
    inc = [[] for _ in range(m + n)]
    for e in range(E):
        inc[int(rows[e])].append(e)
        inc[m + int(cols[e])].append(e)
    deg = [len(x) for x in inc]
    used = [False] * E
    flows = [0.0] * E
    import heapq
    heap = [v for v in range(m + n) if deg[v] == 1]
    heapq.heapify(heap)
    while heap:
        v = heapq.heappop(heap)
        if deg[v] != 1:
            continue
        e = next(k for k in inc[v] if not used[k])
        used[e] = True
        u = m + int(cols[e]) if v < m else int(rows[e])
        flows[e] = rem[v]
        rem[v] = 0.0
        rem[u] -= flows[e]
        deg[v] = 0
        deg[u] -= 1
        if deg[u] == 1:
            heapq.heappush(heap, u)
    imbalance = float(np.abs(np.asarray(rem)).sum())
    return np.asarray(flows), imbalance
