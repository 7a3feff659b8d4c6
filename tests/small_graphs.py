"""Small seeded graphs for tests: CSR builders from edge lists, random small
graphs with optional self-loops and weights, cliques, rings of cliques,
stars.  Input construction only; no community-detection arithmetic."""
from __future__ import annotations

import numpy as np

from paper_1410_1237_amd.graphs import CSR


def from_edges(n, edges, weights=None, name="") -> CSR:
    """Symmetric CSR from undirected edges (u, v) (u == v allowed: a
    self-loop stored once).  Duplicate pairs are not allowed."""
    rows = [dict() for _ in range(n)]
    for idx, (u, v) in enumerate(edges):
        w = 1 if weights is None else int(weights[idx])
        assert v not in rows[u], "duplicate edge"
        rows[u][v] = w
        rows[v][u] = w
    off = np.zeros(n + 1, dtype=np.int64)
    cols, ws = [], []
    for i in range(n):
        for j in sorted(rows[i]):
            cols.append(j)
            ws.append(rows[i][j])
        off[i + 1] = len(cols)
    cols = np.array(cols, dtype=np.int32)
    w = None if weights is None else np.array(ws, dtype=np.int32)
    return CSR(n, off, cols, w, name=name)


def random_graph(rng, n, p=0.3, self_loops=0.0, wmax=1, name="") -> CSR:
    edges, ws = [], []
    for i in range(n):
        if self_loops and rng.random() < self_loops:
            edges.append((i, i))
            ws.append(int(rng.integers(1, wmax + 1)))
        for j in range(i + 1, n):
            if rng.random() < p:
                edges.append((i, j))
                ws.append(int(rng.integers(1, wmax + 1)))
    return from_edges(n, edges, ws if wmax > 1 else None, name=name or f"rand(n={n},p={p})")


def cliques(r, s, perm=None) -> CSR:
    """r disjoint cliques K_s; vertex x of clique q has id perm[q*s + x]."""
    n = r * s
    perm = np.arange(n) if perm is None else perm
    edges = []
    for q in range(r):
        for x in range(s):
            for y in range(x + 1, s):
                edges.append((int(perm[q * s + x]), int(perm[q * s + y])))
    return from_edges(n, edges, name=f"cliques(r={r},s={s})")


def ring_of_cliques(r, s) -> CSR:
    """r cliques K_s; clique q's last vertex joined to clique q+1's first."""
    n = r * s
    edges = []
    for q in range(r):
        for x in range(s):
            for y in range(x + 1, s):
                edges.append((q * s + x, q * s + y))
        nxt = ((q + 1) % r) * s
        if r > 1 and not (r == 2 and q == 1):
            edges.append((q * s + s - 1, nxt))
    return from_edges(n, edges, name=f"ring(r={r},s={s})")


def star(leaves) -> CSR:
    return from_edges(leaves + 1, [(0, i) for i in range(1, leaves + 1)], name=f"star({leaves})")
