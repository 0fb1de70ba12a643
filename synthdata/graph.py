"""Seeded HNSW-structured graphs, an input shared by the oracle and the GPU library.

In the paper the graph index comes from an external library (hnswlib, with
M = 16 and efConstruction = 500, Section 6.1); the method changes only how the
search runs its DCOs.  So here, as with the IVF clustering, the graph is an
input that both sides receive bit for bit.  It has HNSW's structure
(Section 2.2.1): every vector is on layer 0, a vector's top layer is drawn from
the exponential law of the HNSW construction (floor(-ln(U) / ln M)), each layer
keeps at most M neighbours per vertex (2M on layer 0), and the neighbours are
chosen with HNSW's diversity heuristic (keep a candidate only if it is closer
to the vertex than to every neighbour kept so far).  It is built in one batch
instead of by incremental insertion: the candidates of a vertex are its exact
nearest neighbours within the layer, pruned with the heuristic, then united
with the reverse edges and pruned again.

Format (the one both searches read):

* ``levels[n]`` int32 -- top layer of each vertex;
* ``adj0[n][M0]`` int32 -- layer-0 neighbours in stored order, -1 padded;
* ``up_off[n]`` int64 -- for a vertex with level >= 1, the row of its layer-1
  neighbours in ``up_adj`` (its layer-l row is ``up_off + l - 1``); -1 else;
* ``up_adj[rows][M]`` int32 -- upper-layer neighbours, -1 padded;
* ``entry`` -- the lowest id among the vertices of the top layer.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class HnswGraph:
    levels: np.ndarray
    adj0: np.ndarray
    up_off: np.ndarray
    up_adj: np.ndarray
    entry: int
    max_level: int
    M: int
    M0: int

    @property
    def n(self) -> int:
        return int(self.levels.shape[0])


def hnsw_levels(n: int, M: int, seed: int, cap: int = 16) -> np.ndarray:
    """Top layer of each vertex: floor(-ln(1 - U) / ln M), U ~ U[0, 1), capped."""
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    lv = np.floor(-np.log1p(-u) / np.log(M))
    return np.minimum(lv, cap).astype(np.int32)


def _sq_dist_rows(x: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Squared distances between rows a[i] and b[i, j] (difference form, float64)."""
    return np.sum((x[b].astype(np.float64) - x[a].astype(np.float64)[:, None, :]) ** 2, axis=2)


def _knn_candidates(x: np.ndarray, nodes: np.ndarray, C: int) -> tuple[np.ndarray, np.ndarray]:
    """The C nearest other members of ``nodes`` for every member, ascending by
    (squared distance, id); returns global ids and squared distances."""
    xs = x[nodes].astype(np.float64)
    nrm = np.sum(xs * xs, axis=1)
    m = len(nodes)
    C = min(C, m - 1)
    pre = min(m - 1, C + 16)
    ids = np.empty((m, C), dtype=np.int64)
    d2 = np.empty((m, C), dtype=np.float64)
    step = max(1, min(1024, (1 << 25) // max(1, m)))
    sub = max(1, (1 << 26) // (pre * x.shape[1] * 8))
    for s in range(0, m, step):
        e = min(m, s + step)
        g = nrm[s:e, None] + nrm[None, :] - 2.0 * (xs[s:e] @ xs.T)
        g[np.arange(e - s), np.arange(s, e)] = np.inf
        part = np.argpartition(g, pre - 1, axis=1)[:, :pre]
        for a in range(s, e, sub):
            b = min(e, a + sub)
            cand = nodes[part[a - s:b - s]]
            exact = _sq_dist_rows(x, nodes[a:b], cand)
            order = np.lexsort((cand, exact), axis=1)
            ids[a:b] = np.take_along_axis(cand, order, axis=1)[:, :C]
            d2[a:b] = np.take_along_axis(exact, order, axis=1)[:, :C]
    return ids, d2


def _heuristic(x: np.ndarray, nodes: np.ndarray, cand: np.ndarray, cd2: np.ndarray,
               valid: np.ndarray, m: int) -> np.ndarray:
    """HNSW's neighbour selection for every row at once: walk the candidates in
    ascending order and keep one when it is not closer to an already kept
    neighbour than to the vertex; at most m kept.  Returns [rows, m], -1 padded."""
    rows, C = cand.shape
    out = np.full((rows, m), -1, dtype=np.int64)
    step = max(1, min((1 << 24) // (C * C), (1 << 27) // (C * x.shape[1] * 8)))
    for s in range(0, rows, step):
        e = min(rows, s + step)
        c = cand[s:e]
        v = valid[s:e]
        xc = x[np.where(v, c, 0)].astype(np.float64)
        g = np.einsum("rid,rjd->rij", xc, xc)
        nr = np.einsum("rid,rid->ri", xc, xc)
        pd = nr[:, :, None] + nr[:, None, :] - 2.0 * g
        kept = np.zeros((e - s, C), dtype=bool)
        nkept = np.zeros(e - s, dtype=np.int64)
        dq = cd2[s:e]
        for t in range(C):
            closer = (pd[:, t, :] < dq[:, t][:, None]) & kept
            good = v[:, t] & ~closer.any(axis=1) & (nkept < m)
            kept[:, t] = good
            nkept += good
        for r in range(e - s):
            k = c[r][kept[r]]
            out[s + r, :len(k)] = k
    return out


def _layer(x: np.ndarray, nodes: np.ndarray, m: int) -> dict:
    """Adjacency (global ids, -1 padded, m per vertex) of one layer's vertices."""
    if len(nodes) == 1:
        return {int(nodes[0]): np.full(m, -1, dtype=np.int64)}
    C = 2 * m
    cand, cd2 = _knn_candidates(x, nodes, C)
    fwd = _heuristic(x, nodes, cand, cd2, np.ones_like(cand, dtype=bool), m)
    # reverse edges, then the union pruned again (closest 2m of the union first)
    pos = {int(v): i for i, v in enumerate(nodes)}
    rev = [[] for _ in range(len(nodes))]
    for i, row in enumerate(fwd):
        for v in row:
            if v >= 0:
                rev[pos[int(v)]].append(int(nodes[i]))
    width = C
    ucand = np.full((len(nodes), width), -1, dtype=np.int64)
    ud2 = np.full((len(nodes), width), np.inf)
    for i in range(len(nodes)):
        u = sorted(set(int(v) for v in fwd[i] if v >= 0) | set(rev[i]))
        if not u:
            continue
        ua = np.asarray(u, dtype=np.int64)
        d = np.sum((x[ua].astype(np.float64) - x[nodes[i]].astype(np.float64)) ** 2, axis=1)
        o = np.lexsort((ua, d))[:width]
        ucand[i, :len(o)] = ua[o]
        ud2[i, :len(o)] = d[o]
    # the last slot of every vertex is kept free for the links that join the
    # layer's components (clustered data leaves a pruned k-NN graph split)
    final = _heuristic(x, nodes, ucand, ud2, ucand >= 0, m - 1)
    adj = np.full((len(nodes), m), -1, dtype=np.int64)
    adj[:, :m - 1] = final
    _join_components(x, nodes, adj, pos)
    out = {}
    for i in range(len(nodes)):
        row = adj[i][adj[i] >= 0]                 # ids first, -1 padding at the end
        full = np.full(m, -1, dtype=np.int64)
        full[:len(row)] = row
        out[int(nodes[i])] = full
    return out


def _join_components(x: np.ndarray, nodes: np.ndarray, adj: np.ndarray, pos: dict) -> None:
    """Links every vertex into the part reachable from the first one: while a
    vertex is unreached, the lowest unreached one u is joined both ways to the
    nearest reached vertex w that has a free slot (u's own last slot is free).
    Stops early when no reached vertex has a free slot left (possible only for
    tiny M)."""
    m = adj.shape[1]
    reached = np.zeros(len(nodes), dtype=bool)
    xs = x[nodes].astype(np.float64)

    def flood(start: int) -> None:
        stack = [start]
        reached[start] = True
        while stack:
            i = stack.pop()
            for v in adj[i]:
                if v < 0:
                    continue
                j = pos[int(v)]
                if not reached[j]:
                    reached[j] = True
                    stack.append(j)

    flood(0)
    while not reached.all():
        u = int(np.flatnonzero(~reached)[0])
        free = reached & (adj[:, m - 1] < 0)
        cand = np.flatnonzero(free)
        if len(cand) == 0:
            break
        d = np.sum((xs[cand] - xs[u]) ** 2, axis=1)
        w = int(cand[np.lexsort((cand, d))[0]])
        adj[w, m - 1] = nodes[u]
        if adj[u, m - 1] < 0 and nodes[w] not in adj[u]:
            adj[u, m - 1] = nodes[w]
        flood(u)


def hnsw_graph(x: np.ndarray, M: int = 16, seed: int = 0, level_cap: int = 16) -> HnswGraph:
    """HNSW-structured graph over the rows of x (see the module docstring)."""
    n = x.shape[0]
    M0 = 2 * M
    levels = hnsw_levels(n, M, seed, level_cap)
    max_level = int(levels.max())
    entry = int(np.flatnonzero(levels == max_level)[0])
    l0 = _layer(x, np.arange(n, dtype=np.int64), M0)
    adj0 = np.full((n, M0), -1, dtype=np.int32)
    for v, row in l0.items():
        adj0[v] = row
    up_off = np.full(n, -1, dtype=np.int64)
    upper = np.flatnonzero(levels >= 1)
    rows = 0
    for v in upper:
        up_off[v] = rows
        rows += int(levels[v])
    up_adj = np.full((max(rows, 1), M), -1, dtype=np.int32)
    for l in range(1, max_level + 1):
        nodes = np.flatnonzero(levels >= l).astype(np.int64)
        for v, row in _layer(x, nodes, M).items():
            up_adj[up_off[v] + l - 1] = row
    return HnswGraph(levels, adj0, up_off, up_adj, entry, max_level, M, M0)
