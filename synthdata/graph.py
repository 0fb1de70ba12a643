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
    glob2loc = np.full(int(nodes.max()) + 1, -1, dtype=np.int64)
    glob2loc[nodes] = np.arange(len(nodes))
    cand_loc = glob2loc[cand]
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
    _join(nodes, adj, cand_loc, _nearest_free_np(x[nodes].astype(np.float64)))
    out = {}
    for i in range(len(nodes)):
        row = adj[i][adj[i] >= 0]                 # ids first, -1 padding at the end
        full = np.full(m, -1, dtype=np.int64)
        full[:len(row)] = row
        out[int(nodes[i])] = full
    return out


def _join(nodes: np.ndarray, adj: np.ndarray, cand_loc: np.ndarray, nearest_free, say=None) -> int:
    """Links every vertex into the part reachable from the layer's first one:
    while a vertex is unreached, the lowest unreached one u is joined both ways
    to a reached vertex w with a free last slot -- the first such vertex among
    u's own k-NN candidates (ascending distance), else the nearest such vertex
    of the layer (``nearest_free(u, free)``, ties to the lower index).  u's link
    back to w goes into u's last slot when that is free and w is not already a
    neighbour.  Stops early when no reached vertex has a free slot (tiny M).
    Returns the number of joins."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import breadth_first_order
    m = adj.shape[1]
    n = len(nodes)
    glob2loc = np.full(int(nodes.max()) + 1, -1, dtype=np.int64)
    glob2loc[nodes] = np.arange(n)
    loc = np.where(adj >= 0, glob2loc[np.maximum(adj, 0)], -1)
    r, c = np.nonzero(loc >= 0)
    g = csr_matrix((np.ones(len(r), dtype=np.int8), (r, loc[r, c])), shape=(n, n))
    reached = np.zeros(n, dtype=bool)
    reached[breadth_first_order(g, 0, directed=True, return_predecessors=False)] = True
    joins = 0
    pending = np.flatnonzero(~reached)
    if say:
        say(f"  {len(pending)} vertices unreached before joining")
    for u in pending:
        u = int(u)
        if reached[u]:
            continue
        w = -1
        for cnd in cand_loc[u]:
            if cnd >= 0 and reached[cnd] and adj[cnd, m - 1] < 0:
                w = int(cnd)
                break
        if w < 0:
            free = np.flatnonzero(reached & (adj[:, m - 1] < 0))
            if len(free) == 0:
                break
            w = int(nearest_free(u, free))
            if say:
                say(f"  join of {u}: nearest free vertex by a full scan")
        adj[w, m - 1] = nodes[u]
        if adj[u, m - 1] < 0 and nodes[w] not in adj[u]:
            adj[u, m - 1] = nodes[w]
        # the new edges start or end at reached vertices: flooding from u in
        # the layer's original rows reaches exactly what u now adds
        reached[u] = True
        stack = [u]
        while stack:
            i = stack.pop()
            for j in g.indices[g.indptr[i]:g.indptr[i + 1]]:
                if not reached[j]:
                    reached[j] = True
                    stack.append(int(j))
        joins += 1
        if say and joins % 5000 == 0:
            say(f"  {joins} joins, {int((~reached).sum())} vertices unreached")
    return joins


def _nearest_free_np(xs: np.ndarray):
    def pick(u, free):
        d = np.sum((xs[free] - xs[u]) ** 2, axis=1)
        return free[np.lexsort((free, d))[0]]
    return pick


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


# ---------------------------------------------------------------------------
# The same construction on the GPU with torch (for million-vertex inputs)
# ---------------------------------------------------------------------------

def _t_knn(xt, nodes_t, C, say=None):
    """Exact k-NN candidates within nodes_t: GEMM-form screen in float32, the
    best C + 16 recomputed in difference form in float64, sorted by (d2, id)."""
    import torch
    xs = xt[nodes_t]
    m = xs.shape[0]
    C = min(C, m - 1)
    pre = min(m - 1, C + 16)
    nrm = (xs.double() ** 2).sum(1).float()
    ids = torch.empty((m, C), dtype=torch.int64, device=xt.device)
    d2 = torch.empty((m, C), dtype=torch.float64, device=xt.device)
    step = max(1, min(8192, (1 << 33) // (4 * m)))
    nchunks = (m + step - 1) // step
    for ci, s in enumerate(range(0, m, step)):
        if say and nchunks > 20 and ci % max(1, nchunks // 10) == 0:
            say(f"  k-NN chunk {ci}/{nchunks}")
        e = min(m, s + step)
        g = nrm[s:e, None] + nrm[None, :] - 2.0 * (xs[s:e] @ xs.T)
        g[torch.arange(e - s, device=xt.device), torch.arange(s, e, device=xt.device)] = float("inf")
        part = torch.topk(g, pre, dim=1, largest=False).indices
        del g
        cand = nodes_t[part]
        ex = ((xt[cand].double() - xt[nodes_t[s:e]].double()[:, None, :]) ** 2).sum(2)
        # (d2, id) order: sort by id, then stably by distance
        o = torch.argsort(cand, dim=1)
        cand, ex = torch.gather(cand, 1, o), torch.gather(ex, 1, o)
        o = torch.argsort(ex, dim=1, stable=True)
        ids[s:e] = torch.gather(cand, 1, o)[:, :C]
        d2[s:e] = torch.gather(ex, 1, o)[:, :C]
    return ids, d2


def _t_heuristic(xt, cand, cd2, valid, m, say=None):
    """HNSW's selection (see _heuristic) for every row at once, on the GPU."""
    import torch
    rows, C = cand.shape
    out = torch.full((rows, m), -1, dtype=torch.int64, device=xt.device)
    D = xt.shape[1]
    step = max(1, min(16384, (1 << 30) // (C * D * 8)))
    nchunks = (rows + step - 1) // step
    for ci, s in enumerate(range(0, rows, step)):
        if say and nchunks > 20 and ci % max(1, nchunks // 10) == 0:
            say(f"  selection chunk {ci}/{nchunks}")
        e = min(rows, s + step)
        c = cand[s:e]
        v = valid[s:e]
        xc = xt[torch.where(v, c, torch.zeros_like(c))].double()
        g = torch.bmm(xc, xc.transpose(1, 2).contiguous())
        nr = torch.diagonal(g, dim1=1, dim2=2)
        pd = nr[:, :, None] + nr[:, None, :] - 2.0 * g
        kept = torch.zeros((e - s, C), dtype=torch.bool, device=xt.device)
        nkept = torch.zeros(e - s, dtype=torch.int64, device=xt.device)
        dq = cd2[s:e]
        for t in range(C):
            closer = (pd[:, t, :] < dq[:, t][:, None]) & kept
            good = v[:, t] & ~closer.any(dim=1) & (nkept < m)
            kept[:, t] = good
            nkept += good
        # kept candidates in their order, packed to the front
        rank = torch.cumsum(kept, dim=1) - 1
        r, t = torch.nonzero(kept, as_tuple=True)
        blk = torch.full((e - s, m), -1, dtype=torch.int64, device=xt.device)
        blk[r, rank[r, t]] = c[r, t]
        out[s:e] = blk
    return out


def _t_layer(xt, nodes, m, progress=None):
    import time
    import torch
    say = progress or (lambda msg: None)
    t0 = time.time()
    dev = xt.device
    nodes_t = torch.as_tensor(nodes, dtype=torch.int64, device=dev)
    if len(nodes) == 1:
        return np.full((1, m), -1, dtype=np.int64)
    C = 2 * m
    cand, cd2 = _t_knn(xt, nodes_t, C, say)
    if xt.is_cuda:
        torch.cuda.synchronize()
    say(f"  {len(nodes)} vertices: k-NN candidates in {time.time() - t0:.1f}s")
    fwd = _t_heuristic(xt, cand, cd2, torch.ones_like(cand, dtype=torch.bool), m, say)
    if xt.is_cuda:
        torch.cuda.synchronize()
    say(f"  {len(nodes)} vertices: selection in {time.time() - t0:.1f}s")
    # union of forward and reverse edges per vertex, closest 2m first
    pos = torch.full((xt.shape[0],), -1, dtype=torch.int64, device=dev)
    pos[nodes_t] = torch.arange(len(nodes), device=dev)
    src = torch.arange(len(nodes), device=dev)[:, None].expand_as(fwd)
    ok = fwd >= 0
    a = torch.cat([src[ok], pos[fwd[ok]]])                   # row (local index)
    b = torch.cat([nodes_t[pos[fwd[ok]]], nodes_t[src[ok]]])  # neighbour (global id)
    key = a * xt.shape[0] + b
    key = torch.unique(key)
    a, b = key // xt.shape[0], key % xt.shape[0]
    d = torch.empty(len(a), dtype=torch.float64, device=dev)
    for s in range(0, len(a), 1 << 18):
        e = min(len(a), s + (1 << 18))
        d[s:e] = ((xt[b[s:e]].double() - xt[nodes_t[a[s:e]]].double()) ** 2).sum(1)
    o = torch.argsort(b)
    a, b, d = a[o], b[o], d[o]
    o = torch.argsort(d, stable=True)
    a, b, d = a[o], b[o], d[o]
    o = torch.argsort(a, stable=True)
    a, b, d = a[o], b[o], d[o]
    cnt = torch.bincount(a, minlength=len(nodes))
    start = torch.cumsum(cnt, 0) - cnt
    rank = torch.arange(len(a), device=dev) - start[a]
    keep = rank < C
    ucand = torch.full((len(nodes), C), -1, dtype=torch.int64, device=dev)
    ud2 = torch.full((len(nodes), C), float("inf"), dtype=torch.float64, device=dev)
    ucand[a[keep], rank[keep]] = b[keep]
    ud2[a[keep], rank[keep]] = d[keep]
    final = _t_heuristic(xt, ucand, ud2, ucand >= 0, m - 1, say)
    adj = np.full((len(nodes), m), -1, dtype=np.int64)
    adj[:, :m - 1] = final.cpu().numpy()
    say(f"  {len(nodes)} vertices: reverse edges and second selection in {time.time() - t0:.1f}s")
    pos_t = torch.full((xt.shape[0],), -1, dtype=torch.int64, device=dev)
    pos_t[nodes_t] = torch.arange(len(nodes), device=dev)
    cand_loc = pos_t[cand].cpu().numpy()
    joins = _join(nodes, adj, cand_loc, _nearest_free_t(xt, nodes_t), say)
    say(f"  {len(nodes)} vertices: {joins} joins, done in {time.time() - t0:.1f}s")
    out = np.full((len(nodes), m), -1, dtype=np.int64)
    for_rows = adj >= 0
    cnts = for_rows.sum(1)
    order = np.argsort(~for_rows, axis=1, kind="stable")
    packed = np.take_along_axis(adj, order, axis=1)
    out[:] = packed
    out[np.arange(m)[None, :] >= cnts[:, None]] = -1
    return out


def _nearest_free_t(xt, nodes_t):
    def pick(u, free):
        import torch
        ft = torch.as_tensor(free, device=xt.device)
        d = ((xt[nodes_t[ft]].double() - xt[nodes_t[u]].double()) ** 2).sum(1).cpu().numpy()
        return free[np.lexsort((free, d))[0]]
    return pick


def hnsw_graph_torch(x: np.ndarray, M: int = 16, seed: int = 0, level_cap: int = 16,
                     device: str = "cuda", progress=None) -> HnswGraph:
    """hnsw_graph's construction run with torch on the GPU (input generation
    for million-vertex workloads; same levels, candidates, heuristic, reverse
    edges and joins, with a float32 GEMM screen before the float64 recompute)."""
    import torch
    n = x.shape[0]
    M0 = 2 * M
    levels = hnsw_levels(n, M, seed, level_cap)
    max_level = int(levels.max())
    entry = int(np.flatnonzero(levels == max_level)[0])
    xt = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device=device)
    adj0 = _t_layer(xt, np.arange(n, dtype=np.int64), M0, progress).astype(np.int32)
    up_off = np.full(n, -1, dtype=np.int64)
    upper = np.flatnonzero(levels >= 1)
    rows = 0
    for v in upper:
        up_off[v] = rows
        rows += int(levels[v])
    up_adj = np.full((max(rows, 1), M), -1, dtype=np.int32)
    for l in range(1, max_level + 1):
        nodes = np.flatnonzero(levels >= l).astype(np.int64)
        lay = _t_layer(xt, nodes, M, progress)
        up_adj[up_off[nodes] + l - 1] = lay
    del xt
    torch.cuda.empty_cache()
    return HnswGraph(levels, adj0, up_off, up_adj, entry, max_level, M, M0)
