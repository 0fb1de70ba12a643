"""Pins of the graph-search oracle (HNSW, HNSW+, HNSW++) against what the paper
and the mathematics fix: hand-traced searches on a ten-vertex graph, the exact
KNN that a beam wider than the graph must return, the special cases that reduce
to plain HNSW, the local minimum a one-entry beam ends at, Algorithm 1 as the
IVF oracle states it, and the trends of Section 6.2.  CPU only.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
import synthdata as sd
from synthdata.graph import hnsw_graph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _f(v):
    return math.inf if v == "inf" else float(v)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


class _G:
    pass


def _tiny():
    lines = [json.loads(l) for l in open(os.path.join(GOLDEN, "hnsw_tiny.json"))]
    g0 = lines[1]
    n = len(g0["points"])
    g = _G()
    g.levels = np.array(g0["levels"], np.int32)
    g.adj0 = np.array(g0["adj0"], np.int32)
    g.up_off = np.full(n, -1, np.int64)
    rows = []
    for v, nb in g0["up"].items():
        g.up_off[int(v)] = len(rows)
        rows.append(nb)
    g.up_adj = np.array(rows, np.int32)
    g.entry, g.max_level, g.M, g.M0 = g0["entry"], g0["max_level"], g0["M"], g0["M0"]
    return np.array(g0["points"], float), np.array(g0["query"], float), g, lines[2:]


def _tiny_cases():
    return _tiny()[3]


@pytest.mark.parametrize("case", _tiny_cases(), ids=lambda c: c["name"])
def test_hnsw_golden_tiny(case):
    x, q, g, _ = _tiny()
    if "query" in case:
        q = np.array(case["query"], float)
    ids, dist, st = oracle.hnsw_search(x, q[None, :], g, case["K"], case["nef"], _f(case["eps0"]),
                                       case["delta_d"], case["variant"])
    assert ids[0].tolist() == case["ids"]
    assert np.allclose(dist[0] ** 2, case["sq_dist"], rtol=0, atol=1e-9)
    assert st[0, :3].tolist() == [case["dcos"], case["dims"], case["hops"]]


def test_hnsw_dco_is_algorithm_1():
    """The graph search's DCO agrees with the IVF oracle's Algorithm 1, and the
    observed distance of a rejected object is sqrt(D/d) times the norm of its
    first d sampled coordinates (Section 3.1)."""
    rng = np.random.default_rng(5)
    D = 64
    for t in range(400):
        o = rng.standard_normal(D)
        q = rng.standard_normal(D)
        true = float(np.linalg.norm(o - q))
        r = true * rng.uniform(0.6, 1.4) if t % 7 else math.inf
        eps0 = [0.0, 1.0, 2.1, math.inf][t % 4]
        dd = [1, 8, 16, 64][(t // 4) % 4]
        pos, dims, dis, obs, _ = oracle.hnsw_dco(o, q, r, eps0, dd)
        p2, d2, dims2 = oracle.ads_dco(o, q, r, eps0, dd)
        assert (pos, dims) == (bool(p2), dims2)
        if pos:
            assert dis == d2
        expect = math.sqrt(D / dims * float(np.sum((o[:dims] - q[:dims]) ** 2)))
        assert obs == pytest.approx(expect, rel=1e-12)
        if dims == D:
            assert dis == pytest.approx(true, rel=1e-12)
        else:
            assert math.isinf(dis)
        pf, _, dis_f, obs_f, _ = oracle.hnsw_dco(o, q, r, eps0, dd, method=oracle.METHOD_FDS)
        assert pf == (true <= r) and dis_f == pytest.approx(true, rel=1e-12) and obs_f == dis_f


def _connected_everywhere(g):
    n = g.n
    for s in range(n):
        seen = np.zeros(n, bool)
        seen[s] = True
        stack = [s]
        while stack:
            u = stack.pop()
            for v in g.adj0[u]:
                if v >= 0 and not seen[v]:
                    seen[v] = True
                    stack.append(v)
        if not seen.all():
            return False
    return True


@pytest.fixture(scope="module")
def small():
    x = sd.lowrank(300, 24, 41, 42, latent=8, noise=0.2).astype(np.float64)
    q = sd.lowrank(20, 24, 43, 42, latent=8, noise=0.2).astype(np.float64)
    g = hnsw_graph(x, M=6, seed=44)
    return x, q, g


def test_beam_wider_than_graph_is_exact_knn(small):
    """With N_ef >= n the result set never fills, every vertex reachable from
    the start is visited, and the answer is the exact KNN (Section 2.2.1's
    beam search degenerates into a traversal)."""
    x, q, g = small
    assert _connected_everywhere(g)
    K = 5
    gt_ids, gt_d = oracle.brute_knn(x, q, K)
    for variant, eps0 in [(oracle.HNSW_PLAIN, math.inf), (oracle.HNSW_PLUS, 2.1),
                          (oracle.HNSW_PP, math.inf)]:
        ids, dist, st = oracle.hnsw_search(x, q, g, K, g.n, eps0, 8, variant)
        assert np.array_equal(ids, gt_ids), variant
        assert np.allclose(dist, gt_d, rtol=1e-12)
        # every vertex DCO'd exactly once in layer 0, the entry once more per upper pass
        assert np.all(st[:, 0] >= g.n)
    # HNSW++ with a finite eps0 still visits everything (R2 never fills);
    # R1 holds the exact KNN except after a (rare) false rejection
    ids, dist, st = oracle.hnsw_search(x, q, g, K, g.n, 2.1, 8, oracle.HNSW_PP)
    ex = np.stack([oracle.exact_dist(x[ids[i]], q[i]) for i in range(len(q))])
    assert np.allclose(dist, ex, rtol=1e-12)
    assert oracle.recall(ids, ex, gt_d, K) >= 0.98


@pytest.fixture(scope="module")
def medium():
    x = sd.lowrank(4000, 256, 51, 52, latent=16, noise=0.1).astype(np.float64)
    q = sd.lowrank(60, 256, 53, 52, latent=16, noise=0.1).astype(np.float64)
    g = hnsw_graph(x, M=8, seed=54)
    return x, q, g


def test_infinite_eps0_reduces_to_plain_hnsw(medium):
    """eps0 = inf never rejects, so HNSW+ is HNSW, and HNSW++'s observed
    distances are the exact ones, so its R2 is HNSW's R and its R1 the K
    nearest of them: identical answers, DCOs, dims and expansions."""
    x, q, g = medium
    K, nef = 10, 40
    ref = oracle.hnsw_search(x, q, g, K, nef, math.inf, 16, oracle.HNSW_PLAIN)
    for variant in (oracle.HNSW_PLUS, oracle.HNSW_PP):
        out = oracle.hnsw_search(x, q, g, K, nef, math.inf, 16, variant)
        assert np.array_equal(out[0], ref[0])
        assert np.array_equal(out[1], ref[1])
        assert np.array_equal(out[2][:, :3], ref[2][:, :3])


def test_one_entry_beam_ends_at_local_minimum(medium):
    """N_ef = 1 makes the layer-0 beam a greedy walk (Section 2.2.1 notes the
    upper layers are this case): no layer-0 neighbour of the returned vertex is
    closer to the query."""
    x, q, g = medium
    ids, dist, _ = oracle.hnsw_search(x, q, g, 1, 1, math.inf, 16, oracle.HNSW_PLAIN)
    for i in range(len(q)):
        v = ids[i, 0]
        nb = g.adj0[v][g.adj0[v] >= 0]
        d_nb = oracle.exact_dist(x[nb], q[i])
        assert np.all((d_nb > dist[i, 0]) | ((d_nb == dist[i, 0]) & (nb > v)))


def test_trends_of_section_6(medium):
    """Section 6.2's findings on the graph family, here at eps0 = 2.1 and
    delta_d = 16 on synthetic D = 256 data: HNSW+ keeps HNSW's recall and
    samples fewer dimensions; HNSW++ samples fewer than HNSW+ at nearly the
    same recall; HNSW+'s sampled fraction grows with N_ef (its threshold is the
    N_ef-th distance) while HNSW++'s shrinks (its threshold is the K-th)."""
    x, q, g = medium
    K = 10
    _, gt_d = oracle.brute_knn(x, q, K)

    def run(variant, eps0, nef):
        ids, _, st = oracle.hnsw_search(x, q, g, K, nef, eps0, 16, variant)
        ex = np.stack([oracle.exact_dist(x[ids[i]], q[i]) for i in range(len(q))])
        return oracle.recall(ids, ex, gt_d, K), st[:, 1].sum() / (st[:, 0].sum() * x.shape[1])

    r0, f0 = run(oracle.HNSW_PLAIN, math.inf, 60)
    r1, f1 = run(oracle.HNSW_PLUS, 2.1, 60)
    r2, f2 = run(oracle.HNSW_PP, 2.1, 60)
    assert f0 == 1.0
    assert abs(r1 - r0) <= 0.01 and f1 < 0.8
    assert f2 < f1 and abs(r2 - r0) <= 0.02
    _, f1_wide = run(oracle.HNSW_PLUS, 2.1, 200)
    _, f2_wide = run(oracle.HNSW_PP, 2.1, 200)
    assert f1_wide > f1 and f2_wide < f2


def test_band_flags_are_rare_on_integer_data():
    """On integer coordinates every distance is an exact integer square root,
    so only Algorithm 1's irrational boundaries can sit near a decision: the
    band flag marks few queries, which keeps the exact GPU comparison on
    integer data meaningful."""
    x = sd.mixture(3000, 128, 61, 1000).astype(np.float64)
    q = sd.mixture(100, 128, 62, 1000).astype(np.float64)
    g = hnsw_graph(x, M=8, seed=63)
    for variant in (oracle.HNSW_PLAIN, oracle.HNSW_PLUS, oracle.HNSW_PP):
        _, _, st = oracle.hnsw_search(x, q, g, 10, 50, 2.1, 32, variant, rel=1e-6, rel_exact=0.0)
        assert st[:, 3].mean() <= 0.05, (variant, st[:, 3].mean())


@pytest.mark.parametrize("model,n,D,M,seed", [("mix", 2000, 128, 8, 73), ("mix", 40, 32, 2, 92),
                                              ("lowrank", 1500, 64, 16, 84)])
def test_graph_input_format(model, n, D, M, seed):
    """The seeded graph meets the format both searches read: ids in range,
    -1 padding only at the end of a row, no duplicates, at most M (2M on layer
    0) neighbours, upper neighbours present on their layer, the entry on the
    top layer, and (for M >= 4, where the free slots suffice) every vertex
    reachable from the first one on every layer."""
    x = sd.mixture(n, D, seed, 1000) if model == "mix" else sd.lowrank(n, D, seed, seed + 1, latent=8)
    g = hnsw_graph(x, M=M, seed=seed)
    assert g.adj0.shape == (n, 2 * M) and g.up_adj.shape[1] == M
    assert g.levels[g.entry] == g.max_level == g.levels.max()
    assert g.entry == int(np.flatnonzero(g.levels == g.max_level)[0])
    for v in range(n):
        rows = [(0, g.adj0[v])] + [(l, g.up_adj[g.up_off[v] + l - 1]) for l in range(1, g.levels[v] + 1)]
        for l, r in rows:
            ids = r[r >= 0]
            assert np.all(r[len(ids):] == -1), (v, l)
            assert len(set(ids.tolist())) == len(ids) and v not in ids
            assert ids.max(initial=-1) < n
            assert all(g.levels[u] >= l for u in ids)
    for l in range(g.max_level + 1 if M >= 4 else 0):
        nodes = np.flatnonzero(g.levels >= l)
        seen = {int(nodes[0])}
        stack = [int(nodes[0])]
        while stack:
            u = stack.pop()
            r = g.adj0[u] if l == 0 else g.up_adj[g.up_off[u] + l - 1]
            for v in r[r >= 0]:
                if int(v) not in seen:
                    seen.add(int(v))
                    stack.append(int(v))
        assert seen == set(nodes.tolist()), l
