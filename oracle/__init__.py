"""FP64 CPU oracle for ADSampling inside an IVF scan.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_2303_09855_amd``): neither imports the other, and
the only common inputs come from the seeded generators in ``synthdata``.

What it computes, each function citing the passage it follows:

* :func:`make_rotation` -- Section 3.1: a random orthogonal matrix obtained by
  orthonormalising a Gaussian matrix (QR, sign-fixed so the result is Haar);
* :func:`rotate` -- y = P x (Section 3.1, the transformation of data and query
  vectors);
* :func:`brute_knn` -- the exact KNN query of Section 2.1 (ground truth);
* :func:`probes` -- IVF probe selection, the N_probe nearest centroids
  (Section 2.2.2);
* :func:`dco_batch` -- Definition 2.1 by FDScanning, Algorithm 1
  (ADSampling) or PDScanning (Section 6.1) for a fixed threshold;
* :func:`ip_dco_batch` / :func:`normalize` -- Section 8's reduction (extension (1)) of cosine
  search and inner-product comparisons to DCOs on unit vectors;
* :func:`kmeans` -- the k-means clustering of the IVF index phase (Section 2.2.2,
  Section 6.1), seeded by :func:`kmeans_init_rows` (SplitMix64 counters);
* :func:`ivf_search` -- the IVF scan with a KNN max-heap (Section 2.2.2), with
  ADSampling as its DCO (IVF+, Section 4).  IVF++ (Section 5.2) changes only the
  memory layout and gives the same result, so one oracle covers both;
* :func:`recall`, :func:`distance_ratio`, :func:`dims_ratio` -- the metrics of
  Section 6.1 (Performance Metrics).

All arithmetic is in float64.  The scan and DCO loops are plain sequential C
(``ads_oracle.c``), threaded over queries only.

Pins (tests/test_oracle_pins.py): orthogonality and Haar sign symmetry of P,
norm preservation, the row-sampling identity (Eq. 2), the exact-distance case
d = D, no false positives (Lemma 3.2), eps0 = inf equal to FDScanning and to a
full sort, monotonicity in eps0, the exact Beta law of the single-test failure
probability, and hand-derived golden cases.  Absolute QPS and dims fractions
are parity unpinned (the paper prints them only in figures).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "libads_oracle.so")
_SRC = os.path.join(_HERE, "ads_oracle.c")
_SRC_HNSW = os.path.join(_HERE, "hnsw_oracle.c")
SOURCES = (_SRC, _SRC_HNSW)

METHOD_ADS, METHOD_FDS, METHOD_PDS = 0, 1, 2

# ---------------------------------------------------------------------------
# build / load
# ---------------------------------------------------------------------------


def build() -> str:
    """Compile the C part with gcc (always recompiles)."""
    os.makedirs(_BUILD, exist_ok=True)
    tmp = f"{_SO}.{os.getpid()}.tmp"     # concurrent builds never share a file
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", tmp, *SOURCES,
           "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    _lib = bind(ctypes.CDLL(_SO))
    return _lib


def bind(lib):
    """Declares the C functions' signatures on a loaded library and returns it."""
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_ads_dco.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, ip, dp]
    lib.orc_ads_dco.restype = ctypes.c_int
    lib.orc_fds_dco.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, dp]
    lib.orc_fds_dco.restype = ctypes.c_int
    lib.orc_pds_dco.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ip, dp]
    lib.orc_pds_dco.restype = ctypes.c_int
    lib.orc_dco_batch.argtypes = [dp, ctypes.c_int, dp, i64p, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_int, u8p, dp, i32p,
                                  u8p, ctypes.c_double]
    lib.orc_dco_batch.restype = None
    lib.orc_ivf_search.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, i64p, i64p, i64p, i32p,
                                   i32p, ctypes.c_int, i32p, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_int, i64p, dp, i64p, ctypes.c_int]
    lib.orc_ivf_search.restype = ctypes.c_int
    lib.orc_hnsw_search.argtypes = [dp, ctypes.c_int64, ctypes.c_int, dp, ctypes.c_int, i32p, i32p,
                                    ctypes.c_int, i64p, i32p, ctypes.c_int, ctypes.c_int32,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    i64p, dp, i64p, ctypes.c_int]
    lib.orc_hnsw_search.restype = ctypes.c_int
    lib.orc_hnsw_dco.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_double, ip, dp, dp, ip]
    lib.orc_hnsw_dco.restype = ctypes.c_int
    return lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ---------------------------------------------------------------------------
# Section 3.1: random orthogonal transformation
# ---------------------------------------------------------------------------


def make_rotation(gaussian: np.ndarray) -> np.ndarray:
    """Orthonormalise a Gaussian matrix (Section 3.1, footnote on random projection).

    Householder QR (LAPACK via numpy), then Q <- Q diag(sign(diag R)) so that
    Q is Haar distributed.  Returns P64 with y = P64 @ x.
    """
    g = np.asarray(gaussian, dtype=np.float64)
    qm, rm = np.linalg.qr(g)
    s = np.sign(np.diag(rm))
    s[s == 0] = 1.0
    return qm * s[None, :]


def rotate(x: np.ndarray, P64: np.ndarray) -> np.ndarray:
    """y = P x for every row x (float64)."""
    return np.asarray(x, dtype=np.float64) @ P64.T


# ---------------------------------------------------------------------------
# Section 2.1: exact KNN (ground truth)
# ---------------------------------------------------------------------------


def exact_dist(x: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Distances ||x_i - q|| in float64, difference form."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(q, dtype=np.float64)[None, :]
    return np.sqrt(np.einsum("ij,ij->i", d, d))


def brute_knn(x: np.ndarray, queries: np.ndarray, K: int, screen: int = 64,
              chunk: int = 65536, qchunk: int = 512) -> tuple[np.ndarray, np.ndarray]:
    """Exact top-K by (distance, id) for every query, float64.

    A float64 GEMM-form screen keeps the best K + screen candidates per query;
    their distances are then recomputed in difference form and sorted by
    (distance, id).  The distances returned are exact; when more than
    ``screen`` objects tie with the K-th, the ids among those ties are a valid
    choice but not necessarily the lowest ones (recall is tie-aware).
    """
    x = np.asarray(x, dtype=np.float32)
    qall = np.asarray(queries, dtype=np.float64)
    n = x.shape[0]
    nq = qall.shape[0]
    keep = min(n, K + screen)
    ids = np.empty((nq, K), dtype=np.int64)
    dist = np.empty((nq, K))
    for qs0 in range(0, nq, qchunk):
        qs = qall[qs0:qs0 + qchunk]
        m = qs.shape[0]
        best_s = np.full((m, keep), np.inf)
        best_i = np.zeros((m, keep), dtype=np.int64)
        qn = np.einsum("ij,ij->i", qs, qs)
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            xb = x[s:e].astype(np.float64)
            xn = np.einsum("ij,ij->i", xb, xb)
            sc = xn[None, :] - 2.0 * (qs @ xb.T) + qn[:, None]
            if sc.shape[1] > keep:
                part = np.argpartition(sc, keep - 1, axis=1)[:, :keep]
                sc_i = part + s
                sc = np.take_along_axis(sc, part, 1)
            else:
                sc_i = np.broadcast_to(np.arange(s, e), sc.shape)
            allv = np.concatenate([best_s, sc], axis=1)
            alli = np.concatenate([best_i, sc_i], axis=1)
            part = np.argpartition(allv, keep - 1, axis=1)[:, :keep]
            best_s = np.take_along_axis(allv, part, 1)
            best_i = np.take_along_axis(alli, part, 1)
        for j in range(m):
            i = qs0 + j
            cand = best_i[j]
            dv = exact_dist(x[cand], qs[j])
            order = np.lexsort((cand, dv))
            kk = min(K, len(order))
            ids[i, :kk] = cand[order[:kk]]
            dist[i, :kk] = dv[order[:kk]]
            ids[i, kk:] = -1
            dist[i, kk:] = np.inf
    return ids, dist


# ---------------------------------------------------------------------------
# Section 2.2.2: IVF probe selection
# ---------------------------------------------------------------------------


def probes(q_rot: np.ndarray, c_rot: np.ndarray, nprobe: int) -> tuple[np.ndarray, np.ndarray]:
    """The nprobe nearest centroids per query, ascending by (distance, list id).

    Returns (list ids [nq, nprobe] int32, squared distances [nq, nlist] float64).
    """
    q = np.asarray(q_rot, dtype=np.float64)
    c = np.asarray(c_rot, dtype=np.float64)
    d2 = np.empty((q.shape[0], c.shape[0]))
    for i in range(q.shape[0]):
        diff = c - q[i][None, :]
        d2[i] = np.einsum("ij,ij->i", diff, diff)
    ids = np.empty((q.shape[0], nprobe), dtype=np.int32)
    ar = np.arange(c.shape[0])
    for i in range(q.shape[0]):
        ids[i] = np.lexsort((ar, d2[i]))[:nprobe]
    return ids, d2


# ---------------------------------------------------------------------------
# Definition 2.1 / Algorithm 1: DCOs with a fixed threshold
# ---------------------------------------------------------------------------


def ads_dco(o: np.ndarray, q: np.ndarray, r: float, eps0: float, delta_d: int):
    """One ADSampling DCO (Algorithm 1). Returns (positive, dist, dims)."""
    lib = _load()
    o = np.ascontiguousarray(o, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    dims = ctypes.c_int(0)
    dist = ctypes.c_double(0.0)
    pos = lib.orc_ads_dco(_p(o, ctypes.c_double), _p(q, ctypes.c_double), o.shape[0],
                          float(r), float(eps0), int(delta_d), ctypes.byref(dims),
                          ctypes.byref(dist))
    return int(pos), dist.value, dims.value


def fds_dco(o: np.ndarray, q: np.ndarray, r: float):
    """One FDScanning DCO (Section 2.1). Returns (positive, dist)."""
    lib = _load()
    o = np.ascontiguousarray(o, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    dist = ctypes.c_double(0.0)
    pos = lib.orc_fds_dco(_p(o, ctypes.c_double), _p(q, ctypes.c_double), o.shape[0],
                          float(r), ctypes.byref(dist))
    return int(pos), dist.value


def dco_batch(base_rot: np.ndarray, q_rot: np.ndarray, rows: np.ndarray, r: float,
              eps0: float, delta_d: int, method: int = METHOD_ADS, band_rel: float = 1e-5):
    """DCOs of query q against base rows ``rows`` with a fixed threshold r.

    Returns dict(mask uint8, dist float64 (+inf for negatives), dims int32,
    band uint8: 1 where the decision lies within band_rel of a test boundary).
    """
    lib = _load()
    base = np.ascontiguousarray(base_rot, dtype=np.float64)
    q = np.ascontiguousarray(q_rot, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    m = rows.shape[0]
    mask = np.zeros(m, dtype=np.uint8)
    dist = np.zeros(m)
    dims = np.zeros(m, dtype=np.int32)
    band = np.zeros(m, dtype=np.uint8)
    lib.orc_dco_batch(_p(base, ctypes.c_double), base.shape[1], _p(q, ctypes.c_double),
                      _p(rows, ctypes.c_int64), m, float(r), float(eps0), int(delta_d),
                      int(method), _p(mask, ctypes.c_uint8), _p(dist, ctypes.c_double),
                      _p(dims, ctypes.c_int32), _p(band, ctypes.c_uint8), float(band_rel))
    return {"mask": mask, "dist": dist, "dims": dims, "band": band}


# ---------------------------------------------------------------------------
# Section 8, extension (1): cosine similarity and inner product
# ---------------------------------------------------------------------------


def normalize(x: np.ndarray) -> np.ndarray:
    """Rows scaled to unit length (a zero row stays zero), float64."""
    x = np.asarray(x, dtype=np.float64)
    n = np.linalg.norm(x, axis=1, keepdims=True)
    return np.divide(x, n, out=np.zeros_like(x), where=n > 0)


def ip_dco_batch(base_raw: np.ndarray, q_raw: np.ndarray, rows: np.ndarray, r: float,
                 P64: np.ndarray, eps0: float, delta_d: int, method: int = METHOD_ADS,
                 band_rel: float = 1e-5):
    """<o, q> >= r decided as a DCO on unit vectors (Section 8, extension (1)): the
    comparison holds iff || o/|o| - q/|q| || <= sqrt(2 - 2 r / (|o| |q|)).

    Returns dict(mask, ip (<o,q> for positives, -inf otherwise), dims, band)."""
    base = np.asarray(base_raw, dtype=np.float64)[np.asarray(rows, dtype=np.int64)]
    q = np.asarray(q_raw, dtype=np.float64)
    no = np.linalg.norm(base, axis=1)
    nq = float(np.linalg.norm(q))
    bu = rotate(normalize(base), P64)
    qu = rotate(normalize(q[None, :]), P64)[0]
    m = len(rows)
    mask = np.zeros(m, dtype=np.uint8)
    ip = np.full(m, -np.inf)
    dims = np.zeros(m, dtype=np.int32)
    band = np.zeros(m, dtype=np.uint8)
    for i in range(m):
        nn = no[i] * nq
        if nn == 0.0:
            mask[i] = 1 if r <= 0 else 0
            ip[i] = 0.0 if mask[i] else -np.inf
            continue
        t = 2.0 - 2.0 * r / nn
        if t < 0.0:
            continue
        res = dco_batch(bu[i:i + 1], qu, np.array([0]), np.sqrt(t), eps0, delta_d, method, band_rel)
        mask[i] = res["mask"][0]
        dims[i] = res["dims"][0]
        band[i] = res["band"][0]
        if mask[i]:
            d = res["dist"][0]
            ip[i] = nn * (1.0 - 0.5 * d * d)
    return {"mask": mask, "ip": ip, "dims": dims, "band": band}


# ---------------------------------------------------------------------------
# Section 2.2.2 + Section 4: the IVF scan (IVF, IVF+, IVF*)
# ---------------------------------------------------------------------------


def lists_from_assignment(assign: np.ndarray, nlist: int):
    """Inverted lists: (offsets [nlist+1], member ids in ascending id order)."""
    assign = np.asarray(assign, dtype=np.int64)
    order = np.argsort(assign, kind="stable")
    counts = np.bincount(assign, minlength=nlist)
    off = np.zeros(nlist + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off, order.astype(np.int64)


def ivf_search(base_rot: np.ndarray, q_rot: np.ndarray, list_off: np.ndarray,
               list_ids: np.ndarray, probe_ids: np.ndarray, K, eps0: float, delta_d: int,
               method: int = METHOD_ADS, nprobe=None, threads: int = 0,
               row_of_id=None, k_max: int | None = None):
    """Sequential IVF scan per query (threads over queries only).

    base_rot rows are addressed by ``row_of_id[id]`` (identity if None), so a
    caller may pass only the rows of the probed lists.  K and nprobe may be
    scalars or per-query arrays.  Returns (ids [nq,k_max], dist [nq,k_max],
    stats [nq,3] = DCOs, sampled dims, positives).
    """
    lib = _load()
    base = np.ascontiguousarray(base_rot, dtype=np.float64)
    qs = np.ascontiguousarray(q_rot, dtype=np.float64)
    nq, D = qs.shape
    probe_ids = np.ascontiguousarray(probe_ids, dtype=np.int32)
    nprobe_max = probe_ids.shape[1]
    if nprobe is None:
        nprobe = nprobe_max
    npr = np.ascontiguousarray(np.broadcast_to(np.asarray(nprobe, dtype=np.int32), (nq,)))
    Ks = np.ascontiguousarray(np.broadcast_to(np.asarray(K, dtype=np.int32), (nq,)))
    if k_max is None:
        k_max = int(Ks.max()) if nq else 0
    list_off = np.ascontiguousarray(list_off, dtype=np.int64)
    list_ids = np.ascontiguousarray(list_ids, dtype=np.int64)
    if row_of_id is None:
        rows = list_ids.copy()
    else:
        rows = np.ascontiguousarray(np.asarray(row_of_id, dtype=np.int64)[list_ids])
    out_ids = np.zeros((nq, k_max), dtype=np.int64)
    out_dist = np.zeros((nq, k_max))
    stats = np.zeros((nq, 3), dtype=np.int64)
    if threads <= 0:
        threads = os.cpu_count() or 1
    rc = lib.orc_ivf_search(_p(base, ctypes.c_double), _p(qs, ctypes.c_double), nq, D,
                            _p(list_off, ctypes.c_int64), _p(rows, ctypes.c_int64),
                            _p(list_ids, ctypes.c_int64), _p(probe_ids, ctypes.c_int32),
                            _p(npr, ctypes.c_int32), nprobe_max, _p(Ks, ctypes.c_int32),
                            int(k_max), float(eps0), int(delta_d), int(method),
                            _p(out_ids, ctypes.c_int64), _p(out_dist, ctypes.c_double),
                            _p(stats, ctypes.c_int64), int(threads))
    if rc != 0:
        raise MemoryError("oracle ivf_search failed to allocate")
    return out_ids, out_dist, stats


# ---------------------------------------------------------------------------
# Section 2.2.1 / Section 4 / Section 5.1: graph search (HNSW, HNSW+, HNSW++)
# ---------------------------------------------------------------------------

HNSW_PLUS, HNSW_PLAIN, HNSW_PP = 0, 1, 2


def hnsw_dco(o: np.ndarray, q: np.ndarray, r: float, eps0: float, delta_d: int,
             method: int = METHOD_ADS, rel: float = 0.0):
    """One DCO as the graph search runs it (Algorithm 1, or FDScanning with
    ``method`` = METHOD_FDS): (positive, dims, exact distance or inf, observed
    distance when it stopped, band flag)."""
    lib = _load()
    o = np.ascontiguousarray(o, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    dims = ctypes.c_int()
    dis = ctypes.c_double()
    obs = ctypes.c_double()
    band = ctypes.c_int()
    pos = lib.orc_hnsw_dco(_p(o, ctypes.c_double), _p(q, ctypes.c_double), o.shape[0], float(r),
                           float(eps0), int(delta_d), int(method), float(rel), ctypes.byref(dims),
                           ctypes.byref(dis), ctypes.byref(obs), ctypes.byref(band))
    return bool(pos), dims.value, dis.value, obs.value, bool(band.value)


def hnsw_search(base_rot: np.ndarray, q_rot: np.ndarray, graph, K: int, nef: int,
                eps0: float = 2.1, delta_d: int = 32, variant: int = HNSW_PLUS,
                rel: float = 1e-6, rel_exact: float = 0.0, threads: int = 0):
    """Graph search on transformed vectors: HNSW (Section 2.2.1, FDScanning
    DCOs), HNSW+ (Section 4, Algorithm 1 as the DCO) or HNSW++ (Section 5.1,
    R1 of K exact distances for the answer and the DCO threshold, R2 of N_ef
    observed distances for the beam).  ``graph`` carries levels, adj0, up_off,
    up_adj, entry, max_level, M and M0 (the format of the graph input).

    Returns (ids [nq, K] int64, distances [nq, K] float64, stats [nq, 4] int64:
    DCOs, sampled dims, layer-0 expansions, band flag).  The band flag marks a
    query one of whose decisions lies within ``rel`` of its boundary (or whose
    new key lies within ``rel`` of a key it is ordered against; ``rel_exact``
    for two exact distances), where rounding could change the path."""
    lib = _load()
    base = np.ascontiguousarray(base_rot, dtype=np.float64)
    q = np.ascontiguousarray(np.atleast_2d(q_rot), dtype=np.float64)
    n, D = base.shape
    nq = q.shape[0]
    levels = np.ascontiguousarray(graph.levels, dtype=np.int32)
    adj0 = np.ascontiguousarray(graph.adj0, dtype=np.int32)
    up_off = np.ascontiguousarray(graph.up_off, dtype=np.int64)
    up_adj = np.ascontiguousarray(graph.up_adj, dtype=np.int32)
    ids = np.empty((nq, K), dtype=np.int64)
    dist = np.empty((nq, K), dtype=np.float64)
    stats = np.zeros((nq, 4), dtype=np.int64)
    if threads <= 0:
        threads = min(16, os.cpu_count() or 1)
    st = lib.orc_hnsw_search(_p(base, ctypes.c_double), n, D, _p(q, ctypes.c_double), nq,
                             _p(levels, ctypes.c_int32), _p(adj0, ctypes.c_int32),
                             adj0.shape[1], _p(up_off, ctypes.c_int64),
                             _p(up_adj, ctypes.c_int32), up_adj.shape[1], int(graph.entry),
                             int(graph.max_level), int(K), int(nef), float(eps0), int(delta_d),
                             int(variant), float(rel), float(rel_exact),
                             _p(ids, ctypes.c_int64), _p(dist, ctypes.c_double),
                             _p(stats, ctypes.c_int64), int(threads))
    if st != 0:
        raise ValueError("oracle hnsw_search: bad arguments or allocation failure")
    return ids, dist, stats


# ---------------------------------------------------------------------------
# Section 2.2.2 (index phase): k-means clustering into the inverted lists
# ---------------------------------------------------------------------------

_MASK64 = (1 << 64) - 1
_GOLDEN64 = 0x9E3779B97F4A7C15


def splitmix64(x: int) -> int:
    """The SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014) of a
    64-bit state value."""
    z = x & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def kmeans_init_rows(n: int, nlist: int, seed: int) -> np.ndarray:
    """The nlist distinct rows of the seeded initialisation: row i draws the
    SplitMix64 value of the counter seed + (i + 1) * golden gamma; the rows with
    the nlist smallest values, in ascending value order, seed lists 0..nlist-1."""
    keys = [splitmix64((seed + (i + 1) * _GOLDEN64) & _MASK64) for i in range(n)]
    return np.array(sorted(range(n), key=lambda i: keys[i])[:nlist], dtype=np.int64)


def _nearest(x: np.ndarray, c: np.ndarray):
    """Nearest centre of every row (difference form, ties to the lower id) and
    the squared distance to it."""
    lab = np.empty(x.shape[0], dtype=np.int64)
    d2 = np.empty(x.shape[0])
    for i in range(x.shape[0]):
        diff = c - x[i][None, :]
        dd = np.einsum("ij,ij->i", diff, diff)
        j = int(np.argmin(dd))          # first minimum: the lower id on ties
        lab[i] = j
        d2[i] = dd[j]
    return lab, d2


def kmeans(x: np.ndarray, nlist: int, iters: int, seed: int = 0, init=None):
    """Lloyd's k-means in float64 (the IVF index phase clusters the data with
    k-means, Section 2.2.2; Section 6.1).  Readings where the paper is silent:
    the seeded initial rows of kmeans_init_rows; every iteration assigns each
    row to its nearest centre (ties to the lower id), then gives every empty
    list, in ascending id order, the member of the currently largest list
    (lower id on ties) that lies farthest from its centre (lower row on ties),
    then moves every centre to the mean of its members; a final assignment to
    the final centres gives the lists.

    ``init`` (row indices) replaces the seeded initial rows when given.

    Returns (centres [nlist, D] float64, assignment [n] int64)."""
    xd = np.asarray(x, dtype=np.float64)
    n = xd.shape[0]
    if init is None:
        init = kmeans_init_rows(n, nlist, seed)
    init = np.asarray(init, dtype=np.int64)
    c = xd[init].copy()
    for _ in range(iters):
        lab, d2 = _nearest(xd, c)
        counts = np.bincount(lab, minlength=nlist)
        for j in range(nlist):
            if counts[j] > 0:
                continue
            big = int(np.argmax(counts))            # first maximum: the lower id
            members = np.flatnonzero(lab == big)
            far = members[np.argmax(d2[members])]   # first maximum: the lower row
            lab[far] = j
            counts[big] -= 1
            counts[j] = 1
        for j in range(nlist):
            c[j] = xd[lab == j].mean(axis=0)
    lab, _ = _nearest(xd, c)
    return c, lab


# ---------------------------------------------------------------------------
# Section 6.1: metrics
# ---------------------------------------------------------------------------


def recall(ret_ids: np.ndarray, ret_dist_exact: np.ndarray, gt_dist: np.ndarray, K) -> float:
    """Mean recall@K, tie-aware.

    A returned object counts as a retrieved ground-truth neighbour when its
    exact distance is at most the exact K-th ground-truth distance (objects
    tied at that distance are interchangeable); the count is capped at K.
    """
    nq = ret_ids.shape[0]
    Ks = np.broadcast_to(np.asarray(K), (nq,))
    tot = 0.0
    for i in range(nq):
        k = int(Ks[i])
        if k == 0:
            tot += 1.0
            continue
        kth = gt_dist[i, k - 1]
        valid = ret_ids[i, :k] >= 0
        hit = np.count_nonzero(valid & (ret_dist_exact[i, :k] <= kth))
        tot += min(hit, k) / k
    return tot / nq


def distance_ratio(ret_dist_exact: np.ndarray, gt_dist: np.ndarray, K) -> float:
    """Average distance ratio: mean over ranks of dis(returned_i) / dis(gt_i) (0/0 := 1)."""
    nq = ret_dist_exact.shape[0]
    Ks = np.broadcast_to(np.asarray(K), (nq,))
    vals = []
    for i in range(nq):
        k = int(Ks[i])
        a = ret_dist_exact[i, :k]
        b = gt_dist[i, :k]
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where((a == 0) & (b == 0), 1.0, a / b)
        vals.append(np.mean(r) if k else 1.0)
    return float(np.mean(vals))


def dims_ratio(stats: np.ndarray, D: int) -> float:
    """Total sampled dimensions over D times the number of DCOs."""
    s = np.asarray(stats)
    return float(s[:, 1].sum()) / float(D * max(1, s[:, 0].sum()))
