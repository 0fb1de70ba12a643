"""ctypes binding of libads.so (include/ads.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; PyTorch only
provides device memory and the current HIP stream.  If the library is not
built, every call raises: there is no fallback.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libads.so")

ADS_OK, ADS_EINVAL, ADS_ENOMEM, ADS_EHIP, ADS_EUNSUPPORTED = 0, -1, -2, -3, -4
F32, BF16, F16 = 0, 1, 2
ADSAMPLING, FDSCANNING, PDSCANNING = 0, 1, 2
STAT_DCOS, STAT_DIMS, STAT_POSITIVES, STAT_BYTES, NSTATS = 0, 1, 2, 3, 4

EXPORTED = [
    "ads_make_rotation", "ads_rotate", "ads_ivf_build", "ads_index_info", "ads_index_lists",
    "ads_index_free", "ads_dco_batch", "ads_search", "ads_search_workspace_size",
    "ads_last_error", "ads_version", "ads_profile_enable", "ads_profile_collect",
    "ads_set_tuning", "ads_get_tuning", "ads_plan_create", "ads_plan_launch", "ads_plan_free",
    "ads_dco_batch_ip", "ads_search_noalloc", "ads_kmeans", "ads_build_ivf",
    "ads_hnsw_create", "ads_hnsw_workspace_size", "ads_hnsw_search", "ads_hnsw_free",
]
HNSW_PLUS, HNSW_PLAIN, HNSW_PP = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 256 << 20       # ADS_NOALLOC_SCRATCH_BYTES
METRIC_L2, METRIC_COSINE = 0, 1
PHASES = ["rotate", "probe", "group", "scan", "merge", "output"]


class Tuning(ctypes.Structure):
    _fields_ = [("dense_frac", ctypes.c_float), ("queries_per_unit", ctypes.c_int32),
                ("sweep_log2", ctypes.c_int32), ("grid_per_xcd", ctypes.c_int32),
                ("prefetch_units", ctypes.c_int32)]


class AdsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"ads status {status}: {message}")
        self.status = status


class IndexDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("D", ctypes.c_int32), ("nlist", ctypes.c_int32),
                ("delta_d", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("has_fp32_copy", ctypes.c_int32), ("max_list", ctypes.c_int32),
                ("metric", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("rotated", ctypes.c_int32), ("a1_dims", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libads.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2303_09855_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    lib.ads_make_rotation.argtypes = [vp, i32, vp, vp]
    lib.ads_rotate.argtypes = [vp, i32, vp, i64, vp, vp]
    lib.ads_ivf_build.argtypes = [vp, i64, i32, vp, vp, i32, vp, i32, i32, i32, i32, vp,
                                  ctypes.POINTER(vp)]
    lib.ads_dco_batch_ip.argtypes = [vp, vp, vp, i64, f32, f32, i32, i32, vp, vp, vp, vp, vp]
    lib.ads_index_info.argtypes = [vp, ctypes.POINTER(IndexDesc)]
    lib.ads_index_lists.argtypes = [vp, vp, vp, vp, vp]
    lib.ads_index_free.argtypes = [vp]
    lib.ads_dco_batch.argtypes = [vp, vp, vp, i64, f32, f32, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.ads_search.argtypes = [vp, vp, i32, vp, vp, i32, i32, f32, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.ads_kmeans.argtypes = [vp, i64, i32, i32, i32, ctypes.c_uint64, vp, vp, vp]
    lib.ads_build_ivf.argtypes = [vp, i64, i32, vp, i32, i32, ctypes.c_uint64, i32, i32, i32, i32, vp, vp,
                                  vp, ctypes.POINTER(vp)]
    lib.ads_search_noalloc.argtypes = [vp, vp, i32, vp, vp, i32, i32, f32, i32, i32, vp, vp, vp, vp, vp]
    lib.ads_search_workspace_size.argtypes = [vp, i32, i32, i32, i32]
    lib.ads_search_workspace_size.restype = ctypes.c_uint64
    lib.ads_plan_create.argtypes = [vp, vp, i32, vp, vp, i32, i32, f32, i32, i32, vp, vp, vp, vp,
                                    ctypes.POINTER(vp)]
    lib.ads_plan_launch.argtypes = [vp, vp]
    lib.ads_plan_free.argtypes = [vp]
    lib.ads_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.ads_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.ads_profile_enable.argtypes = [i32]
    lib.ads_profile_collect.argtypes = [vp, vp]
    lib.ads_hnsw_create.argtypes = [vp, i64, i32, vp, vp, vp, i32, vp, vp, i64, i32, i32, i32, vp,
                                    ctypes.POINTER(vp)]
    lib.ads_hnsw_workspace_size.argtypes = [vp, i32]
    lib.ads_hnsw_workspace_size.restype = ctypes.c_uint64
    lib.ads_hnsw_search.argtypes = [vp, vp, i32, i32, i32, f32, i32, vp, vp, vp, vp, vp, vp]
    lib.ads_hnsw_free.argtypes = [vp]
    lib.ads_last_error.restype = ctypes.c_char_p
    lib.ads_version.restype = ctypes.c_char_p
    for name in ["ads_make_rotation", "ads_rotate", "ads_ivf_build", "ads_index_info",
                 "ads_index_lists", "ads_index_free", "ads_dco_batch", "ads_search",
                 "ads_profile_enable", "ads_profile_collect", "ads_set_tuning", "ads_get_tuning",
                 "ads_plan_create", "ads_plan_launch", "ads_plan_free", "ads_dco_batch_ip",
                 "ads_hnsw_create", "ads_hnsw_search", "ads_hnsw_free"]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st: int) -> None:
    if st != ADS_OK:
        raise AdsError(st, load().ads_last_error().decode())


def last_error() -> str:
    return load().ads_last_error().decode()


def version() -> str:
    return load().ads_version().decode()


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.ascontiguousarray(t))
    t = t.to(device="cuda", dtype=dtype)
    return t.contiguous()


# ---------------------------------------------------------------------------
# Rotation
# ---------------------------------------------------------------------------

def make_rotation(gaussian: np.ndarray):
    """Host Householder QR of a Gaussian matrix -> (P float32, P float64)."""
    g = np.ascontiguousarray(gaussian, dtype=np.float64)
    D = g.shape[0]
    if g.shape != (D, D):
        raise ValueError("gaussian must be square")
    P = np.empty((D, D), dtype=np.float32)
    P64 = np.empty((D, D), dtype=np.float64)
    _check(load().ads_make_rotation(g.ctypes.data_as(ctypes.c_void_p), D,
                                    P.ctypes.data_as(ctypes.c_void_p),
                                    P64.ctypes.data_as(ctypes.c_void_p)))
    return P, P64


def rotate(P, X):
    """Y = X P^T on the GPU (float32 tensors)."""
    torch = _torch()
    P = _dev(P, torch.float32)
    X = _dev(X, torch.float32)
    n, D = X.shape
    Y = torch.empty((n, D), dtype=torch.float32, device="cuda")
    _check(load().ads_rotate(_ptr(P), D, _ptr(X), n, _ptr(Y), _stream()))
    return Y


# ---------------------------------------------------------------------------
# Index
# ---------------------------------------------------------------------------

class Index:
    """Owning handle of an ads_index."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("index was freed")
        return self._h

    def info(self) -> dict:
        d = IndexDesc()
        _check(load().ads_index_info(self.handle, ctypes.byref(d)))
        return {f: getattr(d, f) for f, _ in IndexDesc._fields_}

    def lists(self):
        """(offsets [nlist+1] int64, stored ids [n] int64, rotated centres) as CPU arrays."""
        torch = _torch()
        inf = self.info()
        off = torch.empty(inf["nlist"] + 1, dtype=torch.int64, device="cuda")
        ids = torch.empty(inf["n"], dtype=torch.int64, device="cuda")
        cen = torch.empty((inf["nlist"], inf["D"]), dtype=torch.float32, device="cuda")
        _check(load().ads_index_lists(self.handle, _ptr(off), _ptr(ids), _ptr(cen), _stream()))
        torch.cuda.current_stream().synchronize()
        return off.cpu().numpy(), ids.cpu().numpy(), cen.cpu().numpy()

    def free(self) -> None:
        if self._h:
            load().ads_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def ivf_build(base, P, centroids, assign, delta_d: int = 32, storage: int = F32,
              keep_fp32: bool = True, metric: int = METRIC_L2) -> Index:
    torch = _torch()
    base = _dev(base, torch.float32)
    P = _dev(P, torch.float32) if P is not None else None      # None: unrotated index
    centroids = _dev(centroids, torch.float32)
    assign = _dev(assign, torch.int32)
    n, D = base.shape
    out = ctypes.c_void_p()
    _check(load().ads_ivf_build(_ptr(base), n, D, _ptr(P), _ptr(centroids), centroids.shape[0],
                                _ptr(assign), int(delta_d), int(storage), int(bool(keep_fp32)),
                                int(metric), _stream(), ctypes.byref(out)))
    return Index(out)


class HnswIndex:
    """Owning handle of an ads_hnsw graph index."""

    def __init__(self, handle: ctypes.c_void_p, n: int, D: int):
        self._h = handle
        self.n, self.D = n, D

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("graph index was freed")
        return self._h

    def free(self) -> None:
        if self._h:
            load().ads_hnsw_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def hnsw_create(base, P, graph, delta_d: int = 16) -> HnswIndex:
    """ads_hnsw_create from a graph given on the host (``graph`` carries levels,
    adj0, up_off, up_adj, entry, M).  P None stores the vectors unrotated."""
    torch = _torch()
    base = _dev(base, torch.float32)
    P = _dev(P, torch.float32) if P is not None else None
    n, D = base.shape
    levels = np.ascontiguousarray(graph.levels, dtype=np.int32)
    adj0 = np.ascontiguousarray(graph.adj0, dtype=np.int32)
    up_off = np.ascontiguousarray(graph.up_off, dtype=np.int64)
    up_adj = np.ascontiguousarray(graph.up_adj, dtype=np.int32)
    rows = int(up_adj.shape[0]) if int(levels.max()) > 0 else 0
    out = ctypes.c_void_p()
    _check(load().ads_hnsw_create(_ptr(base), n, D, _ptr(P), levels.ctypes.data, adj0.ctypes.data,
                                  int(adj0.shape[1]), up_off.ctypes.data, up_adj.ctypes.data, rows,
                                  int(up_adj.shape[1]), int(graph.entry), int(delta_d), _stream(),
                                  ctypes.byref(out)))
    return HnswIndex(out, n, D)


def hnsw_search(index: HnswIndex, q, K: int, nef: int, eps0: float = 2.1,
                variant: int = HNSW_PLUS, qstats=None, stats=None, workspace=None):
    """ads_hnsw_search.  Returns (ids int64 [nq, K], dist float32 [nq, K])."""
    torch = _torch()
    q = _dev(q, torch.float32)
    nq = q.shape[0]
    ids = torch.empty((nq, K), dtype=torch.int64, device="cuda")
    dist = torch.empty((nq, K), dtype=torch.float32, device="cuda")
    e = math.inf if eps0 is None else float(eps0)
    _check(load().ads_hnsw_search(index.handle, _ptr(q), nq, int(K), int(nef), e, int(variant),
                                  _ptr(ids), _ptr(dist), _ptr(qstats), _ptr(stats), _ptr(workspace),
                                  _stream()))
    return ids, dist


def hnsw_workspace_size(index: HnswIndex, nq: int) -> int:
    return int(load().ads_hnsw_workspace_size(index.handle, nq))


def kmeans(x, nlist: int, iters: int = 10, seed: int = 0):
    """GPU k-means (ads_kmeans).  Returns (centroids [nlist, D] float32,
    assignment [n] int32) as device tensors."""
    torch = _torch()
    x = _dev(x, torch.float32)
    n, D = x.shape
    cent = torch.empty((nlist, D), dtype=torch.float32, device="cuda")
    assign = torch.empty(n, dtype=torch.int32, device="cuda")
    _check(load().ads_kmeans(_ptr(x), n, D, int(nlist), int(iters), ctypes.c_uint64(seed), _ptr(cent),
                             _ptr(assign), _stream()))
    return cent, assign


def build_ivf(base, P, nlist: int, iters: int = 10, seed: int = 0, delta_d: int = 32,
              storage: int = F32, keep_fp32: bool = True, metric: int = METRIC_L2,
              want_clustering: bool = False):
    """Index phase on the GPU: k-means then the blocked layout (ads_build_ivf).
    Returns the Index, or (Index, centroids, assignment) with want_clustering."""
    torch = _torch()
    base = _dev(base, torch.float32)
    P = _dev(P, torch.float32) if P is not None else None
    n, D = base.shape
    cent = torch.empty((nlist, D), dtype=torch.float32, device="cuda") if want_clustering else None
    assign = torch.empty(n, dtype=torch.int32, device="cuda") if want_clustering else None
    out = ctypes.c_void_p()
    _check(load().ads_build_ivf(_ptr(base), n, D, _ptr(P), int(nlist), int(iters), ctypes.c_uint64(seed),
                                int(delta_d), int(storage), int(bool(keep_fp32)), int(metric), _ptr(cent),
                                _ptr(assign), _stream(), ctypes.byref(out)))
    ix = Index(out)
    if want_clustering:
        return ix, cent, assign
    return ix


# ---------------------------------------------------------------------------
# Query phase
# ---------------------------------------------------------------------------

def dco_batch(index: Index, q_rot, cand, r: float, eps0: float, delta_d: int,
              method: int = ADSAMPLING, source: int = 0, stats=None):
    """Returns (mask uint8, dist float32, dims int32) tensors on the GPU."""
    torch = _torch()
    q_rot = _dev(q_rot, torch.float32).reshape(-1)
    cand = _dev(cand, torch.int64).reshape(-1)
    m = cand.shape[0]
    mask = torch.empty(m, dtype=torch.uint8, device="cuda")
    dist = torch.empty(m, dtype=torch.float32, device="cuda")
    dims = torch.empty(m, dtype=torch.int32, device="cuda")
    _check(load().ads_dco_batch(index.handle, _ptr(q_rot), _ptr(cand), m, float(r), float(eps0),
                                int(delta_d), int(method), int(source), _ptr(mask), _ptr(dist),
                                _ptr(dims), _ptr(stats), _stream()))
    return mask, dist, dims


def dco_batch_ip(index: Index, q, cand, r: float, eps0: float, delta_d: int,
                 method: int = ADSAMPLING, stats=None):
    """Inner-product comparisons <o,q> >= r on a cosine index (q raw).
    Returns (mask uint8, ip float32 (-inf for negatives), dims int32)."""
    torch = _torch()
    q = _dev(q, torch.float32).reshape(-1)
    cand = _dev(cand, torch.int64).reshape(-1)
    m = cand.shape[0]
    mask = torch.empty(m, dtype=torch.uint8, device="cuda")
    ip = torch.empty(m, dtype=torch.float32, device="cuda")
    dims = torch.empty(m, dtype=torch.int32, device="cuda")
    _check(load().ads_dco_batch_ip(index.handle, _ptr(q), _ptr(cand), m, float(r), float(eps0),
                                   int(delta_d), int(method), _ptr(mask), _ptr(ip), _ptr(dims),
                                   _ptr(stats), _stream()))
    return mask, ip, dims


def search_workspace_size(index: Index, nq: int, k_max: int, nprobe_max: int, rerank: int = 0) -> int:
    v = load().ads_search_workspace_size(index.handle, nq, k_max, nprobe_max, rerank)
    if v == 0:
        raise AdsError(ADS_EINVAL, last_error())
    return int(v)


def search(index: Index, q, k_max: int, nprobe_max: int, eps0: float = 2.1,
           method: int = ADSAMPLING, K=None, nprobe=None, rerank: int = 0,
           want_probes: bool = False, stats=None, workspace=None, out=None):
    """Batched IVF+ search.  Returns (ids int64 [nq,k_max], dist float32[, probes])."""
    torch = _torch()
    q = _dev(q, torch.float32)
    nq = q.shape[0]
    Kt = _dev(K, torch.int32) if K is not None else None
    Nt = _dev(nprobe, torch.int32) if nprobe is not None else None
    if out is None:
        ids = torch.empty((nq, k_max), dtype=torch.int64, device="cuda")
        dist = torch.empty((nq, k_max), dtype=torch.float32, device="cuda")
    else:
        ids, dist = out
    probes = torch.empty((nq, nprobe_max), dtype=torch.int32, device="cuda") if want_probes else None
    e = math.inf if eps0 is None else float(eps0)
    _check(load().ads_search(index.handle, _ptr(q), nq, _ptr(Kt), _ptr(Nt), int(k_max),
                             int(nprobe_max), e, int(method), int(rerank), _ptr(ids), _ptr(dist),
                             _ptr(probes), _ptr(stats), _ptr(workspace), _stream()))
    if want_probes:
        return ids, dist, probes
    return ids, dist


def search_noalloc(index: Index, q, k_max: int, nprobe_max: int, eps0: float = 2.1,
                   method: int = ADSAMPLING, K=None, nprobe=None, rerank: int = 0,
                   want_probes: bool = False, stats=None, out=None):
    """ads_search_noalloc: the search with the library's file-scope scratch
    array as workspace (no device allocation by the library).  Output buffers
    are allocated here unless ``out`` = (ids, dist) is given."""
    torch = _torch()
    q = _dev(q, torch.float32)
    nq = q.shape[0]
    Kt = _dev(K, torch.int32) if K is not None else None
    Nt = _dev(nprobe, torch.int32) if nprobe is not None else None
    if out is None:
        ids = torch.empty((nq, k_max), dtype=torch.int64, device="cuda")
        dist = torch.empty((nq, k_max), dtype=torch.float32, device="cuda")
    else:
        ids, dist = out
    probes = torch.empty((nq, nprobe_max), dtype=torch.int32, device="cuda") if want_probes else None
    e = math.inf if eps0 is None else float(eps0)
    _check(load().ads_search_noalloc(index.handle, _ptr(q), nq, _ptr(Kt), _ptr(Nt), int(k_max),
                                     int(nprobe_max), e, int(method), int(rerank), _ptr(ids),
                                     _ptr(dist), _ptr(probes), _ptr(stats), _stream()))
    if want_probes:
        return ids, dist, probes
    return ids, dist


# ---------------------------------------------------------------------------
# Per-phase event timing
# ---------------------------------------------------------------------------

def profile_enable(on: bool = True) -> None:
    _check(load().ads_profile_enable(1 if on else 0))


def profile_collect() -> dict:
    """{phase: (milliseconds, launches)} accumulated since the last collect."""
    ms = np.zeros(len(PHASES), dtype=np.float64)
    n = np.zeros(len(PHASES), dtype=np.int64)
    _check(load().ads_profile_collect(ms.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p)))
    return {p: (float(ms[i]), int(n[i])) for i, p in enumerate(PHASES)}


# ---------------------------------------------------------------------------
# Scheduling knobs
# ---------------------------------------------------------------------------

def get_tuning() -> dict:
    t = Tuning()
    _check(load().ads_get_tuning(ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in Tuning._fields_}


def set_tuning(**kw) -> None:
    """Update the calling thread's scan knobs (dense_frac, queries_per_unit,
    sweep_log2, grid_per_xcd, prefetch_units); unspecified ones keep their value."""
    cur = get_tuning()
    unknown = set(kw) - set(cur)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    cur.update({k: v for k, v in kw.items() if v is not None})
    t = Tuning(float(cur["dense_frac"]), int(cur["queries_per_unit"]), int(cur["sweep_log2"]),
               int(cur["grid_per_xcd"]), int(cur["prefetch_units"]))
    _check(load().ads_set_tuning(ctypes.byref(t)))


# ---------------------------------------------------------------------------
# Captured searches (one HIP graph launch per batch)
# ---------------------------------------------------------------------------

class Plan:
    """A search recorded into a HIP graph for fixed buffers.

    Write new queries into ``plan.q`` (and per-query ``plan.K`` / ``plan.nprobe``)
    in place, call ``launch()``, read ``plan.ids`` / ``plan.dist``."""

    def __init__(self, index: Index, nq: int, k_max: int, nprobe_max: int, eps0: float = 2.1,
                 method: int = ADSAMPLING, rerank: int = 0, stream=None):
        torch = _torch()
        self.index = index
        D = index.info()["D"]
        self.q = torch.zeros((nq, D), dtype=torch.float32, device="cuda")
        self.K = torch.full((nq,), k_max, dtype=torch.int32, device="cuda")
        self.nprobe = torch.full((nq,), nprobe_max, dtype=torch.int32, device="cuda")
        self.ids = torch.empty((nq, k_max), dtype=torch.int64, device="cuda")
        self.dist = torch.empty((nq, k_max), dtype=torch.float32, device="cuda")
        ws = search_workspace_size(index, nq, k_max, nprobe_max, rerank)
        self.workspace = torch.empty(ws + 256, dtype=torch.uint8, device="cuda")
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = ctypes.c_void_p(self.workspace.data_ptr() + off)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        e = math.inf if eps0 is None else float(eps0)
        _check(load().ads_plan_create(index.handle, _ptr(self.q), nq, _ptr(self.K), _ptr(self.nprobe),
                                      int(k_max), int(nprobe_max), e, int(method), int(rerank),
                                      _ptr(self.ids), _ptr(self.dist), self._ws_ptr,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None) -> None:
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(load().ads_plan_launch(self._h, ctypes.c_void_p(s.cuda_stream)))

    def free(self) -> None:
        if self._h:
            load().ads_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
