"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library.

This module draws random numbers and nothing else of the method: it holds no
distance comparison, no hypothesis test, no rotation arithmetic and no top-K
logic.  Everything here is a pure function of its seeds, so the oracle and the
GPU path receive bit-identical inputs.

What it provides:

* base and query vectors shaped like the paper's workloads (Table 1 gives
  million-scale sets with D from 256 to 960; the D=128 integer mixture follows
  the SIFT-style data the introduction cites).  The real datasets are not used;
  these generators stand in for them;
* the Gaussian matrix G whose orthonormalisation is the random rotation of
  Section 3.1 (the QR itself belongs to each side, not to this module);
* the IVF clustering handed to both sides.  In the paper the clustering comes
  from an external k-means library (Section 6.1, Implementation), not from the
  method, so here it is an input as well: a seeded Lloyd k-means on a
  subsample plus a nearest-centre assignment of every vector;
* per-query K and nprobe draws for the uneven batched workload.

Generation is chunked: chunk ``i`` of a stream with seed ``s`` uses
``numpy.random.default_rng([s, i])``, so results do not depend on the number of
worker threads.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

CHUNK_ROWS = 16384


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n: int, D: int, seed: int, fill) -> np.ndarray:
    """Fill an [n, D] float32 array chunk by chunk; chunk i gets rng([seed, i])."""
    out = np.empty((n, D), dtype=np.float32)
    starts = list(range(0, n, CHUNK_ROWS))

    def work(ci: int) -> None:
        s = starts[ci]
        e = min(n, s + CHUNK_ROWS)
        rng = np.random.default_rng([seed, ci])
        out[s:e] = fill(rng, e - s)

    if len(starts) == 1:
        work(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(len(starts))))
    return out


# ---------------------------------------------------------------------------
# Vector models
# ---------------------------------------------------------------------------

def mixture_centres(D: int, n_centres: int, model_seed: int) -> np.ndarray:
    """Centres of the integer Gaussian mixture, uniform on [0, 100]^D."""
    rng = np.random.default_rng(model_seed)
    return rng.uniform(0.0, 100.0, size=(n_centres, D))


def mixture(n: int, D: int, seed: int, model_seed: int, n_centres: int = 32,
            sigma: float = 10.0) -> np.ndarray:
    """Integer-valued Gaussian mixture: x = rint(clip(c_k + sigma*N(0, I), 0, 255)).

    The component k of each row is uniform over the centres.  All values are
    integers in [0, 255], stored as float32 (exactly representable).
    """
    centres = mixture_centres(D, n_centres, model_seed)

    def fill(rng, m):
        comp = rng.integers(0, n_centres, size=m)
        x = centres[comp] + sigma * rng.standard_normal((m, D))
        return np.rint(np.clip(x, 0.0, 255.0))

    return _chunked(n, D, seed, fill)


def lowrank_basis(latent: int, D: int, w_seed: int) -> np.ndarray:
    """W ~ N(0, 1/latent) of shape [latent, D], float64."""
    rng = np.random.default_rng(w_seed)
    return rng.standard_normal((latent, D)) / np.sqrt(latent)


def lowrank(n: int, D: int, seed: int, w_seed: int, latent: int = 64,
            noise: float = 0.1) -> np.ndarray:
    """Low-rank-plus-noise vectors: x = z W + noise * N(0, I_D), z ~ N(0, I_latent)."""
    W = lowrank_basis(latent, D, w_seed).astype(np.float32)

    def fill(rng, m):
        z = rng.standard_normal((m, latent), dtype=np.float32)
        e = rng.standard_normal((m, D), dtype=np.float32)
        return z @ W + np.float32(noise) * e

    return _chunked(n, D, seed, fill)


def gaussian_matrix(D: int, seed: int) -> np.ndarray:
    """G with i.i.d. N(0, 1) entries, [D, D] float64 (input of the rotation QR)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((D, D))


# ---------------------------------------------------------------------------
# IVF clustering (an input to the index build, as in the paper)
# ---------------------------------------------------------------------------

def _nearest(x: np.ndarray, c: np.ndarray, c_norm: np.ndarray,
             rows: int = 8192) -> tuple[np.ndarray, np.ndarray]:
    """Nearest centre per row of x (float32 GEMM form, ties to the lower id)."""
    n = x.shape[0]
    lab = np.empty(n, dtype=np.int32)
    dist = np.empty(n, dtype=np.float32)
    ct = np.ascontiguousarray(c.T)
    for s in range(0, n, rows):
        e = min(n, s + rows)
        xb = x[s:e]
        score = c_norm[None, :] - 2.0 * (xb @ ct)
        j = np.argmin(score, axis=1)
        lab[s:e] = j
        xn = np.einsum("ij,ij->i", xb, xb)
        dist[s:e] = np.maximum(score[np.arange(e - s), j] + xn, 0.0)
    return lab, dist


def clustering(x: np.ndarray, nlist: int, seed: int, iters: int = 10,
               train_per_list: int = 16) -> tuple[np.ndarray, np.ndarray]:
    """Seeded Lloyd k-means; returns (centroids [nlist, D] f32, list id per row i32).

    * training set: min(n, train_per_list * nlist) rows drawn without
      replacement with ``default_rng(seed)``;
    * initial centres: nlist distinct training rows drawn with the same rng;
    * ``iters`` Lloyd iterations (assign to the nearest centre, ties to the
      lower id; move each centre to the mean of its members);
    * an empty cluster takes the training row that is farthest from its own
      centre (lowest row index first), one row per empty cluster;
    * finally every row of x is assigned to its nearest centre.
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, D = x.shape
    if nlist < 1 or nlist > n:
        raise ValueError("nlist must be in [1, n]")
    rng = np.random.default_rng(seed)
    n_train = min(n, train_per_list * nlist)
    train_idx = np.sort(rng.choice(n, size=n_train, replace=False))
    xt = x[train_idx]
    init = rng.choice(n_train, size=nlist, replace=False)
    c = xt[init].astype(np.float32).copy()
    for _ in range(iters):
        c_norm = np.einsum("ij,ij->i", c, c)
        lab, dist = _nearest(xt, c, c_norm)
        sums = np.zeros((nlist, D), dtype=np.float64)
        _segsum(sums, lab, xt)
        cnt = np.bincount(lab, minlength=nlist)
        nz = cnt > 0
        c[nz] = (sums[nz] / cnt[nz, None]).astype(np.float32)
        empty = np.flatnonzero(~nz)
        if empty.size:
            order = np.lexsort((np.arange(n_train), -dist.astype(np.float64)))
            for k, j in enumerate(empty):
                c[j] = xt[order[k]]
    c_norm = np.einsum("ij,ij->i", c, c)
    lab, _ = _nearest(x, c, c_norm)
    return c, lab


def _segsum(sums: np.ndarray, lab: np.ndarray, xt: np.ndarray) -> None:
    order = np.argsort(lab, kind="stable")
    ls = lab[order]
    bounds = np.flatnonzero(np.diff(ls)) + 1
    starts = np.concatenate(([0], bounds))
    red = np.add.reduceat(xt[order].astype(np.float64), starts, axis=0)
    sums[ls[starts]] = red


# ---------------------------------------------------------------------------
# Workload presets (sizes and seeds of the five benchmark workloads)
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    model: str              # "mix" or "lowrank"
    n: int
    nq: int
    D: int
    nlist: int
    p_seed: int
    base_seed: int
    query_seed: int
    kmeans_seed: int = 0
    model_seed: int = 0     # mixture centres or low-rank basis W
    draw_seed: int = 0      # per-query K / nprobe draws
    latent: int = 64
    noise: float = 0.1
    K: int = 10
    nprobe: int = 16
    delta_d: int = 32
    eps0: float = 2.1
    kmeans_iters: int = 10
    extra: dict = field(default_factory=dict)

    def scaled(self, **kw) -> "Workload":
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


WORKLOADS = {
    # flat ADSampling scan of one list (nlist = 1)
    "flat_d128": Workload("flat_d128", "mix", n=10_000, nq=100, D=128, nlist=1,
                          p_seed=1001, base_seed=1002, query_seed=1003,
                          model_seed=1000, K=10, nprobe=1),
    "ivf_d128": Workload("ivf_d128", "mix", n=1_000_000, nq=10_000, D=128, nlist=4096,
                         p_seed=1001, base_seed=1012, query_seed=1013,
                         kmeans_seed=1014, model_seed=1000, K=10, nprobe=16),
    "ivf_d960": Workload("ivf_d960", "lowrank", n=1_000_000, nq=1_000, D=960, nlist=4096,
                         p_seed=1001, base_seed=1022, query_seed=1023,
                         kmeans_seed=1024, model_seed=1025, latent=64, noise=0.1,
                         K=10, nprobe=768, delta_d=16),
    "batched_d256": Workload("batched_d256", "lowrank", n=2_000_000, nq=4_096, D=256,
                             nlist=8192, p_seed=1001, base_seed=1032, query_seed=1033,
                             kmeans_seed=1034, model_seed=1035, draw_seed=1036,
                             latent=32, noise=0.05, K=100, nprobe=128),
}


def base_vectors(w: Workload) -> np.ndarray:
    if w.model == "mix":
        return mixture(w.n, w.D, w.base_seed, w.model_seed)
    return lowrank(w.n, w.D, w.base_seed, w.model_seed, w.latent, w.noise)


def query_vectors(w: Workload) -> np.ndarray:
    if w.model == "mix":
        return mixture(w.nq, w.D, w.query_seed, w.model_seed)
    return lowrank(w.nq, w.D, w.query_seed, w.model_seed, w.latent, w.noise)


def rotation_gaussian(w: Workload) -> np.ndarray:
    return gaussian_matrix(w.D, w.p_seed)


def ivf_clustering(w: Workload, x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    if w.nlist == 1:
        return x.mean(axis=0, dtype=np.float64)[None, :].astype(np.float32), \
            np.zeros(x.shape[0], dtype=np.int32)
    return clustering(x, w.nlist, w.kmeans_seed, w.kmeans_iters)


def uneven_draws(w: Workload, nprobe_lo: int = 8, nprobe_hi: int = 128,
                 k_choices=(10, 100)) -> tuple[np.ndarray, np.ndarray]:
    """Per-query (K, nprobe): K uniform over k_choices, nprobe uniform on [lo, hi]."""
    rng = np.random.default_rng(w.draw_seed)
    K = rng.choice(np.asarray(k_choices, dtype=np.int32), size=w.nq).astype(np.int32)
    nprobe = rng.integers(nprobe_lo, nprobe_hi + 1, size=w.nq).astype(np.int32)
    return K, nprobe


def poisson_arrivals(rate: float, count: int, seed: int = 1047) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
