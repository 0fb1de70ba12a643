"""Shared setup for the parity tests: seeded inputs, the oracle's view and the
GPU library's view of the same IVF workload."""

from __future__ import annotations

import math

import numpy as np

import oracle
import synthdata as sd


class Workload:
    """Raw inputs plus the oracle's FP64 rotated copies (no GPU involved)."""

    def __init__(self, model: str, n: int, nq: int, D: int, nlist: int, seed: int,
                 latent: int = 64, noise: float = 0.1, kmeans_iters: int = 5, kmeans: bool = True):
        self.n, self.nq, self.D, self.nlist = n, nq, D, nlist
        if model == "mix":
            self.x = sd.mixture(n, D, seed, 1000)
            self.q = sd.mixture(nq, D, seed + 1, 1000)
        else:
            self.x = sd.lowrank(n, D, seed, seed + 7, latent, noise)
            self.q = sd.lowrank(nq, D, seed + 1, seed + 7, latent, noise)
        self.G = sd.gaussian_matrix(D, seed + 2)
        if nlist == 1:
            self.cent = self.x.mean(axis=0, dtype=np.float64)[None, :].astype(np.float32)
            self.assign = np.zeros(n, dtype=np.int32)
        elif not kmeans:
            # row i in list i mod nlist; centres are the list means
            self.assign = (np.arange(n) % nlist).astype(np.int32)
            sums = np.zeros((nlist, D))
            np.add.at(sums, self.assign, self.x.astype(np.float64))
            self.cent = (sums / np.bincount(self.assign, minlength=nlist)[:, None]).astype(np.float32)
        else:
            self.cent, self.assign = sd.clustering(self.x, nlist, seed + 3, iters=kmeans_iters)
        # oracle side
        self.P64 = oracle.make_rotation(self.G)
        self.xr = oracle.rotate(self.x, self.P64)
        self.qr = oracle.rotate(self.q, self.P64)
        self.cr = oracle.rotate(self.cent, self.P64)
        self.off, self.members = oracle.lists_from_assignment(self.assign, nlist)

    def gt(self, K: int):
        return oracle.brute_knn(self.x, self.q, K)

    def oracle_probes(self, nprobe: int):
        return oracle.probes(self.qr, self.cr, nprobe)

    def exact(self, ids):
        """Exact raw-space distances of returned ids (inf for padding)."""
        out = np.full(ids.shape, np.inf)
        for i in range(ids.shape[0]):
            v = ids[i] >= 0
            out[i][v] = oracle.exact_dist(self.x[ids[i][v]], self.q[i])
        return out

    def oracle_search(self, probes, K, eps0, delta_d, method=oracle.METHOD_ADS, nprobe=None):
        return oracle.ivf_search(self.xr, self.qr, self.off, self.members, probes, K, eps0,
                                 delta_d, method=method, nprobe=nprobe)


def tie_band_equal(ids_a, d_a, ids_b, d_b, rel=1e-5):
    """True if two ascending top-K lists agree outside the tie band at the K-th
    distance: ids strictly below (1 - rel) * kth must match as sets, and the
    distances must agree rank by rank within rel."""
    ka = ids_a[ids_a >= 0]
    kb = ids_b[ids_b >= 0]
    if len(ka) != len(kb):
        return False
    if len(ka) == 0:
        return True
    kth = max(d_a[len(ka) - 1], d_b[len(kb) - 1])
    sa = set(ka[d_a[:len(ka)] < kth * (1 - rel)].tolist())
    sb = set(kb[d_b[:len(kb)] < kth * (1 - rel)].tolist())
    if sa != sb:
        return False
    return bool(np.all(np.abs(d_a[:len(ka)] - d_b[:len(kb)]) <= rel * np.maximum(d_b[:len(kb)], 1e-30)))


def probe_band(q_rot: np.ndarray, c_rot: np.ndarray, d2: np.ndarray) -> np.ndarray:
    """Per-centre rounding band (absolute, on squared distance) of the GPU's
    probe keys against the FP64 oracle's, for one query.

    The GPU rotates q and the centres in FP32 (each rotated vector is off by
    about sqrt(D) u |x| in norm, u = 2^-24, for rounding errors of random
    sign), which moves a squared distance by up to 2 dis (|dq| + |dc|); it then
    scores in the GEMM form |q|^2 + |c|^2 - 2 q.c with FP32 sums of D terms,
    whose rounding is about sqrt(D) u (|q| + |c|)^2.  The band is four times
    the sum of both (four standard deviations).
    """
    D = q_rot.shape[0]
    u = 2.0 ** -24
    qn = float(np.linalg.norm(q_rot))
    cn = np.linalg.norm(c_rot, axis=1)
    s = qn + cn
    return 4.0 * math.sqrt(D) * u * (s * s + 2.0 * np.sqrt(np.maximum(d2, 0.0)) * s)


def probes_agree(probes_gpu: np.ndarray, probes_orc: np.ndarray, q_rot: np.ndarray,
                 c_rot: np.ndarray, d2: np.ndarray) -> bool:
    """Checks one query's probe list against the oracle's.  Returns True when
    they are identical; otherwise asserts that every centre in one list but not
    the other lies within the rounding band of the oracle's nprobe-th squared
    distance (both bands added), and returns False."""
    g = [int(v) for v in probes_gpu if v >= 0]
    o = [int(v) for v in probes_orc if v >= 0]
    if g == o:
        return True
    band = probe_band(q_rot, c_rot, d2)
    kth_id = o[-1]
    kth = d2[kth_id]
    near = np.abs(d2 - kth) <= band + band[kth_id]
    diff = set(g) ^ set(o)
    outside = [j for j in diff if not near[j]]
    assert not outside, f"probe lists differ outside the rounding band: {outside[:5]}"
    return False
