"""Autotuner for the ADSampling-IVF search on one GPU.

Picks the stored block width delta_d (which fixes the index layout) and the
scan's scheduling knobs (queries per unit, dense-phase switch fraction, sweep
growth, persistent grid per XCD) for a workload shape, subject to a recall
constraint, and caches the choice per shape key.

The recall constraint is relative to FDScanning on the same index and probes:
the tuned ADSampling search may lose at most ``max_recall_loss`` of the
FDScanning result's neighbours (the paper's claim that ADSampling keeps the
KNN of the generated candidates with high probability, Corollary 4.2).
Everything is measured with the library itself; nothing here calls the
test oracle.

Search strategy: coordinate descent over the knobs (two passes), started
from the library defaults, for each delta_d candidate; the median of a few
timed searches decides.
"""

from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import _binding as B

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ads_mi355x", "tune.json")

KNOB_CHOICES = {
    "queries_per_unit": [4, 8, 16],
    "dense_frac": [0.0625, 0.125, 0.25],
    "sweep_log2": [3, 4, 5],
    "grid_per_xcd": [0, 512, 2048],
}


def shape_key(D: int, storage: int, k_max: int, nprobe_max: int, nq: int) -> str:
    """Cache key: dimensionality, storage type, K, and power-of-two bands of
    nprobe and of the batch size."""
    band = lambda v: 1 << max(0, int(math.floor(math.log2(max(1, v)))))  # noqa: E731
    return f"D{D}_s{storage}_K{k_max}_np{band(nprobe_max)}_nq{band(nq)}"


def coordinate_descent(evaluate, start: dict, choices: dict, passes: int = 2):
    """Minimise evaluate(config) -> cost (None = infeasible) one knob at a time.

    Returns (best config, best cost, number of evaluations)."""
    best = dict(start)
    best_cost = evaluate(best)
    n_eval = 1
    seen = {json.dumps(best, sort_keys=True): best_cost}
    for _ in range(passes):
        improved = False
        for knob, values in choices.items():
            for v in values:
                if best.get(knob) == v:
                    continue
                cand = dict(best)
                cand[knob] = v
                key = json.dumps(cand, sort_keys=True)
                if key in seen:
                    cost = seen[key]
                else:
                    cost = evaluate(cand)
                    seen[key] = cost
                    n_eval += 1
                if cost is not None and (best_cost is None or cost < best_cost):
                    best, best_cost, improved = cand, cost, True
        if not improved:
            break
    return best, best_cost, n_eval


@dataclass
class TuneResult:
    key: str
    delta_d: int
    knobs: dict
    ms: float
    recall_vs_fds: float
    evaluations: int
    trials: list = field(default_factory=list)

    def as_dict(self) -> dict:
        return {"key": self.key, "delta_d": self.delta_d, "knobs": self.knobs, "ms": self.ms,
                "recall_vs_fds": self.recall_vs_fds, "evaluations": self.evaluations}


class Autotuner:
    def __init__(self, cache_path: str | None = None):
        self.cache_path = cache_path or os.environ.get("ADS_TUNE_CACHE", DEFAULT_CACHE)
        self.cache = self._read()

    def _read(self) -> dict:
        try:
            with open(self.cache_path) as fh:
                return json.load(fh)
        except (OSError, ValueError):
            return {}

    def _write(self) -> None:
        d = os.path.dirname(self.cache_path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    def lookup(self, key: str):
        return self.cache.get(key)

    def apply(self, entry: dict) -> None:
        """Set the calling thread's scan knobs from a cached entry."""
        B.set_tuning(**entry["knobs"])

    def tune(self, base, P, centroids, assign, queries, k_max: int, nprobe_max: int,
             K=None, nprobe=None, eps0: float = 2.1, storage: int = B.F32,
             delta_d_choices=(16, 32, 64), max_recall_loss: float = 0.002, reps: int = 3,
             choices: dict | None = None, force: bool = False, log=None):
        """Tune for this workload; returns (TuneResult, index built with the best delta_d)."""
        import torch
        D = int(base.shape[1])
        nq = int(queries.shape[0])
        key = shape_key(D, storage, k_max, nprobe_max, nq)
        choices = choices or KNOB_CHOICES
        rerank = 0 if storage == B.F32 else 1
        qd = B._dev(queries, torch.float32)
        Kt = B._dev(K, torch.int32) if K is not None else None
        Nt = B._dev(nprobe, torch.int32) if nprobe is not None else None
        saved = B.get_tuning()
        best_overall = None
        trials = []
        try:
            for dd in delta_d_choices:
                if D % dd:
                    continue
                ix = B.ivf_build(base, P, centroids, assign, delta_d=dd, storage=storage,
                                 keep_fp32=bool(rerank))
                ref_ids, _ = B.search(ix, qd, k_max, nprobe_max, eps0=math.inf, K=Kt, nprobe=Nt,
                                      rerank=rerank)
                ref = ref_ids.cpu().numpy()
                n_ref = max(1, int(np.count_nonzero(ref >= 0)))

                def evaluate(cfg):
                    B.set_tuning(**cfg)
                    ids, _ = B.search(ix, qd, k_max, nprobe_max, eps0=eps0, K=Kt, nprobe=Nt,
                                      rerank=rerank)
                    got = ids.cpu().numpy()
                    hit = sum(len(set(r[r >= 0].tolist()) & set(g[g >= 0].tolist()))
                              for r, g in zip(ref, got))
                    rec = hit / n_ref
                    ts = []
                    for _ in range(reps):
                        torch.cuda.synchronize()
                        t = time.perf_counter()
                        B.search(ix, qd, k_max, nprobe_max, eps0=eps0, K=Kt, nprobe=Nt, rerank=rerank)
                        torch.cuda.synchronize()
                        ts.append((time.perf_counter() - t) * 1e3)
                    ms = float(np.median(ts))
                    trials.append({"delta_d": dd, **cfg, "ms": round(ms, 4), "recall_vs_fds": rec})
                    if log:
                        log(f"autotune dd={dd} {cfg} {ms:.3f} ms recall/fds {rec:.4f}")
                    return ms if rec >= 1.0 - max_recall_loss else None

                start = {k: saved[k] for k in choices}
                cfg, ms, n_eval = coordinate_descent(evaluate, start, choices)
                if ms is not None and (best_overall is None or ms < best_overall[2]):
                    if best_overall is not None:
                        best_overall[3].free()
                    rec = [t for t in trials if t["delta_d"] == dd and all(t[k] == cfg[k] for k in cfg)]
                    best_overall = (dd, cfg, ms, ix, rec[-1]["recall_vs_fds"] if rec else 1.0, n_eval)
                else:
                    ix.free()
        finally:
            B.set_tuning(**saved)
        if best_overall is None:
            raise RuntimeError("no configuration met the recall constraint")
        dd, cfg, ms, ix, rec, n_eval = best_overall
        res = TuneResult(key, dd, cfg, round(ms, 4), rec, n_eval, trials)
        if force or key not in self.cache or self.cache[key]["ms"] > res.ms:
            self.cache[key] = res.as_dict()
            self._write()
        return res, ix
