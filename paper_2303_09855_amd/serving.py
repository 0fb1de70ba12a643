"""Continuous-batching request loop for the ADSampling-IVF search.

Requests (one query each, with its own K and nprobe) arrive over time.  The
loop admits waiting requests into a batch whenever a stream slot is free and
the batch's device memory (workspace + buffers) fits in the HBM budget next to
the batches already in flight; several batches run concurrently on separate
streams (default priority), so requests that arrive while others are on the
GPU start as soon as a slot and memory free up.  The index stays resident.

A query's result does not depend on the other queries of its batch (the
search is batch independent), so a request gets the same answer alone and in
the mix.  Requests wait in one queue per K class (K rounded up to a power of
two): a batch's KNN-set capacity follows its largest K, so mixing K = 10 with
K = 100 would run the K = 10 requests with 100-entry sets and fewer queries
per scan unit.  The class whose oldest request arrived first is served next.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass

import numpy as np

from . import _binding as B


@dataclass
class Request:
    rid: int
    q: np.ndarray
    K: int
    nprobe: int
    t_arrival: float          # seconds from the start of the run


class AdmissionController:
    """Chooses how many waiting requests to launch now.

    Host logic only: the caller supplies the byte cost of a batch of n
    requests and the bytes already held by in-flight batches."""

    def __init__(self, budget_bytes: int, max_batch: int = 512, max_inflight: int = 2):
        if budget_bytes <= 0 or max_batch < 1 or max_inflight < 1:
            raise ValueError("budget, max_batch and max_inflight must be positive")
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight)

    def admit(self, n_waiting: int, n_inflight: int, inflight_bytes: int, batch_bytes) -> int:
        """Largest n <= min(max_batch, n_waiting) whose batch fits, else 0."""
        if n_waiting <= 0 or n_inflight >= self.max_inflight:
            return 0
        room = self.budget - inflight_bytes
        n = min(self.max_batch, n_waiting)
        if batch_bytes(n) <= room:
            return n
        lo, hi = 0, n                       # bytes grow with n: binary search
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if batch_bytes(mid) <= room:
                lo = mid
            else:
                hi = mid - 1
        return lo


class _Batch:
    def __init__(self, reqs, stream, ws, q, K, nprobe, ids, dist, h_ids, h_dist, event, nbytes):
        self.reqs, self.stream, self.ws = reqs, stream, ws
        self.q, self.K, self.nprobe, self.ids, self.dist = q, K, nprobe, ids, dist
        self.h_ids, self.h_dist, self.event, self.nbytes = h_ids, h_dist, event, nbytes


class Server:
    def __init__(self, index: B.Index, k_max: int, nprobe_max: int, eps0: float = 2.1,
                 max_batch: int = 512, n_streams: int = 2, hbm_budget: int | None = None,
                 rerank: int = 0):
        import torch
        self.torch = torch
        self.index = index
        self.D = index.info()["D"]
        self.k_max, self.nprobe_max, self.eps0, self.rerank = k_max, nprobe_max, eps0, rerank
        free, _ = torch.cuda.mem_get_info()
        budget = int(free * 0.8) if hbm_budget is None else int(hbm_budget)
        self.admission = AdmissionController(budget, max_batch, n_streams)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]

    def batch_bytes(self, n: int, k_max: int | None = None, nprobe_max: int | None = None) -> int:
        if n <= 0:
            return 0
        k_max = self.k_max if k_max is None else k_max
        nprobe_max = self.nprobe_max if nprobe_max is None else nprobe_max
        ws = B.search_workspace_size(self.index, n, k_max, nprobe_max, self.rerank)
        return ws + 256 + n * (self.D * 4 + 8 + k_max * 12)

    @staticmethod
    def k_class(K: int) -> int:
        c = 1
        while c < K:
            c *= 2
        return c

    def _launch(self, reqs, stream):
        torch = self.torch
        n = len(reqs)
        k_max = max(r.K for r in reqs)
        np_max = max(r.nprobe for r in reqs)
        nbytes = self.batch_bytes(n, k_max, np_max)
        with torch.cuda.stream(stream):
            hq = torch.from_numpy(np.stack([r.q for r in reqs]).astype(np.float32)).pin_memory()
            hk = torch.tensor([r.K for r in reqs], dtype=torch.int32).pin_memory()
            hp = torch.tensor([r.nprobe for r in reqs], dtype=torch.int32).pin_memory()
            q = hq.to("cuda", non_blocking=True)
            K = hk.to("cuda", non_blocking=True)
            npb = hp.to("cuda", non_blocking=True)
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            off = (-ws.data_ptr()) % 256
            ids = torch.empty((n, k_max), dtype=torch.int64, device="cuda")
            dist = torch.empty((n, k_max), dtype=torch.float32, device="cuda")
            B._check(B.load().ads_search(
                self.index.handle, B._ptr(q), n, B._ptr(K), B._ptr(npb), k_max, np_max,
                float(self.eps0), B.ADSAMPLING, self.rerank, B._ptr(ids), B._ptr(dist), None, None,
                B.ctypes.c_void_p(ws.data_ptr() + off), B.ctypes.c_void_p(stream.cuda_stream)))
            h_ids = torch.empty((n, k_max), dtype=torch.int64).pin_memory()
            h_dist = torch.empty((n, k_max), dtype=torch.float32).pin_memory()
            h_ids.copy_(ids, non_blocking=True)
            h_dist.copy_(dist, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return _Batch(reqs, stream, ws, q, K, npb, ids, dist, h_ids, h_dist, ev, nbytes)

    def run(self, requests, realtime: bool = True, poll_s: float = 20e-6):
        """Serve requests (sorted by arrival).  Returns (results {rid: (ids, dist)},
        latencies {rid: seconds}, stats)."""
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        for r in pending:
            if not (1 <= r.K <= self.k_max and 1 <= r.nprobe <= self.nprobe_max):
                raise ValueError(f"request {r.rid}: K and nprobe must be in [1, k_max] and [1, nprobe_max]")
        waiting = collections.OrderedDict()     # K class -> deque of requests
        inflight = []
        free_streams = list(self.streams)
        results, lat = {}, {}
        batches = 0
        t0 = time.perf_counter()
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].t_arrival <= now):
                r = pending.popleft()
                waiting.setdefault(self.k_class(r.K), collections.deque()).append(r)
            done = [b for b in inflight if b.event.query()]
            if done:
                t_done = time.perf_counter() - t0
                for b in done:
                    inflight.remove(b)
                    free_streams.append(b.stream)
                    for i, r in enumerate(b.reqs):
                        k = r.K
                        results[r.rid] = (b.h_ids[i, :k].numpy().copy(), b.h_dist[i, :k].numpy().copy())
                        lat[r.rid] = t_done - r.t_arrival if realtime else t_done
            if waiting and free_streams:
                cls = min(waiting, key=lambda c: waiting[c][0].t_arrival)
                queue = waiting[cls]
                k_cls = min(cls, self.k_max)
                n = self.admission.admit(len(queue), len(inflight), sum(b.nbytes for b in inflight),
                                         lambda m: self.batch_bytes(m, k_cls))
                if n > 0:
                    reqs = [queue.popleft() for _ in range(n)]
                    if not queue:
                        del waiting[cls]
                    inflight.append(self._launch(reqs, free_streams.pop()))
                    batches += 1
                    continue
            if not done:
                time.sleep(poll_s)
        el = time.perf_counter() - t0
        lv = np.array([lat[r.rid] for r in requests])
        stats = {"requests": len(requests), "batches": batches, "seconds": el,
                 "qps": len(requests) / el if el > 0 else float("inf"),
                 "p50_ms": float(np.percentile(lv, 50) * 1e3) if len(lv) else 0.0,
                 "p99_ms": float(np.percentile(lv, 99) * 1e3) if len(lv) else 0.0}
        return results, lat, stats
