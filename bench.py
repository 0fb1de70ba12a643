#!/usr/bin/env python3
"""Benchmark: ADSampling-IVF vs FDScanning-IVF on one MI355X.

Metric: QPS at recall@10 >= 0.95 (end to end: query rotation, probe
selection, scan, merges, output), DCOs/s, and the roofline fraction of the
scan kernel.  A step is one search of the whole query batch with the inputs
already resident in HBM.  Prints ONE JSON line on stdout; progress on stderr.

Workload (default ivf_d960): N = 1,000,000 synthetic low-rank vectors of
D = 960 (x = zW + 0.1 noise, z ~ N(0, I_64)), 1,000 queries from the same
model, 4,096 lists, K = 10, delta_d = 16, eps0 = 2.1, float32 storage.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz: the FP32 vector rate
# without packed FP32 instructions (which this library does not emit); the
# published 157.3 TFLOP/s counts packed FP32.
FP32_VALU_PEAK_TFLOPS = 78.6

# operating-point search: the smallest grid nprobe that reaches the recall target
# (steps of 1/8 between 512 and 1024)
NPROBE_GRID = [8, 16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 576, 640, 704, 768, 896, 1024, 1536, 2048,
               3072, 4096]
NPROBE_LIMIT = 4096            # the library's largest nprobe_max


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ivf_d960")
    ap.add_argument("--nq", type=int, default=None, help="override the number of queries")
    ap.add_argument("--n", type=int, default=None, help="override the number of base vectors")
    ap.add_argument("--target-recall", type=float, default=0.95)
    ap.add_argument("--K", type=int, default=10)
    ap.add_argument("--eps0", type=float, default=2.1)
    ap.add_argument("--delta-d", type=int, default=16)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fds", action="store_true")
    ap.add_argument("--no-pds", action="store_true",
                    help="skip the PDScanning leg (IVF** on an unrotated index)")
    ap.add_argument("--mode", default="search", choices=["search", "serve", "verify", "batched", "hnsw"],
                    help="search: the throughput benchmark (default); serve: the continuous-"
                         "batching request loop at Poisson arrival rates; verify: the fixed-"
                         "threshold failure-rate / dims sweep over eps0 and the linear-scan "
                         "feasibility run; batched: one captured search per batch with "
                         "per-query K in {10, 100} and nprobe uniform on [8, 128]; hnsw: graph "
                         "search (HNSW, HNSW+, HNSW++) on the workload's vectors")
    ap.add_argument("--verify-queries", type=int, default=20, help="verify mode: queries")
    ap.add_argument("--verify-n", type=int, default=200_000,
                    help="verify mode: base vectors of the linear scans (the first n of the workload)")
    ap.add_argument("--rates", default="5000,20000,50000", help="serve mode: arrivals per second")
    ap.add_argument("--serve-requests", type=int, default=20000, help="serve mode: requests per rate")
    ap.add_argument("--serve-nprobe", default="32,64",
                    help="serve mode: per-request nprobe drawn uniformly from this list")
    ap.add_argument("--max-batch", type=int, default=512, help="serve mode: largest batch")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device-to-device copy first (reference kernel "
                         "of known size for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--hnsw-m", type=int, default=16, help="hnsw mode: M (2M on layer 0)")
    ap.add_argument("--nef", type=int, default=None,
                    help="hnsw mode: use this N_ef for every variant instead of searching")
    ap.add_argument("--tune", default="",
                    help="scan scheduling knobs, e.g. sweep_log2=4,dense_frac=0.25 (ads_tuning fields)")
    ap.add_argument("--nprobe", type=int, default=None,
                    help="use this nprobe for both methods instead of searching for the "
                         "smallest one that reaches the target recall")
    return ap.parse_args()


def exact_for(x, q, ids):
    import oracle
    out = np.full(ids.shape, np.inf)
    for i in range(ids.shape[0]):
        v = ids[i] >= 0
        if v.any():
            out[i][v] = oracle.exact_dist(x[ids[i][v]], q[i])
    return out


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design, not a measured configuration.", file=sys.stderr)
        return 2
    import torch

    import oracle
    import paper_2303_09855_amd as ads
    import synthdata as sd

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    ads.load()
    knobs = {}
    for kv in filter(None, args.tune.split(",")):
        k, v = kv.split("=")
        knobs[k.strip()] = float(v) if k.strip() == "dense_frac" else int(v)
    ads.set_tuning(**knobs)
    w = sd.WORKLOADS[args.workload]
    if args.nq or args.n:
        w = w.scaled(nq=args.nq or w.nq, n=args.n or w.n)
    K = args.K
    storage = {"f32": ads.F32, "bf16": ads.BF16, "f16": ads.F16}[args.storage]
    rerank = 0 if storage == ads.F32 else 1

    t0 = time.time()
    x = sd.base_vectors(w)
    q = sd.query_vectors(w)
    G = sd.rotation_gaussian(w)
    log(f"data {w.n}x{w.D} + {w.nq} queries in {time.time() - t0:.1f}s")
    t0 = time.time()
    cent, assign = sd.ivf_clustering(w, x)
    log(f"clustering into {w.nlist} lists in {time.time() - t0:.1f}s")
    t0 = time.time()
    _, gt = oracle.brute_knn(x, q, K)
    log(f"exact ground truth in {time.time() - t0:.1f}s")

    t0 = time.time()
    P32, _ = ads.make_rotation(G)
    ix = ads.ivf_build(x, P32, cent, assign, delta_d=args.delta_d, storage=storage,
                       keep_fp32=bool(rerank))
    torch.cuda.synchronize()
    info = ix.info()
    log(f"index built in {time.time() - t0:.1f}s ({info['device_bytes'] / 1e9:.2f} GB, "
        f"max list {info['max_list']})")
    qd = torch.as_tensor(q).cuda()
    if args.calibrate_copy:
        src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 1 GiB read + 1 GiB written")

    def run(nprobe, eps0, stats=None, index=None, method=ads.ADSAMPLING):
        ids, dist = ads.search(index or ix, qd, K, nprobe, eps0=eps0, rerank=rerank, stats=stats,
                               method=method)
        return ids, dist

    last_ids = {}

    def recall_at(nprobe, eps0):
        ids, _ = run(nprobe, eps0)
        torch.cuda.synchronize()
        ids = ids.cpu().numpy()
        last_ids[eps0] = ids
        return oracle.recall(ids, exact_for(x, q, ids), gt, K)

    def operating_point(eps0, label):
        if args.nprobe:
            r = recall_at(args.nprobe, eps0)
            log(f"{label}: nprobe {args.nprobe:5d} recall@{K} {r:.4f} (fixed)")
            return args.nprobe, r
        top = min(w.nlist, NPROBE_LIMIT)
        grid = [p for p in NPROBE_GRID if p < top] + [top]
        best = None
        for p in grid:
            r = recall_at(p, eps0)
            log(f"{label}: nprobe {p:5d} recall@{K} {r:.4f}")
            best = (p, r)
            if r >= args.target_recall:
                break
        return best

    def timed(nprobe, eps0, label, **kw):
        for _ in range(args.warmup):
            run(nprobe, eps0, **kw)
        stats = torch.zeros(ads.NSTATS, dtype=torch.int64, device="cuda")
        run(nprobe, eps0, stats, **kw)
        torch.cuda.synchronize()
        st = stats.cpu().numpy()
        ads.profile_enable(True)
        ads.profile_collect()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            run(nprobe, eps0, **kw)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        ads.profile_enable(False)
        ph = ads.profile_collect()
        ms = el * 1e3 / args.steps
        log(f"{label}: nprobe {nprobe} {ms:.3f} ms/step, {w.nq / (ms / 1e3):.0f} QPS, "
            f"scan {ph['scan'][0] / args.steps:.3f} ms/step")
        return ms, st, ph

    if args.mode == "serve":
        return serve(args, w, ix, q, gt, x)
    if args.mode == "batched":
        return batched(args, w, ix, q, x)
    if args.mode == "verify":
        ix.free()
        return verify(args, w, x, q, G)
    if args.mode == "hnsw":
        ix.free()
        return hnsw(args, w, x, q, G, gt)

    p_ads, r_ads = operating_point(args.eps0, "ADSampling")
    ids_ads = last_ids[args.eps0]
    ms_ads, st_ads, ph_ads = timed(p_ads, args.eps0, "ADSampling")
    fds = None
    if not args.no_fds:
        p_fds, r_fds = operating_point(math.inf, "FDScanning")
        ms_fds, st_fds, ph_fds = timed(p_fds, math.inf, "FDScanning")
        fds = {"nprobe": p_fds, "recall": round(r_fds, 4), "ms_per_step": round(ms_fds, 4),
               "qps": round(w.nq / (ms_fds / 1e3), 1),
               "dcos_per_s": round(float(st_fds[ads.STAT_DCOS]) / (ms_fds / 1e3), 1),
               "scan_ms_per_step": round(ph_fds["scan"][0] / args.steps, 4)}

    pds = None
    if not args.no_pds and storage == ads.F32:
        # IVF** (Section 6.1): PDScanning on the original coordinates, same lists,
        # an index built without the rotation, at the ADSampling operating point
        ix_raw = ads.ivf_build(x, None, cent, assign, delta_d=args.delta_d, storage=ads.F32,
                               keep_fp32=False)
        torch.cuda.synchronize()
        p_ids, _ = run(p_ads, math.inf, index=ix_raw, method=ads.PDSCANNING)
        torch.cuda.synchronize()
        p_ids = p_ids.cpu().numpy()
        r_pds = oracle.recall(p_ids, exact_for(x, q, p_ids), gt, K)
        ms_pds, st_pds, ph_pds = timed(p_ads, math.inf, "PDScanning (unrotated)", index=ix_raw,
                                       method=ads.PDSCANNING)
        pds = {"nprobe": p_ads, "recall": round(r_pds, 4), "ms_per_step": round(ms_pds, 4),
               "qps": round(w.nq / (ms_pds / 1e3), 1),
               "dims_ratio": round(float(st_pds[ads.STAT_DIMS]) / max(1.0, float(st_pds[ads.STAT_DCOS]) * w.D), 5),
               "dcos_per_s": round(float(st_pds[ads.STAT_DCOS]) / (ms_pds / 1e3), 1),
               "scan_ms_per_step": round(ph_pds["scan"][0] / args.steps, 4)}
        ix_raw.free()

    qps = w.nq / (ms_ads / 1e3)
    dcos = float(st_ads[ads.STAT_DCOS])
    dims = float(st_ads[ads.STAT_DIMS])
    alg_bytes = float(st_ads[ads.STAT_BYTES])
    scan_ms, scan_launches = ph_ads["scan"]
    scan_ms_step = scan_ms / args.steps
    launches_per_step = scan_launches / args.steps
    avg_launch_ms = scan_ms / max(1, scan_launches)
    bytes_per_launch = alg_bytes / max(1.0, launches_per_step)
    achieved_gbs = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    flops = 3.0 * dims  # one subtract and one fused multiply-add per sampled coordinate
    achieved_tflops = flops / (scan_ms_step * 1e-3) / 1e12
    scan_kernel = "scan_kernel"
    traffic = scan_traffic_from_profile(
        scan_kernel, profiled_config(w, p_ads, K, args.delta_d, args.eps0, args.storage, args.tune))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, x, q, G, cent, assign, p_ads, K, args, gt=gt, gpu_ids=ids_ads)

    out = {
        "metric": "QPS @ recall@10>=0.95 and DCOs/s vs FDScanning, same GPU; % HBM roofline",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_ads, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if storage == ads.F32 else args.storage,
        "data": "synthetic",
        "config": {"workload": f"{w.name}: N={w.n}, D={w.D}, {w.model} model, {w.nq} queries, "
                               f"nlist={w.nlist}, K={K}, delta_d={args.delta_d}, eps0={args.eps0}, "
                               f"storage={args.storage}",
                   "nprobe": p_ads, "recall_at_10": round(r_ads, 4), "global_batch": w.nq,
                   "parallelism": "single GPU"},
        "dcos_per_s": round(dcos / (ms_ads / 1e3), 1),
        "dims_ratio": round(dims / max(1.0, dcos * w.D), 5),
        "speedup_vs_fdscanning": round(fds["ms_per_step"] / ms_ads, 3) if fds else None,
        "fdscanning": fds,
        "pdscanning_unrotated": pds,
        "speedup_vs_pdscanning": round(pds["ms_per_step"] / ms_ads, 3) if pds else None,
        "phase_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in ph_ads.items()},
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3),
                     "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tflops / FP32_VALU_PEAK_TFLOPS, 4),
                     "traffic": traffic, "kernel": scan_kernel,
                     "avg_launch_ms": round(avg_launch_ms, 4),
                     "launches_per_step": launches_per_step,
                     "alg_flops_per_launch": round(flops / max(1.0, launches_per_step), 1)},
        "roofline_hbm_algorithmic": {"bound": "hbm", "achieved": round(achieved_gbs, 1),
                                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                                     "alg_bytes_per_launch": round(bytes_per_launch, 1),
                                     "note": "bytes the DCOs need (sampled dims x 4 B); a list "
                                             "tile is fetched once and reused by its queries, so "
                                             "this exceeds the HBM traffic"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ix.free()
    return 0


def serve(args, w, ix, q, gt, x):
    """Continuous-batching loop at each arrival rate; one JSON line."""
    import oracle
    import synthdata as sd
    from paper_2303_09855_amd.serving import Request, Server
    rng = np.random.default_rng(1048)
    nps = [int(v) for v in args.serve_nprobe.split(",")]
    out = []
    for rate in [float(v) for v in args.rates.split(",")]:
        n = args.serve_requests
        t = sd.poisson_arrivals(rate, n, seed=1047)
        qi = np.arange(n) % w.nq
        Ks = rng.choice([10, 100], size=n)
        Ps = rng.choice(nps, size=n)
        reqs = [Request(i, q[qi[i]], int(Ks[i]), int(Ps[i]), float(t[i])) for i in range(n)]
        srv = Server(ix, k_max=100, nprobe_max=max(nps), eps0=args.eps0, max_batch=args.max_batch, n_streams=3)
        res, lat, st = srv.run(reqs)
        # recall@10 of the first 10 results of every request against the exact top-10
        ids = np.stack([np.pad(res[i][0][:10], (0, max(0, 10 - len(res[i][0][:10]))),
                               constant_values=-1) for i in range(n)])
        rec = oracle.recall(ids, np.stack([exact_for(x, q[qi[i]:qi[i] + 1], ids[i:i + 1])[0]
                                           for i in range(n)]), gt[qi], 10)
        log(f"serve rate {rate:.0f}/s: {st['qps']:.0f} QPS, p50 {st['p50_ms']:.2f} ms, "
            f"p99 {st['p99_ms']:.2f} ms, {st['batches']} batches, recall@10 {rec:.4f}")
        out.append({"rate": rate, "qps": round(st["qps"], 1), "p50_ms": round(st["p50_ms"], 3),
                    "p99_ms": round(st["p99_ms"], 3), "batches": st["batches"],
                    "recall_at_10": round(rec, 4)})
    line = {"metric": "serving latency at Poisson arrival rates (p50/p99) and QPS",
            "value": out[-1]["qps"], "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{w.name} index, requests cycle its {w.nq} queries, "
                                   f"K in {{10,100}} (one queue per K class), nprobe in {nps}, "
                                   f"batches <= {args.max_batch}, 3 streams"},
            "rates": out}
    print(json.dumps(line), flush=True)
    ix.free()
    return 0


def batched(args, w, ix, q, x):
    """One HIP-graph launch per batch of uneven queries: per-query K in {10, 100}
    and nprobe uniform on [8, 128] (ADSampling, the same eps0); QPS of graph
    replays and of the eager call, recall@K against the exact K nearest."""
    import torch

    import oracle
    import paper_2303_09855_amd as ads
    import synthdata as sd
    Ks, Ps = sd.uneven_draws(w)
    kmax, pmax = int(Ks.max()), int(Ps.max())
    _, gt = oracle.brute_knn(x, q, kmax)
    plan = ads.Plan(ix, w.nq, kmax, pmax, eps0=args.eps0)
    plan.q.copy_(torch.as_tensor(q))
    plan.K.copy_(torch.as_tensor(Ks))
    plan.nprobe.copy_(torch.as_tensor(Ps))
    torch.cuda.synchronize()
    plan.launch()
    torch.cuda.synchronize()
    ids = plan.ids.cpu().numpy()
    ex = exact_for(x, q, ids)
    rec = oracle.recall(ids, ex, gt, Ks)
    qd = torch.as_tensor(q).cuda()
    Kd, Pd = torch.as_tensor(Ks).cuda(), torch.as_tensor(Ps).cuda()

    def clock(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps

    ms_graph = clock(plan.launch)
    ms_eager = clock(lambda: ads.search(ix, qd, kmax, pmax, eps0=args.eps0, K=Kd, nprobe=Pd))
    st = torch.zeros(ads.NSTATS, dtype=torch.int64, device="cuda")
    ads.search(ix, qd, kmax, pmax, eps0=args.eps0, K=Kd, nprobe=Pd, stats=st)
    torch.cuda.synchronize()
    stv = st.cpu().numpy()
    log(f"batched: graph {ms_graph:.3f} ms, eager {ms_eager:.3f} ms per {w.nq} queries, "
        f"recall {rec:.4f}")
    line = {"metric": "QPS of uneven batches (per-query K and nprobe), one graph launch per batch",
            "value": round(w.nq / (ms_graph / 1e3), 1), "unit": "queries/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_graph, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"{w.name}: N={w.n}, D={w.D}, {w.nq} queries, nlist={w.nlist}, "
                                   f"K in {{10,100}}, nprobe U[8,128], delta_d={args.delta_d}, "
                                   f"eps0={args.eps0}"},
            "eager_ms_per_step": round(ms_eager, 4), "recall_at_K": round(rec, 4),
            "dcos_per_s": round(float(stv[ads.STAT_DCOS]) / (ms_graph / 1e3), 1),
            "dims_ratio": round(float(stv[ads.STAT_DIMS]) / max(1.0, float(stv[ads.STAT_DCOS]) * w.D), 5)}
    print(json.dumps(line), flush=True)
    plan.free()
    ix.free()
    return 0


NEF_GRID = [10, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096]


def hnsw(args, w, x, q, G, gt):
    """Graph search on the workload's vectors: an HNSW-structured graph
    (M, 2M on layer 0) built once, then HNSW (full distances), HNSW+ and HNSW++
    (Sections 2.2.1, 4, 5.1), each at the smallest N_ef of NEF_GRID whose
    recall@K reaches the target; QPS, DCOs and sampled dims of each."""
    import torch

    import oracle
    import paper_2303_09855_amd as ads
    from synthdata.graph import hnsw_graph_torch
    K = args.K
    t0 = time.time()
    g = hnsw_graph_torch(x, M=args.hnsw_m, seed=w.kmeans_seed, progress=log)
    log(f"graph built in {time.time() - t0:.1f}s (levels 0..{g.max_level}, layer-0 degree "
        f"{(g.adj0 >= 0).sum(1).mean():.1f})")
    P32, _ = ads.make_rotation(G)
    ix = ads.hnsw_create(x, P32, g, delta_d=args.delta_d)
    qd = torch.as_tensor(q).cuda()
    torch.cuda.synchronize()

    def recall_of(nef, variant):
        ids, _ = ads.hnsw_search(ix, qd, K, nef, eps0=args.eps0, variant=variant)
        torch.cuda.synchronize()
        ids = ids.cpu().numpy()
        return oracle.recall(ids, exact_for(x, q, ids), gt, K), ids

    def operating_point(variant, label):
        grid = [args.nef] if args.nef else [v for v in NEF_GRID if v >= K] or [K]
        best = None
        for nef in grid:
            r, ids = recall_of(nef, variant)
            log(f"{label}: nef {nef:5d} recall@{K} {r:.4f}")
            best = (nef, r, ids)
            if r >= args.target_recall:
                break
        return best

    def timed(nef, variant, label):
        for _ in range(args.warmup):
            ads.hnsw_search(ix, qd, K, nef, eps0=args.eps0, variant=variant)
        st = torch.zeros(3, dtype=torch.int64, device="cuda")
        ads.hnsw_search(ix, qd, K, nef, eps0=args.eps0, variant=variant, stats=st)
        ws = torch.empty(ads.hnsw_workspace_size(ix, w.nq) + 256, dtype=torch.uint8, device="cuda")
        off = (-ws.data_ptr()) % 256
        wsv = ws[off:]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            ads.hnsw_search(ix, qd, K, nef, eps0=args.eps0, variant=variant, workspace=wsv)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / args.steps
        stv = st.cpu().numpy()
        log(f"{label}: nef {nef} {ms:.3f} ms/step, {w.nq / (ms / 1e3):.0f} QPS")
        return ms, stv

    rows = {}
    for variant, label in ((ads.HNSW_PLAIN, "HNSW"), (ads.HNSW_PLUS, "HNSW+"), (ads.HNSW_PP, "HNSW++")):
        nef, r, ids = operating_point(variant, label)
        ms, stv = timed(nef, variant, label)
        rows[label] = {"nef": nef, "recall": round(r, 4), "ms_per_step": round(ms, 4),
                       "qps": round(w.nq / (ms / 1e3), 1), "dcos_per_query": round(stv[0] / w.nq, 1),
                       "dims_ratio": round(float(stv[1]) / max(1.0, float(stv[0]) * w.D), 5),
                       "expansions_per_query": round(stv[2] / w.nq, 1),
                       "dcos_per_s": round(float(stv[0]) / (ms / 1e3), 1),
                       "dco_bytes_per_s": round(float(stv[1]) * 4 / (ms / 1e3), 1)}
    cpu = None
    if not args.no_cpu_baseline:
        nef = rows["HNSW++"]["nef"]
        P64 = oracle.make_rotation(G)
        xr = oracle.rotate(x, P64)
        nsamp = min(w.nq, 200)
        qr = oracle.rotate(q[:nsamp], P64)
        threads = min(16, os.cpu_count() or 1)
        t = time.perf_counter()
        o_ids, _, o_st = oracle.hnsw_search(xr, qr, g, K, nef, args.eps0, args.delta_d, oracle.HNSW_PP,
                                            threads=threads)
        el = time.perf_counter() - t
        t = time.perf_counter()
        oracle.hnsw_search(xr, qr[:20], g, K, nef, args.eps0, args.delta_d, oracle.HNSW_PP, threads=1)
        el1 = time.perf_counter() - t
        o_rec = oracle.recall(o_ids, exact_for(x, q[:nsamp], o_ids), gt[:nsamp], K)
        cpu = {"value": round(nsamp / el, 2), "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"HNSW++ at nef {nef} on the first {nsamp} queries (FP64); one thread: "
                         f"{round(20 / el1, 2)} queries/s on 20 queries",
               "oracle_recall": round(o_rec, 4)}
        del xr
    pp, plain, plus = rows["HNSW++"], rows["HNSW"], rows["HNSW+"]
    line = {"metric": "graph search QPS @ recall@10>=0.95: HNSW++ / HNSW+ vs HNSW, same GPU",
            "value": pp["qps"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": pp["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{w.name} vectors: N={w.n}, D={w.D}, {w.nq} queries; HNSW-structured "
                                   f"graph M={args.hnsw_m}; K={K}, delta_d={args.delta_d}, eps0={args.eps0}"},
            "hnsw": plain, "hnsw_plus": plus, "hnsw_pp": pp,
            "speedup_pp_vs_hnsw": round(plain["ms_per_step"] / pp["ms_per_step"], 3),
            "speedup_plus_vs_hnsw": round(plain["ms_per_step"] / plus["ms_per_step"], 3),
            "roofline": {"bound": "hbm", "achieved": round(pp["dco_bytes_per_s"] / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(pp["dco_bytes_per_s"] / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": None, "kernel": "hnsw_search_kernel",
                         "note": "sampled coordinates x 4 B per second (the bytes the DCOs need)"},
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)
    ix.free()
    return 0


def verify(args, w, x, q, G):
    """Section 6.2.6: a linear scan with the threshold fixed at the exact K-th
    NN distance, delta_d = 1, eps0 from 0 to 4: failure rate (true neighbours
    rejected) and evaluated dims.  Section 6.2.4 (Fig. 8 methodology): an exact
    KNN by linear scan (one list, sequential thresholds) with ADSampling DCOs,
    recall and evaluated dims per eps0 at delta_d 8 and 32."""
    import torch

    import oracle
    import paper_2303_09855_amd as ads
    n = min(args.verify_n, w.n)
    nq = min(args.verify_queries, w.nq)
    xs, qs = x[:n], q[:nq]
    K = args.K
    _, gt = oracle.brute_knn(xs, qs, K)
    P32, _ = ads.make_rotation(G)
    qrot = ads.rotate(P32, qs)
    eps_grid = [0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0]
    fixed = []
    ix = ads.ivf_build(xs, P32, xs.mean(axis=0, keepdims=True), np.zeros(n, dtype=np.int32),
                       delta_d=32 if w.D % 32 == 0 else 8, storage=ads.F32, keep_fp32=True)
    cand = torch.arange(n, dtype=torch.int64, device="cuda")
    for eps0 in eps_grid:
        fails = pos = 0
        dims = 0
        for i in range(nq):
            r = float(gt[i, K - 1])
            mask, _, dd = ads.dco_batch(ix, qrot[i], cand, r, eps0, 1)
            torch.cuda.synchronize()
            m = mask.cpu().numpy()
            raw = oracle.exact_dist(xs, qs[i])
            # true neighbours strictly inside r (objects tied with the K-th sit on the boundary)
            tp = raw < r * (1 - 1e-6)
            pos += int(tp.sum())
            fails += int(np.sum(tp & (m == 0)))
            dims += int(dd.sum().item())
        row = {"eps0": eps0, "failure_rate": round(fails / max(1, pos), 6),
               "dims_frac": round(dims / (n * nq * w.D), 5)}
        log(f"verify fixed r: eps0 {eps0}: failure rate {row['failure_rate']:.5f}, dims {row['dims_frac']:.4f}")
        fixed.append(row)
    ix.free()
    scans = []
    for dd_layout in (8, 32):
        if w.D % dd_layout:
            continue
        ixf = ads.ivf_build(xs, P32, xs.mean(axis=0, keepdims=True), np.zeros(n, dtype=np.int32),
                            delta_d=dd_layout, storage=ads.F32, keep_fp32=False)
        for eps0 in eps_grid[1:] + [math.inf]:
            st = torch.zeros(ads.NSTATS, dtype=torch.int64, device="cuda")
            ids, _ = ads.search(ixf, qs, K, 1, eps0=eps0, stats=st)
            torch.cuda.synchronize()
            ids = ids.cpu().numpy()
            stv = st.cpu().numpy()
            rec = oracle.recall(ids, exact_for(xs, qs, ids), gt, K)
            row = {"delta_d": dd_layout, "eps0": eps0 if math.isfinite(eps0) else "inf",
                   "recall": round(rec, 5),
                   "dims_ratio": round(float(stv[ads.STAT_DIMS]) / max(1.0, float(stv[ads.STAT_DCOS]) * w.D), 5)}
            log(f"verify linear scan: delta_d {dd_layout} eps0 {eps0}: recall {rec:.4f}, dims {row['dims_ratio']:.4f}")
            scans.append(row)
        ixf.free()
    best = {}
    for row in scans:
        if row["recall"] >= 0.999 and row["eps0"] != "inf":
            b = best.get(row["delta_d"])
            if b is None or row["dims_ratio"] < b["dims_ratio"]:
                best[row["delta_d"]] = row
    line = {"metric": "fixed-threshold failure rate and evaluated dims vs eps0; linear-scan dims at recall > 0.999",
            "value": fixed[4]["failure_rate"], "unit": "failure rate at eps0 = 2", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{w.name}: first {n} base vectors, {nq} queries, K={K}, D={w.D}"},
            "fixed_threshold_delta_d_1": fixed, "linear_scan": scans,
            "linear_scan_best_at_recall_0_999": best}
    print(json.dumps(line), flush=True)
    return 0


# Sources the scan kernels are compiled from (the counter summary records
# their digest; a changed kernel invalidates the traffic figure).
SCAN_SOURCES = {
    "scan_kernel": ["scan_kernel.h", "scan_sparse.h", "common.h", "kernels.h"],
}


def scan_source_sha(kernel: str = "scan_kernel") -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SCAN_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2303_09855_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def profiled_config(w, nprobe, K, delta_d, eps0, storage, tune) -> str:
    """The key naming the search configuration a counter summary was taken on."""
    return (f"{w.name} n={w.n} nq={w.nq} nprobe={nprobe} K={K} delta_d={delta_d} eps0={eps0} "
            f"storage={storage} tune={tune or '-'}")


def scan_traffic_from_profile(kernel: str = "scan_kernel", config: str = ""):
    """HBM bytes per scan launch from the committed counter summary, or None
    when the scan kernel sources changed since the counters were taken or the
    summary was taken on another search configuration."""
    prof = os.path.join(ROOT, "profiles", f"{kernel}_ivf_d960_counters.txt")
    try:
        sha = scan_source_sha(kernel)
        fields = {}
        for line in open(prof):
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        if fields.get("scan_source_sha256") != sha:
            return None
        if fields.get("profiled_config") != config:
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(w, x, q, G, cent, assign, nprobe, K, args, gt=None, gpu_ids=None):
    """The FP64 oracle's IVF+ search (as it stands) on a bounded query sample,
    on every host core and on one thread; with the oracle's recall on the
    sample next to the GPU's recall on the same queries."""
    import oracle
    t0 = time.time()
    P64 = oracle.make_rotation(G)
    qr = oracle.rotate(q, P64)
    cr = oracle.rotate(cent, P64)
    off, members = oracle.lists_from_assignment(assign, w.nlist)
    threads = os.cpu_count() or 1

    def sample_rows(m):
        pr, _ = oracle.probes(qr[:m], cr, nprobe)
        lists = np.unique(pr)
        rows = np.concatenate([members[off[l]:off[l + 1]] for l in lists])
        return pr, np.sort(rows)

    # calibrate on a few queries, then size the sample for the time budget
    m0 = min(w.nq, max(2, threads))
    pr0, rows0 = sample_rows(m0)
    row_of = np.full(w.n, -1, dtype=np.int64)
    row_of[rows0] = np.arange(len(rows0))
    xr = np.empty((len(rows0), w.D))
    for s in range(0, len(rows0), 65536):
        xr[s:s + 65536] = oracle.rotate(x[rows0[s:s + 65536]], P64)
    log(f"cpu baseline: rotated {len(rows0)} rows in {time.time() - t0:.1f}s")
    t = time.perf_counter()
    oracle.ivf_search(xr, qr[:m0], off, members, pr0, K, args.eps0, args.delta_d, threads=threads,
                      row_of_id=row_of)
    per_q = (time.perf_counter() - t) / m0
    m = int(min(w.nq, max(m0, args.cpu_seconds / max(per_q, 1e-6) * 1.0)))
    m = max(m0, (m // threads) * threads if m >= threads else m)
    pr, rows = sample_rows(m)
    if len(rows) > len(rows0):
        row_of = np.full(w.n, -1, dtype=np.int64)
        row_of[rows] = np.arange(len(rows))
        xr = np.empty((len(rows), w.D))
        for s in range(0, len(rows), 65536):
            xr[s:s + 65536] = oracle.rotate(x[rows[s:s + 65536]], P64)
    t = time.perf_counter()
    ids, dist, st = oracle.ivf_search(xr, qr[:m], off, members, pr, K, args.eps0, args.delta_d,
                                      threads=threads, row_of_id=row_of)
    el = time.perf_counter() - t
    log(f"cpu baseline: {m} queries in {el:.1f}s on {threads} threads")
    # one thread (the paper's setting): a sample sized for about a third of the budget
    m1 = int(max(1, min(m, args.cpu_seconds / 3.0 / max(per_q * threads, 1e-6))))
    t = time.perf_counter()
    oracle.ivf_search(xr, qr[:m1], off, members, pr[:m1], K, args.eps0, args.delta_d, threads=1,
                      row_of_id=row_of)
    el1 = time.perf_counter() - t
    log(f"cpu baseline: {m1} queries in {el1:.1f}s on 1 thread")
    out = {"value": round(m / el, 3), "unit": "queries/s", "cores": threads, "kind": "oracle",
           "sample": f"first {m} of {w.nq} queries, same index, nprobe={nprobe}, FP64 sequential "
                     f"IVF+ scan per query (threads over queries)",
           "dims_ratio": round(float(st[:, 1].sum()) / max(1, st[:, 0].sum() * w.D), 5),
           "one_thread": {"value": round(m1 / el1, 3), "unit": "queries/s", "cores": 1,
                          "sample": f"first {m1} queries"}}
    if gt is not None and gpu_ids is not None:
        r_orc = oracle.recall(ids, exact_for(x, q[:m], ids), gt[:m], K)
        g = gpu_ids[:m]
        r_gpu = oracle.recall(g, exact_for(x, q[:m], g), gt[:m], K)
        out.update({"oracle_recall": round(r_orc, 5), "gpu_recall_same_queries": round(r_gpu, 5),
                    "abs_recall_diff": round(abs(r_gpu - r_orc), 5)})
        log(f"cpu baseline: recall on the sample oracle {r_orc:.4f} gpu {r_gpu:.4f}")
    return out


if __name__ == "__main__":
    sys.exit(main())
