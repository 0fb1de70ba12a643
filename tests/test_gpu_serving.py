"""Serving loop: continuous batching, overlapping in-flight batches, HBM
admission; each request's result equals its result when run alone."""

import numpy as np
import pytest

import synthdata as sd
from helpers import Workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ads():
    import paper_2303_09855_amd as m
    m.load()
    assert torch.cuda.is_available(), "the GPU tests need a visible GPU"
    return m


@pytest.fixture(scope="module")
def served(ads):
    w = Workload("lowrank", 40_000, 300, 256, 64, 9001, latent=32, noise=0.05)
    P32, _ = ads.make_rotation(w.G)
    ix = ads.ivf_build(w.x, P32, w.cent, w.assign, delta_d=32, storage=ads.F32, keep_fp32=True)
    rng = np.random.default_rng(3)
    t = sd.poisson_arrivals(20000.0, w.nq, seed=1047)
    from paper_2303_09855_amd.serving import Request
    reqs = [Request(i, w.q[i], int(rng.choice([10, 50])), int(rng.choice([8, 16])), float(t[i]))
            for i in range(w.nq)]
    return w, ix, reqs


def _alone(ads, ix, r):
    ids, dist = ads.search(ix, r.q[None, :], r.K, r.nprobe, eps0=2.1)
    torch.cuda.synchronize()
    return ids.cpu().numpy()[0], dist.cpu().numpy()[0]


def test_results_in_the_mix_equal_alone(ads, served):
    from paper_2303_09855_amd.serving import Server
    w, ix, reqs = served
    srv = Server(ix, k_max=50, nprobe_max=16, max_batch=64, n_streams=3)
    res, lat, st = srv.run(reqs)
    assert st["requests"] == len(reqs) and st["batches"] >= 2
    assert all(v >= 0 for v in lat.values())
    for r in reqs[::17]:
        a_ids, a_d = _alone(ads, ix, r)
        assert np.array_equal(res[r.rid][0], a_ids), r.rid
        assert np.array_equal(res[r.rid][1], a_d), r.rid


def test_small_hbm_budget_forces_small_batches(ads, served):
    from paper_2303_09855_amd.serving import Server
    w, ix, reqs = served
    srv = Server(ix, k_max=50, nprobe_max=16, max_batch=512, n_streams=2)
    budget = srv.batch_bytes(24)
    srv.admission.budget = budget
    res, _, st = srv.run(reqs[:120], realtime=False)
    assert st["batches"] >= 120 // 24
    for r in reqs[:120:13]:
        a_ids, a_d = _alone(ads, ix, r)
        assert np.array_equal(res[r.rid][0], a_ids)
