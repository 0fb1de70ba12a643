"""Batched launches: a whole uneven search captured into one HIP graph and
replayed, and the autotuner."""

import math

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
def wl(ads):
    w = Workload("lowrank", 40_000, 256, 256, 64, 7001, latent=32, noise=0.05)
    P32, _ = ads.make_rotation(w.G)
    ix = ads.ivf_build(w.x, P32, w.cent, w.assign, delta_d=32, storage=ads.F32, keep_fp32=True)
    return w, ix, P32


def test_graph_replays_match_eager(ads, wl):
    """Replays of the captured search, with the program's own eager work and
    synchronisations between them, each equal the eager search bit for bit."""
    w, ix, _ = wl
    rng = np.random.default_rng(11)
    nq, k_max, p_max = 200, 50, 24
    plan = ads.Plan(ix, nq, k_max, p_max, eps0=2.1)
    for rep in range(4):
        rows = rng.choice(w.nq, size=nq)
        K = rng.choice([1, 10, 50], size=nq).astype(np.int32)
        npb = rng.integers(1, p_max + 1, size=nq).astype(np.int32)
        plan.q.copy_(torch.as_tensor(w.q[rows]))
        plan.K.copy_(torch.as_tensor(K))
        plan.nprobe.copy_(torch.as_tensor(npb))
        plan.launch()
        torch.cuda.synchronize()
        g_ids, g_d = plan.ids.cpu().numpy(), plan.dist.cpu().numpy()
        # eager work between replays
        e_ids, e_d = ads.search(ix, w.q[rows], k_max, p_max, eps0=2.1, K=K, nprobe=npb)
        torch.cuda.synchronize()
        assert np.array_equal(g_ids, e_ids.cpu().numpy()), rep
        assert np.array_equal(g_d, e_d.cpu().numpy()), rep
    plan.free()


def test_plan_rejects_missing_workspace_and_bad_sizes(ads, wl):
    import ctypes
    w, ix, _ = wl
    lib = ads.load()
    out = ctypes.c_void_p()
    st = lib.ads_plan_create(ix.handle, None, 4, None, None, 10, 4, 2.1, 0, 0, None, None, None, None,
                             ctypes.byref(out))
    assert st == -1 and "workspace" in ads.last_error()


def test_autotuner_meets_recall_constraint_and_caches(ads, wl, tmp_path):
    from paper_2303_09855_amd.autotune import Autotuner
    w, _, P32 = wl
    tuner = Autotuner(str(tmp_path / "tune.json"))
    small = {"queries_per_unit": [4, 8], "dense_frac": [0.125, 0.25], "sweep_log2": [2, 3],
             "grid_per_xcd": [0, 512]}
    before = ads.get_tuning()
    res, ix = tuner.tune(w.x, P32, w.cent, w.assign, w.q, 10, 16, delta_d_choices=(16, 32),
                         choices=small, reps=2)
    assert res.recall_vs_fds >= 0.998
    assert res.delta_d in (16, 32)
    assert ix.info()["delta_d"] == res.delta_d
    assert ads.get_tuning() == before          # the tuner restores the thread's knobs
    again = Autotuner(str(tmp_path / "tune.json"))
    entry = again.lookup(res.key)
    assert entry and entry["delta_d"] == res.delta_d
    again.apply(entry)
    assert ads.get_tuning()["dense_frac"] == pytest.approx(entry["knobs"]["dense_frac"])
    ads.set_tuning(**before)
    ix.free()
