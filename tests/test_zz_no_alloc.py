"""The allocation-free search (ads_search_noalloc) through the C ABI: its
results equal ads_search's bit for bit on two calls in a row (the second with
a smaller batch, so the scratch array keeps the first call's contents), and a
request whose workspace exceeds the scratch array is rejected."""

import math

import numpy as np
import pytest

from helpers import Workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ads():
    import paper_2303_09855_amd as m
    m.load()
    assert torch.cuda.is_available(), "the GPU tests need a visible GPU"
    return m


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_noalloc_search_equals_search(ads):
    w = Workload("lowrank", 20_000, 48, 256, 64, 6002, latent=32, noise=0.05)
    P32, _ = ads.make_rotation(w.G)
    ix = ads.ivf_build(w.x, P32, w.cent, w.assign, delta_d=16, storage=ads.F32, keep_fp32=True)
    try:
        rng = np.random.default_rng(7)
        K = rng.choice([1, 10, 40], size=w.nq).astype(np.int32)
        npb = rng.integers(1, 24, size=w.nq).astype(np.int32)
        cases = [
            # (queries, k_max, nprobe_max, eps0, method, rerank, per-query K / nprobe)
            (slice(0, 48), 40, 24, 2.1, ads.ADSAMPLING, 0, True),
            (slice(5, 17), 10, 8, math.inf, ads.FDSCANNING, 1, False),
        ]
        for sl, k_max, p_max, eps0, method, rerank, per_query in cases:
            qs = w.q[sl]
            kw = dict(K=np.minimum(K[sl], k_max), nprobe=np.minimum(npb[sl], p_max)) if per_query else {}
            s_ref = torch.zeros(ads.NSTATS, dtype=torch.int64, device="cuda")
            s_na = torch.zeros(ads.NSTATS, dtype=torch.int64, device="cuda")
            ref = ads.search(ix, qs, k_max, p_max, eps0=eps0, method=method, rerank=rerank,
                             want_probes=True, stats=s_ref, **kw)
            got = ads.search_noalloc(ix, qs, k_max, p_max, eps0=eps0, method=method, rerank=rerank,
                                     want_probes=True, stats=s_na, **kw)
            for a, b in zip(ref, got):
                assert np.array_equal(_np(a), _np(b))
            assert np.array_equal(_np(s_ref), _np(s_na))
            assert int(_np(got[0] >= 0).sum()) > 0
        # a workspace beyond the scratch array is rejected with a message
        big_nq = 4096
        need = ads.search_workspace_size(ix, big_nq, 512, 64)
        assert need > ads.NOALLOC_SCRATCH_BYTES
        with pytest.raises(ads.AdsError) as ei:
            ads.search_noalloc(ix, torch.zeros((big_nq, w.D), device="cuda"), 512, 64)
        assert "scratch" in str(ei.value)
    finally:
        ix.free()
