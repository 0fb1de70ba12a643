"""GPU k-means (ads_kmeans / ads_build_ivf) against the oracle's FP64 Lloyd
iterations with the same SplitMix64 initialisation (the IVF index phase,
Section 2.2.2).  The GPU scores centres in the FP32 GEMM form, so a row may
take a different centre only when its two nearest centres lie within the
rounding band; integer data of small magnitude is exact in FP32, so there
both sides agree row for row, empty-list repairs included."""

import math

import numpy as np
import pytest

import oracle
import synthdata as sd

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


def _band(x, c):
    """FP32 GEMM-form rounding band of the squared distances, per (row, centre)."""
    D = x.shape[1]
    s = np.linalg.norm(x, axis=1)[:, None] + np.linalg.norm(c, axis=1)[None, :]
    return 4.0 * math.sqrt(D) * 2.0 ** -24 * s * s


def _d2(x, c):
    x = x.astype(np.float64)
    c = c.astype(np.float64)
    return np.maximum(np.sum(x * x, 1)[:, None] + np.sum(c * c, 1)[None, :] - 2 * x @ c.T, 0)


def test_kmeans_initial_centres_and_assignment(ads):
    x = sd.lowrank(20_000, 64, 901, 902, latent=8, noise=0.3)
    nlist, seed = 48, 123
    cent, assign = ads.kmeans(x, nlist, iters=0, seed=seed)
    cent, assign = _np(cent), _np(assign)
    init = oracle.kmeans_init_rows(len(x), nlist, seed)
    assert np.array_equal(cent, x[init])                     # the seeded rows, bit for bit
    c64, lab = oracle.kmeans(x, nlist, 0, seed=seed)
    d2 = _d2(x, c64)
    band = _band(x, c64)
    diff = np.flatnonzero(assign != lab)
    for i in diff:
        assert d2[i, assign[i]] - d2[i, lab[i]] <= band[i, assign[i]] + band[i, lab[i]], i
    assert len(diff) <= 5


def test_kmeans_iterations_match_oracle(ads):
    x = sd.lowrank(20_000, 64, 911, 912, latent=8, noise=0.3)
    nlist, seed, iters = 40, 7, 4
    cent, assign = ads.kmeans(x, nlist, iters=iters, seed=seed)
    cent, assign = _np(cent), _np(assign)
    c64, lab = oracle.kmeans(x, nlist, iters, seed=seed)
    agree = np.mean(assign == lab)
    assert agree >= 0.998, agree
    # centres of lists with the same members agree to float32 rounding
    same = [j for j in range(nlist) if np.array_equal(np.flatnonzero(assign == j), np.flatnonzero(lab == j))]
    assert len(same) >= nlist // 2
    for j in same:
        assert np.linalg.norm(cent[j] - c64[j]) <= 1e-6 * (np.linalg.norm(c64[j]) + 1e-3), j
    obj_g = float(np.sum((x.astype(np.float64) - cent[assign].astype(np.float64)) ** 2))
    obj_o = float(np.sum((x.astype(np.float64) - c64[lab]) ** 2))
    assert abs(obj_g - obj_o) <= 1e-4 * obj_o


def test_kmeans_empty_list_repair_exact(ads):
    """Integer rows with many duplicates: several initial centres coincide,
    their lists come up empty, and the repair moves the farthest members of
    the largest lists.  Every distance is an exact integer in FP32, so the
    GPU's lists equal the oracle's row for row."""
    rng = np.random.default_rng(5)
    distinct = rng.integers(0, 12, size=(9, 8)).astype(np.float32)
    x = distinct[rng.integers(0, 9, size=600)]
    noisy = rng.random(600) < 0.3
    x[noisy, rng.integers(0, 8, size=noisy.sum())] += 1
    nlist = 30
    for iters in (1, 3):
        cent, assign = ads.kmeans(x, nlist, iters=iters, seed=99)
        cent, assign = _np(cent), _np(assign)
        c64, lab = oracle.kmeans(x, nlist, iters, seed=99)
        assert np.array_equal(assign, lab)
        assert np.allclose(cent, c64, rtol=1e-6, atol=1e-6)
        # the repair ran: without it some list would be empty after the first assignment
        _, lab0 = oracle.kmeans(x, nlist, 0, seed=99)
        assert len(np.unique(lab0)) < nlist


def test_build_ivf_equals_build_from_its_clustering(ads):
    """ads_build_ivf is k-means followed by ads_ivf_build: searching its index
    equals searching an index built from the clustering it returns."""
    x = sd.lowrank(12_000, 128, 921, 922, latent=16, noise=0.2)
    q = sd.lowrank(20, 128, 923, 922, latent=16, noise=0.2)
    P32, _ = ads.make_rotation(sd.gaussian_matrix(128, 924))
    ix, cent, assign = ads.build_ivf(x, P32, 32, iters=5, seed=3, delta_d=32, want_clustering=True)
    ix2 = ads.ivf_build(x, P32, cent, assign, delta_d=32)
    try:
        c64, lab = oracle.kmeans(x, 32, 5, seed=3)
        assert np.mean(_np(assign) == lab) >= 0.998
        for eps0 in (math.inf, 2.1):
            a = [_np(t) for t in ads.search(ix, q, 10, 6, eps0=eps0)]
            b = [_np(t) for t in ads.search(ix2, q, 10, 6, eps0=eps0)]
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    finally:
        ix.free()
        ix2.free()
