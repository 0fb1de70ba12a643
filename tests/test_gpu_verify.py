"""The failure law of the ADSampling test on the GPU (Lemma 3.2, Section 3.1's
equivalence with random projection; the verification methodology of
Section 6.2.6).

For a fixed vector x and Haar-random rotations P_s, the partial sums of the
rotated coordinates of x have the law of the partial sums of a normalised
Gaussian vector.  The GPU decides DCOs of q = 0 against the candidates P_s x
with r = |x| / rho through ads_dco_batch; its failure rate (positives
rejected) and the mean sampled dimensions of negatives must match what an
independent FP64 Monte Carlo over Gaussian vectors predicts, within binomial
error.  Expected values come from numpy, never from the GPU."""

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


def _rotated_copies(D, S, seed):
    """S rotations P_s x of one fixed x (FP64 QR per seed), as float32 rows."""
    x = np.random.default_rng(seed).standard_normal(D)
    rows = np.empty((S, D), dtype=np.float32)
    for s in range(S):
        P = oracle.make_rotation(sd.gaussian_matrix(D, seed + 1 + s))
        rows[s] = P @ x
    return x, rows


def _gaussian_law(D, dd, eps0, rho, M=400_000, seed=77):
    """Monte Carlo over g ~ N(0, I_D): P{some test at d < D rejects} and the
    mean number of sampled dims, for dis / r = rho (Algorithm 1 with blocks of
    dd coordinates)."""
    g = np.random.default_rng(seed).standard_normal((M, D))
    part = np.cumsum(g ** 2, axis=1) / np.sum(g ** 2, axis=1, keepdims=True)
    ds = np.arange(dd, D, dd)
    thr = (ds / D) * (1 + eps0 / np.sqrt(ds)) ** 2 / rho ** 2
    rej = part[:, ds - 1] > thr[None, :]
    any_rej = rej.any(axis=1)
    first = np.where(any_rej, ds[np.argmax(rej, axis=1)], D)
    return float(any_rej.mean()), float(first.mean()), float(first.std())


@pytest.mark.parametrize("D,dd,eps0,rho", [(64, 8, 1.0, 0.9), (64, 1, 1.5, 0.95), (128, 32, 0.5, 0.97)])
def test_gpu_failure_rate_matches_gaussian_law(ads, D, dd, eps0, rho):
    S = 4000
    x, rows = _rotated_copies(D, S, 300_000 + D + dd)
    eye = np.eye(D, dtype=np.float32)
    assign = np.zeros(S, dtype=np.int32)
    cent = rows.mean(axis=0, keepdims=True)
    # the rows are already rotated: an identity P keeps them as they are
    ix = ads.ivf_build(rows, eye, cent, assign, delta_d=8, storage=ads.F32,
                       keep_fp32=True)
    try:
        r = float(np.linalg.norm(x)) / rho
        mask, dist, dims = ads.dco_batch(ix, np.zeros(D, dtype=np.float32), np.arange(S), r, eps0, dd)
        torch.cuda.synchronize()
        mask = mask.cpu().numpy()
        rate = float(np.mean(mask == 0))
        p, _, _ = _gaussian_law(D, dd, eps0, rho)
        sigma = math.sqrt(p * (1 - p) / S + p * (1 - p) / 400_000)
        assert 0.005 < p < 0.7
        assert abs(rate - p) < 4.5 * sigma, (rate, p)
    finally:
        ix.free()


def test_gpu_dims_of_negatives_match_gaussian_law(ads):
    D, dd, eps0, rho, S = 64, 8, 1.0, 1.25, 4000
    x, rows = _rotated_copies(D, S, 410_000)
    ix = ads.ivf_build(rows, np.eye(D, dtype=np.float32), rows.mean(axis=0, keepdims=True),
                       np.zeros(S, dtype=np.int32), delta_d=8, storage=ads.F32, keep_fp32=True)
    try:
        r = float(np.linalg.norm(x)) / rho
        mask, _, dims = ads.dco_batch(ix, np.zeros(D, dtype=np.float32), np.arange(S), r, eps0, dd)
        torch.cuda.synchronize()
        mask, dims = mask.cpu().numpy(), dims.cpu().numpy()
        assert mask.sum() == 0                       # dis > r: never positive (Lemma 3.2)
        _, mean_dims, sd_dims = _gaussian_law(D, dd, eps0, rho)
        assert abs(dims.mean() - mean_dims) < 4.5 * sd_dims / math.sqrt(S)
    finally:
        ix.free()
