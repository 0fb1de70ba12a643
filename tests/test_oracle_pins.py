"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's own formula: each checks it against
an independent fact (a closed form, a library distribution, a brute-force sort,
an invariant of the method, or a hand-derived case).
"""

import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
import synthdata as sd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _f(v):
    return math.inf if v == "inf" else float(v)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


# --------------------------------------------------------------------------
# Section 3.1: the random orthogonal transformation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("D", [16, 128, 960])
def test_rotation_is_orthogonal_and_preserves_norms(D):
    P = oracle.make_rotation(sd.gaussian_matrix(D, 1001))
    assert np.max(np.abs(P.T @ P - np.eye(D))) <= 1e-10
    x = np.random.default_rng(3).standard_normal((20, D))
    y = oracle.rotate(x, P)
    ratio = np.linalg.norm(y, axis=1) / np.linalg.norm(x, axis=1)
    assert np.max(np.abs(ratio - 1.0)) <= 1e-12


def test_rotation_orientation_and_row_sampling_identity():
    """Eq. 2: sampling the first d rows after the product equals the product
    with the first d rows of P' (y = P' x, not x^T P')."""
    D, d = 32, 7
    P = oracle.make_rotation(sd.gaussian_matrix(D, 5))
    x = np.random.default_rng(4).standard_normal((9, D))
    y = oracle.rotate(x, P)
    assert np.allclose(y[:, :d], x @ P[:d].T, rtol=0, atol=1e-13)
    # the first coordinate of y for x = e_j is P[0, j] (column-vector convention)
    e = np.zeros((1, D))
    e[0, 3] = 1.0
    assert abs(oracle.rotate(e, P)[0, 0] - P[0, 3]) < 1e-15


def test_rotation_is_haar_sign_symmetric():
    """A Haar orthogonal matrix has E[P_00] = 0.  Plain Householder QR without
    the sign fix gives P_00 of one sign only, which this catches."""
    D, S = 8, 3000
    v = np.array([oracle.make_rotation(sd.gaussian_matrix(D, 10_000 + s))[0, 0] for s in range(S)])
    sigma = 1.0 / math.sqrt(D * S)
    assert abs(v.mean()) < 5 * sigma
    assert 0.3 < np.mean(v > 0) < 0.7


def test_rotation_partial_norm_follows_beta_law():
    """For Haar P and fixed x, ||(Px)|[1..d]||^2 / ||x||^2 ~ Beta(d/2, (D-d)/2)
    (the equivalence of Section 3.1 between sampling rotated coordinates and a
    random projection)."""
    D, d, S = 24, 6, 3000
    x = np.random.default_rng(8).standard_normal(D)
    vals = []
    for s in range(S):
        P = oracle.make_rotation(sd.gaussian_matrix(D, 20_000 + s))
        y = P @ x
        vals.append(np.sum(y[:d] ** 2) / np.sum(x ** 2))
    res = stats.kstest(vals, stats.beta(d / 2, (D - d) / 2).cdf)
    assert res.pvalue > 1e-3


# --------------------------------------------------------------------------
# Algorithm 1: hand-derived golden cases
# --------------------------------------------------------------------------

def _golden():
    with open(os.path.join(GOLDEN, "dco_cases.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("case", _golden()["ads"], ids=lambda c: c["name"])
def test_ads_golden_cases(case):
    pos, dist, dims = oracle.ads_dco(np.array(case["o"], float), np.array(case["q"], float),
                                     _f(case["r"]), _f(case["eps0"]), case["delta_d"])
    ex = case["expect"]
    assert pos == ex["positive"]
    assert dims == ex["dims"]
    if ex["dist"] == "inf":
        assert math.isinf(dist)
    else:
        assert dist == pytest.approx(ex["dist"], rel=1e-15, abs=1e-15)


@pytest.mark.parametrize("case", _golden()["pds"], ids=lambda c: c["name"])
def test_pds_golden_cases(case):
    res = oracle.dco_batch(np.array([case["o"]], float), np.array(case["q"], float),
                           np.array([0]), _f(case["r"]), math.inf, case["delta_d"],
                           method=oracle.METHOD_PDS)
    ex = case["expect"]
    assert res["mask"][0] == ex["positive"]
    assert res["dims"][0] == ex["dims"]
    assert math.isinf(res["dist"][0]) == (ex["dist"] == "inf")


@pytest.mark.parametrize("case", _golden()["band"], ids=lambda c: c["name"])
def test_band_golden_cases(case):
    """The parity band (a decision taken within 1e-5 relative of its test
    boundary): hand-derived cases just inside and just outside the boundary of
    the Section 3.2 test, at the exact compare of Case 3, and for PDScanning."""
    res = oracle.dco_batch(np.array([case["o"]], float), np.array(case["q"], float),
                           np.array([0]), _f(case["r"]), _f(case["eps0"]), case["delta_d"],
                           method=case["method"])
    ex = case["expect"]
    assert res["band"][0] == ex["band"]
    assert res["mask"][0] == ex["positive"]
    assert res["dims"][0] == ex["dims"]


# --------------------------------------------------------------------------
# Closed forms and invariants of Algorithm 1
# --------------------------------------------------------------------------

def _pairs(D=128, n=3000, seed=11):
    x = sd.mixture(n, D, seed, 1000)
    q = sd.mixture(4, D, seed + 1, 1000)
    P = oracle.make_rotation(sd.gaussian_matrix(D, 1001))
    return x, q, P


def test_exact_case_returns_raw_space_distance():
    """Case 3: at d = D, dis' equals the true distance (rotation preserves
    norms), so every positive's distance equals the unrotated distance."""
    x, q, P = _pairs()
    xr, qr = oracle.rotate(x, P), oracle.rotate(q, P)
    raw = oracle.exact_dist(x, q[0])
    r = np.quantile(raw, 0.05)
    res = oracle.dco_batch(xr, qr[0], np.arange(len(x)), r, 2.1, 32)
    pos = res["mask"] == 1
    assert pos.sum() > 10
    assert np.allclose(res["dist"][pos], raw[pos], rtol=1e-12, atol=0)
    assert np.all(res["dims"][pos] == x.shape[1])


def test_no_false_positives_lemma_3_2():
    """Lemma 3.2, first line: a negative object (dis > r) is never reported
    positive; and every positive really has dis <= r."""
    x, q, P = _pairs()
    xr, qr = oracle.rotate(x, P), oracle.rotate(q, P)
    for qi in range(4):
        raw = oracle.exact_dist(x, q[qi])
        for quant in (0.01, 0.2, 0.6):
            r = np.quantile(raw, quant)
            for eps0 in (0.0, 1.0, 2.1):
                res = oracle.dco_batch(xr, qr[qi], np.arange(len(x)), r, eps0, 16)
                assert np.all(raw[res["mask"] == 1] <= r * (1 + 1e-12))
                assert np.all(res["mask"][raw > r * (1 + 1e-12)] == 0)


def test_eps_inf_and_full_block_equal_fdscanning():
    """eps0 = +inf (never reject) or delta_d = D (no test before d = D) is
    FDScanning: identical masks and distances, D dims each."""
    x, q, P = _pairs()
    xr, qr = oracle.rotate(x, P), oracle.rotate(q, P)
    raw = oracle.exact_dist(x, q[1])
    r = np.quantile(raw, 0.1)
    rows = np.arange(len(x))
    fds = oracle.dco_batch(xr, qr[1], rows, r, math.inf, 32, method=oracle.METHOD_FDS)
    a = oracle.dco_batch(xr, qr[1], rows, r, math.inf, 32)
    b = oracle.dco_batch(xr, qr[1], rows, r, 2.1, x.shape[1])
    for res in (a, b):
        assert np.array_equal(res["mask"], fds["mask"])
        assert np.array_equal(res["dist"], fds["dist"])
        assert np.all(res["dims"] == x.shape[1])


def test_pdscanning_is_exact():
    """PDScanning (Section 6.1) is an exact DCO: same masks as FDScanning."""
    x, q, P = _pairs()
    raw = oracle.exact_dist(x, q[2])
    r = np.quantile(raw, 0.1)
    rows = np.arange(len(x))
    xd = x.astype(np.float64)
    fds = oracle.dco_batch(xd, q[2].astype(np.float64), rows, r, math.inf, 32,
                           method=oracle.METHOD_FDS)
    pds = oracle.dco_batch(xd, q[2].astype(np.float64), rows, r, math.inf, 32,
                           method=oracle.METHOD_PDS)
    assert np.array_equal(pds["mask"], fds["mask"])
    assert np.all(pds["dims"] <= x.shape[1])
    assert np.mean(pds["dims"][pds["mask"] == 0]) < x.shape[1]


def test_monotone_in_eps0():
    """For fixed P, data and r, a larger eps0 raises every test boundary, so
    per-pair sampled dims are non-decreasing and an accepted positive stays
    accepted (failures are non-increasing), as Lemmas 3.2 and 3.3 describe."""
    x, q, P = _pairs()
    xr, qr = oracle.rotate(x, P), oracle.rotate(q, P)
    raw = oracle.exact_dist(x, q[0])
    r = np.quantile(raw, 0.3)
    rows = np.arange(len(x))
    prev = None
    fails = []
    for eps0 in (0.0, 0.5, 1.0, 1.5, 2.1, 3.0, 4.0):
        res = oracle.dco_batch(xr, qr[0], rows, r, eps0, 8)
        if prev is not None:
            assert np.all(res["dims"] >= prev["dims"])
            assert np.all(res["mask"] >= prev["mask"])
        fails.append(int(np.sum((raw <= r) & (res["mask"] == 0))))
        prev = res
    assert fails == sorted(fails, reverse=True)
    assert fails[0] > fails[-1]


def _single_test_failure(D, dd, eps0, rho, S, seed0):
    """Empirical failure rate of Algorithm 1 over S independent rotations for
    one fixed positive pair with dis / r = rho (<= 1)."""
    rng = np.random.default_rng(seed0)
    x = rng.standard_normal(D)
    r = np.linalg.norm(x) / rho
    fails = 0
    dims = 0
    for s in range(S):
        P = oracle.make_rotation(sd.gaussian_matrix(D, seed0 + 1 + s))
        pos, _, dd_used = oracle.ads_dco(P @ x, np.zeros(D), r, eps0, dd)
        fails += (pos == 0)
        dims += dd_used
    return fails / S, dims / S


def test_single_test_failure_probability_matches_beta_law():
    """With D = 2 * delta_d there is exactly one test (at d = D/2).  A positive
    with dis/r = rho fails iff (D/d) B > gamma^2 / rho^2 with
    B ~ Beta(d/2, (D-d)/2) (Section 3.2 test + the Beta law of Section 3.1)."""
    D, dd, eps0, rho, S = 32, 16, 0.6, 0.95, 4000
    rate, _ = _single_test_failure(D, dd, eps0, rho, S, 50_000)
    gamma = 1 + eps0 / math.sqrt(dd)
    p = stats.beta(dd / 2, (D - dd) / 2).sf((dd / D) * gamma ** 2 / rho ** 2)
    sigma = math.sqrt(p * (1 - p) / S)
    assert 0.01 < p < 0.5
    assert abs(rate - p) < 4.5 * sigma


def test_expected_dims_of_negative_matches_beta_law():
    """Negative with dis/r = rho > 1, one test at d = D/2:
    E[dims] = d + (D - d) * P{no rejection} = d + (D-d) * Beta.cdf(...)."""
    D, dd, eps0, rho, S = 32, 16, 1.0, 1.3, 4000
    _, mean_dims = _single_test_failure(D, dd, eps0, rho, S, 70_000)
    gamma = 1 + eps0 / math.sqrt(dd)
    p_keep = stats.beta(dd / 2, (D - dd) / 2).cdf((dd / D) * gamma ** 2 / rho ** 2)
    expect = dd + (D - dd) * p_keep
    sd_dims = (D - dd) * math.sqrt(p_keep * (1 - p_keep) / S)
    assert abs(mean_dims - expect) < 4.5 * sd_dims


def test_sequential_failure_rate_matches_gaussian_monte_carlo():
    """Several tests (delta_d = 4, D = 48): the failure rate over random
    rotations equals the probability computed independently from a Gaussian
    vector g ~ N(0, I_D), whose normalised partial sums have the same law as
    the rotated coordinates of a fixed vector."""
    D, dd, eps0, rho, S = 48, 4, 1.2, 0.9, 3000
    rate, _ = _single_test_failure(D, dd, eps0, rho, S, 90_000)
    g = np.random.default_rng(123).standard_normal((200_000, D))
    part = np.cumsum(g ** 2, axis=1) / np.sum(g ** 2, axis=1, keepdims=True)
    ds = np.arange(dd, D, dd)
    thr = (ds / D) * (1 + eps0 / np.sqrt(ds)) ** 2 / rho ** 2
    p = np.mean(np.any(part[:, ds - 1] > thr[None, :], axis=1))
    sigma = math.sqrt(p * (1 - p) / S + p * (1 - p) / 200_000)
    assert 0.01 < p < 0.6
    assert abs(rate - p) < 4.5 * sigma


def test_failure_rate_decreases_with_eps0_like_figure_12():
    """Fixed threshold = exact K-th NN distance, linear scan, delta_d = 1
    (the verification protocol of Section 6.2.6): the recall of positives
    rises towards 1 as eps0 grows and is near 1 by eps0 = 2."""
    w = sd.WORKLOADS["flat_d128"]
    x = sd.base_vectors(w)[:3000]
    q = sd.query_vectors(w)[:5]
    P = oracle.make_rotation(sd.rotation_gaussian(w))
    xr, qr = oracle.rotate(x, P), oracle.rotate(q, P)
    _, gt = oracle.brute_knn(x, q, 10)
    rates = []
    for eps0 in (0.5, 1.0, 2.0, 3.0):
        ok = tot = 0
        for i in range(5):
            res = oracle.dco_batch(xr, qr[i], np.arange(len(x)), gt[i, 9], eps0, 1)
            raw = oracle.exact_dist(x, q[i])
            # strict positives: objects tied with the K-th distance sit on the
            # boundary, where the rounding of the rotation decides
            posmask = raw < gt[i, 9] * (1 - 1e-9)
            ok += int(np.sum(res["mask"][posmask]))
            tot += int(np.sum(posmask))
        rates.append(ok / tot)
    assert rates == sorted(rates)
    assert rates[0] < 0.9
    assert rates[2] >= 0.97


# --------------------------------------------------------------------------
# Exact KNN, IVF scan and metrics
# --------------------------------------------------------------------------

def test_brute_knn_equals_full_sort():
    x = sd.mixture(3000, 16, 31, 32)
    q = sd.mixture(20, 16, 33, 32)
    ids, dist = oracle.brute_knn(x, q, 7, screen=8, chunk=500)
    for i in range(len(q)):
        dv = np.sqrt(np.sum((x.astype(np.float64) - q[i]) ** 2, axis=1))
        order = np.lexsort((np.arange(len(x)), dv))[:7]
        assert np.array_equal(dist[i], dv[order])
        # exact integer data: equal distances are exact ties, check the id set
        # within the tie band at the K-th distance only
        kth = dv[order[-1]]
        assert set(ids[i][dist[i] < kth]) == set(order[dv[order] < kth])


def test_ivf_golden_tiny():
    with open(os.path.join(GOLDEN, "ivf_tiny.json")) as fh:
        g = json.load(fh)
    base = np.array(g["base"], float)
    cent = np.array(g["centroids"], float)
    off, members = oracle.lists_from_assignment(np.array(g["assign"]), len(cent))
    for case in g["cases"]:
        q = np.array([case["q"]], float)
        pr, _ = oracle.probes(q, cent, case["nprobe"])
        assert pr[0].tolist() == case["probes"]
        for method in (oracle.METHOD_FDS, oracle.METHOD_ADS, oracle.METHOD_PDS):
            ids, dist, _ = oracle.ivf_search(base, q, off, members, pr, case["K"], 2.1, 1,
                                             method=method)
            assert ids[0].tolist() == case["ids"]
            assert np.allclose(dist[0], case["dist"], rtol=1e-12)


def test_probe_selection_golden_ties():
    """Probe order with exact ties at the boundary: ascending distance, then
    the lower list id."""
    with open(os.path.join(GOLDEN, "ivf_tiny.json")) as fh:
        g = json.load(fh)["probe_cases"]
    cent = np.array(g["centroids"], float)
    for case in g["cases"]:
        pr, _ = oracle.probes(np.array([case["q"]], float), cent, case["nprobe"])
        assert pr[0].tolist() == case["probes"], case["why"]


@pytest.mark.parametrize("method", [oracle.METHOD_FDS, oracle.METHOD_ADS])
def test_ivf_all_lists_equals_brute_force(method):
    """nprobe = nlist with exact DCOs (eps0 = +inf) is an exact KNN: identical
    ids (lower id first on ties) and distances to a full sort.  P = I keeps the
    integer data exact, so ties are exact too."""
    x = sd.mixture(4000, 24, 41, 42)
    q = sd.mixture(15, 24, 43, 42)
    cent, assign = sd.clustering(x, 16, 44, iters=3)
    off, members = oracle.lists_from_assignment(assign, 16)
    pr, _ = oracle.probes(q, cent, 16)
    ids, dist, st = oracle.ivf_search(x.astype(np.float64), q, off, members, pr, 9,
                                      math.inf, 8, method=method)
    assert np.all(st[:, 0] == len(x))
    for i in range(len(q)):
        dv = np.sqrt(np.sum((x.astype(np.float64) - q[i]) ** 2, axis=1))
        order = np.lexsort((np.arange(len(x)), dv))[:9]
        assert ids[i].tolist() == order.tolist()
        assert np.array_equal(dist[i], dv[order])


def test_ivf_ads_keeps_accuracy_and_saves_dims():
    """Section 6.2 trends on a small low-rank set: ADSampling (eps0 = 2.1,
    delta_d = 32) loses almost no recall against FDScanning while sampling a
    fraction of the dimensions; negatives vastly outnumber positives."""
    D = 256
    x = sd.lowrank(20000, D, 51, 52, latent=32, noise=0.05)
    q = sd.lowrank(40, D, 53, 52, latent=32, noise=0.05)
    P = oracle.make_rotation(sd.gaussian_matrix(D, 54))
    xr, qr = oracle.rotate(x, P), oracle.rotate(q, P)
    cent, assign = sd.clustering(x, 64, 55, iters=5)
    cr = oracle.rotate(cent, P)
    off, members = oracle.lists_from_assignment(assign, 64)
    pr, _ = oracle.probes(qr, cr, 12)
    _, gt = oracle.brute_knn(x, q, 10)
    f_ids, f_d, f_st = oracle.ivf_search(xr, qr, off, members, pr, 10, math.inf, 32,
                                         method=oracle.METHOD_FDS)
    a_ids, a_d, a_st = oracle.ivf_search(xr, qr, off, members, pr, 10, 2.1, 32)
    rf = oracle.recall(f_ids, f_d, gt, 10)
    ra = oracle.recall(a_ids, a_d, gt, 10)
    assert rf - ra <= 0.01
    assert oracle.dims_ratio(a_st, D) < 0.5
    assert oracle.dims_ratio(f_st, D) == 1.0
    neg = a_st[:, 0].sum() - a_st[:, 2].sum()
    assert neg / max(1, a_st[:, 2].sum()) > 10


def test_recall_and_ratio_metrics_hand_cases():
    gt = np.array([[1.0, 2.0, 3.0]])
    # returned ids/dists: one wrong object at 3.5, one tie with the K-th
    ids = np.array([[5, 7, 9]])
    d = np.array([[1.0, 3.0, 3.5]])
    assert oracle.recall(ids, d, gt, 3) == pytest.approx(2 / 3)
    assert oracle.distance_ratio(d, gt, 3) == pytest.approx((1 + 1.5 + 3.5 / 3) / 3)
    # padding (-1) never counts
    ids2 = np.array([[5, -1, -1]])
    d2 = np.array([[1.0, np.inf, np.inf]])
    assert oracle.recall(ids2, d2, gt, 3) == pytest.approx(1 / 3)
    assert oracle.dims_ratio(np.array([[10, 320, 1]]), 128) == pytest.approx(0.25)


# --------------------------------------------------------------------------
# Section 2.2.2 index phase: k-means
# --------------------------------------------------------------------------

def _kmeans_golden():
    with open(os.path.join(GOLDEN, "kmeans_tiny.json")) as fh:
        return json.load(fh)


def test_splitmix64_published_outputs():
    g = _kmeans_golden()["splitmix64"]
    st = g["state"]
    out = []
    for _ in range(3):
        st = (st + 0x9E3779B97F4A7C15) % (1 << 64)
        out.append(oracle.splitmix64(st))
    assert out == g["outputs"]


@pytest.mark.parametrize("case", _kmeans_golden()["cases"], ids=lambda c: c["why"][:30])
def test_kmeans_golden_cases(case):
    c, lab = oracle.kmeans(np.array(case["x"], float), case["nlist"], case["iters"], init=case["init"])
    assert lab.tolist() == case["assign"]
    assert np.allclose(c, np.array(case["centres"], float), rtol=0, atol=1e-12)


def test_kmeans_init_rows_distinct_and_seeded():
    a = oracle.kmeans_init_rows(500, 40, 7)
    assert len(set(a.tolist())) == 40 and a.min() >= 0 and a.max() < 500
    assert np.array_equal(a, oracle.kmeans_init_rows(500, 40, 7))
    assert not np.array_equal(a, oracle.kmeans_init_rows(500, 40, 8))
    # the prefix property: the first rows of a smaller draw are the same rows
    assert np.array_equal(oracle.kmeans_init_rows(500, 10, 7), a[:10])


def test_kmeans_objective_never_increases():
    """Lloyd's iterations never increase the sum of squared distances to the
    assigned centres (assignment and mean steps each minimise it)."""
    x = sd.lowrank(3000, 16, 71, 72, latent=4, noise=0.2)
    prev = np.inf
    for it in range(0, 6):
        c, lab = oracle.kmeans(x, 12, it, seed=5)
        obj = float(np.sum((x.astype(np.float64) - c[lab]) ** 2))
        assert obj <= prev * (1 + 1e-12)
        prev = obj


def test_kmeans_one_list_per_row_is_the_identity():
    x = np.random.default_rng(3).standard_normal((30, 5))
    c, lab = oracle.kmeans(x, 30, 2, seed=11)
    init = oracle.kmeans_init_rows(30, 30, 11)
    assert np.array_equal(np.sort(lab), np.arange(30))
    assert np.array_equal(c[lab], x)
    assert np.array_equal(lab[init], np.arange(30))


# --------------------------------------------------------------------------
# Section 8, extension (1): cosine similarity and inner product
# --------------------------------------------------------------------------

def test_inner_product_reduction_matches_direct_comparison():
    """With eps0 = +inf the reduced DCO decides <o,q> >= r exactly (away from
    rounding at the boundary) and returns <o,q>."""
    rng = np.random.default_rng(21)
    D = 48
    x = rng.standard_normal((400, D)) * rng.uniform(0.5, 3.0, size=(400, 1))
    x[7] = 0.0                                     # a zero vector
    q = rng.standard_normal(D)
    P = oracle.make_rotation(sd.gaussian_matrix(D, 22))
    ipd = x @ q
    for r in (np.quantile(ipd, 0.9), 0.0, -2.0, np.max(np.linalg.norm(x, axis=1)) * np.linalg.norm(q) * 1.01):
        res = oracle.ip_dco_batch(x, q, np.arange(400), r, P, math.inf, 8)
        clear = np.abs(ipd - r) > 1e-9 * (1 + abs(r))
        assert np.array_equal(res["mask"][clear] == 1, ipd[clear] >= r)
        pos = res["mask"] == 1
        assert np.allclose(res["ip"][pos], ipd[pos], rtol=1e-12, atol=1e-10)
    # unreachable threshold: r above |o||q| can never be met, decided with 0 dims
    res = oracle.ip_dco_batch(x, q, np.arange(400), 1e9, P, 2.1, 8)
    assert res["mask"].sum() == 0 and np.all(res["dims"] == 0)


def test_cosine_search_is_euclidean_search_on_unit_vectors():
    """Cosine search (largest cosine first) equals the Euclidean KNN of the
    normalised vectors (Section 8, extension (1))."""
    x = sd.lowrank(3000, 32, 61, 62, latent=8, noise=0.3)
    q = sd.lowrank(5, 32, 63, 62, latent=8, noise=0.3)
    xu, qu = oracle.normalize(x), oracle.normalize(q)
    ids, dist = oracle.brute_knn(xu.astype(np.float32), qu, 5)
    cos = (xu @ qu.T).T
    for i in range(5):
        top = np.argsort(-cos[i], kind="stable")[:5]
        assert set(top.tolist()) == set(ids[i].tolist())
        assert np.allclose(1 - dist[i] ** 2 / 2, cos[i][ids[i]], atol=1e-6)
