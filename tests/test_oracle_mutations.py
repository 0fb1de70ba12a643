"""Planted mistakes in the oracle must fail its pins.

Each case plants one plausible mistake in a copy of the oracle (a wrong test
formula, a flipped comparison, a sign error, a broken tie rule, a frozen
threshold, a band flag that fires too often or never, a transposed rotation),
builds it on the CPU, and runs the cheap pins of test_oracle_pins.py against
it: at least one pin must fail.  The unmutated oracle passes all of them (the
pins themselves run in the normal suite), so a pass here shows the pins would
catch that mistake.  CPU only; nothing here touches the GPU library.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "ads_oracle.c")).read()
HNSW_SRC = open(os.path.join(os.path.dirname(oracle.__file__), "hnsw_oracle.c")).read()


def _in_function(fn, old, new):
    """Replace the first occurrence of `old` after the definition of `fn`."""
    start = SRC.index(fn)
    i = SRC.index(old, start)
    return SRC[:i] + new + SRC[i + len(old):]


def _once(old, new):
    assert SRC.count(old) == 1, old
    return SRC.replace(old, new)


# name -> mutated C source
C_MUTANTS = {
    "gamma_without_sqrt": lambda: _in_function(
        "int orc_ads_dco", "(1.0 + eps0 / sqrt((double)d)) * r", "(1.0 + eps0 / (double)d) * r"),
    "estimate_without_sqrt_D_over_d": lambda: _in_function(
        "int orc_ads_dco", "sqrt((double)D / (double)d * sq)", "sqrt(sq)"),
    "reject_on_equality": lambda: _in_function(
        "int orc_ads_dco", "reject = dis_approx > (", "reject = dis_approx >= ("),
    "case3_strict_compare": lambda: _in_function(
        "int orc_ads_dco", "if (dis_approx <= r)", "if (dis_approx < r)"),
    "difference_sign_flip": lambda: _in_function(
        "int orc_ads_dco", "double y = o[i] - q[i];", "double y = o[i] + q[i];"),
    "pds_stops_on_equality": lambda: _in_function(
        "int orc_pds_dco", "if (sqrt(sq) > r)", "if (sqrt(sq) >= r)"),
    "heap_ties_to_higher_id": lambda: _once(
        "(a.dis == b.dis && a.id < b.id)", "(a.dis == b.dis && a.id > b.id)"),
    "frozen_threshold": lambda: _once(
        "double r = (hn < K || K == 0) ? INFINITY : heap[0].dis;", "double r = INFINITY;"),
    "band_always_set": lambda: _in_function(
        "int orc_band", "if (isinf(r)) return 0;", "return 1;"),
    "band_never_set": lambda: _in_function(
        "int orc_band", "if (isinf(r)) return 0;", "return 0;"),
    "band_against_r_not_gamma_r": lambda: _in_function(
        "int orc_band", "bound = d < D ? (isinf(eps0) ? INFINITY : (1.0 + eps0 / sqrt((double)d)) * r) : r;",
        "bound = r;"),
    "band_past_the_stopping_point": lambda: _in_function(
        "int orc_band", "if (d < D && est > bound) return 0;", ";"),
}


def _cheap_pins():
    """The pins of test_oracle_pins.py that run in about a second each."""
    g = pins._golden()
    checks = []
    checks += [("ads_golden:" + c["name"], lambda c=c: pins.test_ads_golden_cases(c)) for c in g["ads"]]
    checks += [("pds_golden:" + c["name"], lambda c=c: pins.test_pds_golden_cases(c)) for c in g["pds"]]
    checks += [("band_golden:" + c["name"], lambda c=c: pins.test_band_golden_cases(c)) for c in g["band"]]
    checks += [
        ("exact_case", pins.test_exact_case_returns_raw_space_distance),
        ("no_false_positives", pins.test_no_false_positives_lemma_3_2),
        ("eps_inf_is_fds", pins.test_eps_inf_and_full_block_equal_fdscanning),
        ("pds_exact", pins.test_pdscanning_is_exact),
        ("monotone", pins.test_monotone_in_eps0),
        ("ivf_golden", pins.test_ivf_golden_tiny),
        ("probe_golden", pins.test_probe_selection_golden_ties),
        ("ivf_all_lists_fds", lambda: pins.test_ivf_all_lists_equals_brute_force(oracle.METHOD_FDS)),
        ("ivf_all_lists_ads", lambda: pins.test_ivf_all_lists_equals_brute_force(oracle.METHOD_ADS)),
        ("ivf_ads_trends", pins.test_ivf_ads_keeps_accuracy_and_saves_dims),
        ("rotation_orthogonal", lambda: pins.test_rotation_is_orthogonal_and_preserves_norms(16)),
        ("rotation_orientation", pins.test_rotation_orientation_and_row_sampling_identity),
        ("rotation_haar", pins.test_rotation_is_haar_sign_symmetric),
        ("single_test_beta", pins.test_single_test_failure_probability_matches_beta_law),
    ]
    return checks


def _failing_pins():
    failed = []
    for name, fn in _cheap_pins():
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _with_library(tmp_path, ads_src, hnsw_src, pins_fn):
    a = tmp_path / "mutant_ads.c"
    h = tmp_path / "mutant_hnsw.c"
    a.write_text(ads_src)
    h.write_text(hnsw_src)
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(a), str(h),
                    "-lm", "-lpthread"], check=True)
    saved = oracle._load()
    oracle._lib = oracle.bind(ctypes.CDLL(str(so)))
    try:
        return pins_fn()
    finally:
        oracle._lib = saved


@pytest.mark.parametrize("name", sorted(C_MUTANTS))
def test_planted_c_mistake_fails_a_pin(name, tmp_path):
    failed = _with_library(tmp_path, C_MUTANTS[name](), HNSW_SRC, _failing_pins)
    assert failed, f"mutant {name} passed every pin"


def _hnsw_in_function(fn, old, new):
    start = HNSW_SRC.index(fn)
    i = HNSW_SRC.index(old, start)
    return HNSW_SRC[:i] + new + HNSW_SRC[i + len(old):]


def _hnsw_once(old, new):
    assert HNSW_SRC.count(old) == 1, old
    return HNSW_SRC.replace(old, new)


HNSW_MUTANTS = {
    "pp_threshold_from_r2": lambda: _hnsw_once(
        "double r = job->variant == 2 ? hset_threshold(&R1) : hset_threshold(&R);",
        "double r = hset_threshold(&R);"),
    "pp_rejected_kept_out_of_r2": lambda: _hnsw_once(
        "hset_insert(&R, c.obs, v, exact);", "if (c.positive) hset_insert(&R, c.obs, v, exact);"),
    "pp_observed_without_scale": lambda: _hnsw_in_function(
        "static hdco h_dco", "double est = sqrt((double)D / (double)d * sq);",
        "double est = d < D ? sqrt(sq) : sqrt((double)D / (double)d * sq);"),
    "no_visited_set": lambda: _hnsw_once("if (visited[v]) continue;", ";"),
    "upper_layers_ignore_threshold": lambda: _hnsw_once(
        "hdco c = h_dco(job->base + v * D, q, D, dcur, job->eps0",
        "hdco c = h_dco(job->base + v * D, q, D, INFINITY, job->eps0"),
    "pop_farthest_unexpanded": lambda: _hnsw_once(
        "int p = 0;\n        while (p < R.n && R.e[p].expanded) ++p;\n        if (p == R.n) break;",
        "int p = R.n - 1;\n        while (p >= 0 && R.e[p].expanded) --p;\n        if (p < 0) break;"),
    "ties_to_higher_id": lambda: _hnsw_once(
        "return ka < kb || (ka == kb && ia < ib);", "return ka < kb || (ka == kb && ia > ib);"),
    "positive_strict": lambda: _hnsw_in_function(
        "static hdco h_dco", "out.positive = est <= r;", "out.positive = est < r;"),
    "threshold_before_full": lambda: _hnsw_once(
        "return s->n < s->cap ? INFINITY : s->e[s->n - 1].key;",
        "return s->n > 0 ? s->e[s->n - 1].key : INFINITY;"),
    "evict_nearest": lambda: _hnsw_once(
        "int last = s->n < s->cap ? s->n : s->cap - 1;",
        "if (s->n == s->cap) { for (int i = 0; i + 1 < s->n; ++i) s->e[i] = s->e[i + 1]; s->n--; if (p > 0) p--; }\n    int last = s->n;"),
}


def _hnsw_pins():
    import test_oracle_hnsw as hp
    checks = [("hnsw_golden:" + c["name"], lambda c=c: hp.test_hnsw_golden_tiny(c))
              for c in hp._tiny_cases()]
    checks.append(("hnsw_dco", hp.test_hnsw_dco_is_algorithm_1))
    failed = []
    for name, fn in checks:
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


@pytest.mark.parametrize("name", sorted(HNSW_MUTANTS))
def test_planted_graph_search_mistake_fails_a_pin(name, tmp_path):
    failed = _with_library(tmp_path, SRC, HNSW_MUTANTS[name](), _hnsw_pins)
    assert failed, f"mutant {name} passed every pin"


def _rotate_transposed(x, P64):
    return np.asarray(x, dtype=np.float64) @ P64


def _rotation_without_sign_fix(gaussian):
    q, _ = np.linalg.qr(np.asarray(gaussian, dtype=np.float64))
    return q


def _probes_ties_to_higher_id(q_rot, c_rot, nprobe):
    ids, d2 = _ORIG_PROBES(q_rot, c_rot, nprobe)
    ar = np.arange(d2.shape[1])
    for i in range(d2.shape[0]):
        ids[i] = np.lexsort((-ar, d2[i]))[:nprobe]
    return ids, d2


def _brute_knn_without_recheck(x, queries, K, screen=64, chunk=65536, qchunk=512):
    ids, _ = _ORIG_BRUTE(x, queries, K, screen, chunk, qchunk)
    # float32 GEMM-form scores returned as distances (no difference-form recompute)
    xf = np.asarray(x, dtype=np.float32)
    qf = np.asarray(queries, dtype=np.float32)
    dist = np.empty(ids.shape)
    for i in range(ids.shape[0]):
        s = np.sum(xf[ids[i]] ** 2, axis=1) - np.float32(2) * (xf[ids[i]] @ qf[i]) + qf[i] @ qf[i]
        dist[i] = np.sqrt(np.maximum(s, 0)).astype(np.float64)
    return ids, dist


_ORIG_PROBES = oracle.probes
_ORIG_BRUTE = oracle.brute_knn

PY_MUTANTS = {
    "rotation_transposed": ("rotate", _rotate_transposed),
    "rotation_without_sign_fix": ("make_rotation", _rotation_without_sign_fix),
    "probe_ties_to_higher_id": ("probes", _probes_ties_to_higher_id),
    "ground_truth_in_gemm_form": ("brute_knn", _brute_knn_without_recheck),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_planted_python_mistake_fails_a_pin(name, monkeypatch):
    attr, fn = PY_MUTANTS[name]
    monkeypatch.setattr(oracle, attr, fn)
    extra = []
    if attr == "brute_knn":
        extra = [("brute_knn_full_sort", pins.test_brute_knn_equals_full_sort)]
    failed = _failing_pins()
    for n, f in extra:
        try:
            f()
        except AssertionError:
            failed.append(n)
    assert failed, f"mutant {name} passed every pin"
