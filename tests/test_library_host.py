"""CPU-side checks of the C ABI library: it loads, exports every entry point
include/ads.h declares, its host-only QR matches the oracle's, and argument
validation rejects bad calls before anything touches a GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synthdata as sd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ads():
    import paper_2303_09855_amd as m
    m.load()
    return m


def declared_symbols():
    with open(os.path.join(ROOT, "include", "ads.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(ads_[a-z_0-9]+)\(", text, re.M)))


def test_header_declares_the_binding_surface(ads):
    assert declared_symbols() == sorted(ads.EXPORTED)


def test_library_exports_every_declared_symbol(ads):
    lib = ads.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert "gfx950" in ads.version()


@pytest.mark.parametrize("D", [8, 128, 960])
def test_host_rotation_matches_oracle_qr(ads, D):
    G = sd.gaussian_matrix(D, 1001)
    P32, P64 = ads.make_rotation(G)
    ref = oracle.make_rotation(G)
    assert np.max(np.abs(P64 - ref)) < 1e-12
    assert np.max(np.abs(P32.astype(np.float64) - ref)) < 1e-7
    assert np.max(np.abs(P64.T @ P64 - np.eye(D))) < 1e-12


def test_rotation_rejects_bad_arguments(ads):
    lib = ads.load()
    out = np.zeros(4, dtype=np.float32)
    assert lib.ads_make_rotation(None, 2, out.ctypes.data_as(ctypes.c_void_p), None) == -1
    g = np.zeros((2, 2))
    assert lib.ads_make_rotation(g.ctypes.data_as(ctypes.c_void_p), 0, out.ctypes.data_as(ctypes.c_void_p), None) == -1
    assert "D must be" in ads.last_error()


def test_calls_validate_before_launching(ads):
    lib = ads.load()
    # NULL index / pointers are rejected on the host with a message
    assert lib.ads_search(None, None, 1, None, None, 10, 1, 2.1, 0, 0, None, None, None, None, None, None) == -1
    assert "index is NULL" in ads.last_error()
    assert lib.ads_dco_batch(None, None, None, 1, 1.0, 2.1, 32, 0, 0, None, None, None, None, None) == -1
    out = ctypes.c_void_p()
    assert lib.ads_ivf_build(None, 10, 128, None, None, 4, None, 32, 0, 1, 0, None, ctypes.byref(out)) == -1
    assert "must not be NULL" in ads.last_error()
    assert lib.ads_rotate(None, 128, None, 0, None, None) == 0   # n == 0 is a no-op
    assert lib.ads_rotate(None, 128, None, 5, None, None) == -1
    assert lib.ads_index_info(None, None) == -1
    assert lib.ads_index_free(None) == 0
    assert lib.ads_search_workspace_size(None, 1, 10, 1, 0) == 0


def test_tuning_knobs_validate_and_round_trip(ads):
    saved = ads.get_tuning()
    assert saved["prefetch_units"] == 0 and saved["dense_frac"] == 0.0
    try:
        ads.set_tuning(prefetch_units=1, queries_per_unit=16, sweep_log2=2)
        t = ads.get_tuning()
        assert (t["prefetch_units"], t["queries_per_unit"], t["sweep_log2"]) == (1, 16, 2)
        for bad in ({"prefetch_units": -1}, {"dense_frac": 0.5}, {"dense_frac": -0.1}, {"queries_per_unit": 3},
                    {"sweep_log2": 7}, {"grid_per_xcd": -1}):
            with pytest.raises(ads.AdsError):
                ads.set_tuning(**bad)
        with pytest.raises(ValueError):
            ads.set_tuning(no_such_knob=1)
    finally:
        ads.set_tuning(**saved)
    assert ads.get_tuning() == saved


def _graph_call(lib, levels, adj0, up_off, up_adj, M0, M, entry, D=64, delta_d=16, rows=None):
    levels = np.ascontiguousarray(levels, dtype=np.int32)
    adj0 = np.ascontiguousarray(adj0, dtype=np.int32)
    up_off = np.ascontiguousarray(up_off, dtype=np.int64)
    up_adj = np.ascontiguousarray(up_adj, dtype=np.int32)
    out = ctypes.c_void_p()
    fake_base = ctypes.c_void_p(4096)       # never dereferenced: validation fails first
    return lib.ads_hnsw_create(fake_base, len(levels), D, None, levels.ctypes.data, adj0.ctypes.data, M0,
                               up_off.ctypes.data, up_adj.ctypes.data,
                               up_adj.shape[0] if rows is None else rows, M, entry, delta_d, None,
                               ctypes.byref(out))


def test_graph_index_validates_the_graph_on_the_host(ads):
    """ads_hnsw_create checks every row before it allocates or copies anything:
    ids in range, -1 padding only at the end of a row, no duplicates, upper
    neighbours present on their layer, the entry on the top layer, shapes the
    kernels support."""
    lib = ads.load()
    levels = [1, 0, 0, 1]
    adj0 = [[1, 2, -1], [0, 3, -1], [3, 0, -1], [2, 1, -1]]
    up_off = [0, -1, -1, 1]
    up_adj = [[3, -1], [0, -1]]
    bad = [
        (dict(adj0=[[1, 2, -1], [0, 4, -1], [3, 0, -1], [2, 1, -1]]), "out of range"),
        (dict(adj0=[[1, -1, 2], [0, 3, -1], [3, 0, -1], [2, 1, -1]]), "after -1 padding"),
        (dict(adj0=[[1, 1, -1], [0, 3, -1], [3, 0, -1], [2, 1, -1]]), "duplicate"),
        (dict(adj0=[[1, 2, -2], [0, 3, -1], [3, 0, -1], [2, 1, -1]]), "neighbour id"),
        (dict(up_adj=[[1, -1], [0, -1]]), "not on that layer"),
        (dict(up_off=[0, -1, -1, 5]), "upper rows"),
        (dict(entry=1), "level"),
        (dict(entry=9), "entry"),
        (dict(D=48), "multiple of 32"),
        (dict(delta_d=64), "delta_d"),
        (dict(M0=40), "M0"),
    ]
    for change, msg in bad:
        args = dict(levels=levels, adj0=adj0, up_off=up_off, up_adj=up_adj, M0=3, M=2, entry=0)
        args.update(change)
        if args["M0"] != 3:
            args["adj0"] = np.full((4, args["M0"]), -1)
        assert _graph_call(lib, **args) == -1, change
        assert msg in ads.last_error(), (change, ads.last_error())
    # search-side checks need no device either
    assert lib.ads_hnsw_search(None, None, 1, 10, 10, 2.1, 0, None, None, None, None, None, None) == -1
    assert lib.ads_hnsw_workspace_size(None, 4) == 0
    assert lib.ads_hnsw_free(None) == 0
