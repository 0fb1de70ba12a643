"""Admission logic of the serving loop (host only, fake memory budget)."""

import pytest

from paper_2303_09855_amd.serving import AdmissionController


def cost(n):
    return 1000 + 100 * n          # fixed part + per-request bytes


def test_admits_full_batch_when_it_fits():
    a = AdmissionController(budget_bytes=10**9, max_batch=512, max_inflight=2)
    assert a.admit(1000, 0, 0, cost) == 512
    assert a.admit(37, 1, 0, cost) == 37


def test_memory_budget_limits_the_batch():
    a = AdmissionController(budget_bytes=1000 + 100 * 50, max_batch=512, max_inflight=4)
    assert a.admit(400, 0, 0, cost) == 50
    # memory held by in-flight batches shrinks what is admitted
    assert a.admit(400, 1, 100 * 20, cost) == 30
    # nothing fits: wait
    assert a.admit(400, 1, 100 * 50, cost) == 0


def test_stream_slots_and_empty_queue():
    a = AdmissionController(budget_bytes=10**9, max_batch=64, max_inflight=2)
    assert a.admit(10, 2, 0, cost) == 0
    assert a.admit(0, 0, 0, cost) == 0


def test_rejects_bad_configuration():
    with pytest.raises(ValueError):
        AdmissionController(0)


def test_k_classes_are_powers_of_two():
    from paper_2303_09855_amd.serving import Server
    assert [Server.k_class(k) for k in (1, 2, 3, 10, 16, 17, 100)] == [1, 2, 4, 16, 16, 32, 128]
