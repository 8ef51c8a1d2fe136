"""Admission policy of the solve server (host logic, no GPU)."""
from collections import deque
from types import SimpleNamespace

from paper_1511_06029_amd.serving import choose_batch


def R(t, k, rid=0):
    return SimpleNamespace(arrival=t, k=k, rid=rid)


def bytes_fn(op, k):
    return 10 * k + (100 if op == "big" else 0)


def test_oldest_operator_first_and_coalescing():
    pending = {"a": deque([R(2.0, 1), R(3.0, 2)]), "b": deque([R(1.0, 4), R(1.5, 4), R(5.0, 1)])}
    op, reqs, k, nb = choose_batch(pending, 0, 10 ** 6, 64, bytes_fn)
    assert op == "b" and k == 9 and len(reqs) == 3 and nb == 90


def test_batch_width_limit_keeps_arrival_order():
    pending = {"a": deque([R(0.0, 5), R(0.1, 5), R(0.2, 5)])}
    op, reqs, k, _ = choose_batch(pending, 0, 10 ** 6, 12, bytes_fn)
    assert k == 10 and [r.arrival for r in reqs] == [0.0, 0.1]


def test_budget_defers_and_skips_to_an_operator_that_fits():
    pending = {"big": deque([R(0.0, 2)]), "a": deque([R(1.0, 1)])}
    # 'big' needs 120 bytes, only 50 left: the later, smaller request is admitted
    op, reqs, k, nb = choose_batch(pending, 950, 1000, 64, bytes_fn)
    assert op == "a" and nb == 10
    # nothing fits at all
    assert choose_batch(pending, 995, 1000, 64, bytes_fn) is None


def test_single_request_wider_than_batch_limit_still_runs():
    pending = {"a": deque([R(0.0, 40)])}
    op, reqs, k, _ = choose_batch(pending, 0, 10 ** 6, 16, bytes_fn)
    assert k == 40 and len(reqs) == 1
