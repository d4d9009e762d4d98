"""Admission policy of the continuous server (host logic, no GPU): how the
waiting requests, in arrival order, are dealt to the free slots."""
import pytest

pytest.importorskip("torch")
from paper_1705_03524_amd.serving import admit  # noqa: E402

ROOMY = (1 << 40, 1 << 30, 1 << 30, 4096)   # (workspace, crop bytes, map floats, centre ints)


def need(ws=1, crop=1, out=1, cen=6):
    return (ws, crop, out, cen)


def test_light_load_one_request_per_slot():
    assert admit([need()] * 2, 3, ROOMY, 64) == [1, 1]
    assert admit([need()] * 3, 3, ROOMY, 64) == [1, 1, 1]


def test_heavier_load_is_spread_evenly():
    # shares ceil(7/3) = 3, then ceil(4/2) = 2, then 2
    assert admit([need()] * 7, 3, ROOMY, 64) == [3, 2, 2]
    # one free slot takes everything that waits (up to max_batch)
    assert admit([need()] * 4, 1, ROOMY, 64) == [4]


def test_max_batch_caps_a_slot():
    assert admit([need()] * 10, 2, ROOMY, 3) == [3, 3]


def test_capacities_bound_a_slot():
    limits = (10, 1 << 30, 1 << 30, 4096)
    # share would be 2, but two 6-byte workspaces do not fit one 10-byte slot
    assert admit([need(ws=6)] * 5, 3, limits, 64) == [1, 1, 1]
    # the staged centres bound it too (6 ints per three-scale request)
    assert admit([need(cen=6)] * 5, 1, (1 << 40, 1 << 30, 1 << 30, 12), 64) == [2]
    # a large request ends a slot's share; the next slot starts with it, and
    # what does not fit beside it waits for the next admission
    assert admit([need(ws=2), need(ws=9), need(ws=2), need(ws=2)], 2, limits, 64) == [1, 1]
    assert admit([need(ws=2), need(ws=7), need(ws=2), need(ws=2)], 2, limits, 64) == [2, 2]


def test_without_direct_single_everything_goes_to_one_slot():
    assert admit([need()] * 5, 3, ROOMY, 64, direct_single=False) == [5]
    assert admit([need()] * 5, 3, ROOMY, 2, direct_single=False) == [2, 2, 1]


def test_counts_never_exceed_what_waits():
    for n in range(0, 12):
        for nfree in range(1, 5):
            out = admit([need()] * n, nfree, ROOMY, 4)
            assert sum(out) <= n and len(out) <= nfree and all(c >= 1 for c in out)
            if n:
                assert sum(out) == min(n, 4 * nfree) if n > nfree else out == [1] * n


def test_a_request_larger_than_a_slot_is_refused():
    with pytest.raises(ValueError):
        admit([need(ws=11)], 1, (10, 1 << 30, 1 << 30, 4096), 64, direct_single=False)


def test_work_cap_keeps_large_requests_apart():
    big, small = need(ws=13), need(ws=3)
    # nothing in flight: the first large request starts, the second waits
    assert admit([big, big], 3, ROOMY, 64, busy=0, work_cap=20) == [1]
    # a small one may join a large one in flight; a large one may not
    assert admit([small], 3, ROOMY, 64, busy=13, work_cap=20) == [1]
    assert admit([big], 3, ROOMY, 64, busy=13, work_cap=20) == []
    # a request larger than the cap still runs alone when nothing is in flight
    assert admit([need(ws=30)], 3, ROOMY, 64, busy=0, work_cap=20) == [1]
    # heavier load: shares stop at the cap, the rest waits
    assert admit([small] * 9, 2, ROOMY, 64, busy=0, work_cap=20) == [5, 1]
    assert admit([small] * 9, 2, ROOMY, 64, busy=18, work_cap=20) == []


def test_work_cap_always_admits_when_idle():
    for n in range(1, 9):
        for ws in (1, 7, 25):
            out = admit([need(ws=ws)] * n, 3, ROOMY, 64, busy=0, work_cap=20)
            assert out and sum(out) >= 1
