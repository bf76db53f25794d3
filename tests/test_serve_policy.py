"""CPU tests of the serving admission policy (pure host logic, no GPU): batch
formation, joins alone, deferral and splitting on overflow, solo requests."""

import numpy as np
import pytest

from paper_2309_16913_amd.serve import Admission, Pending


def win(k=1):
    return np.tile(np.array([[0.1, 0.1, 0.2, 0.2]], np.float32), (k, 1))


def test_packs_windows_up_to_limit():
    a = Admission(max_windows=4, slot_ids=100, pool_ids=300)
    for i in range(10):
        a.push(Pending(i, "select", win(), i * 1e-3))
    b = a.next_batch(all_idle=True)
    assert [r.rid for r in b.reqs] == [0, 1, 2, 3] and b.windows.shape == (4, 4)
    assert len(a) == 6


def test_join_runs_alone_and_does_not_block_windows():
    a = Admission(max_windows=8, slot_ids=100, pool_ids=300)
    a.push(Pending(0, "select", win(), 0.0))
    a.push(Pending(1, "join", win(5), 0.0))
    a.push(Pending(2, "select", win(), 0.0))
    b1 = a.next_batch(True)
    # windows behind a waiting join are packed with the ones before it
    assert b1.kind == "select" and [r.rid for r in b1.reqs] == [0, 2]
    b2 = a.next_batch(True)
    assert b2.kind == "join" and [r.rid for r in b2.reqs] == [1] and b2.windows.shape[0] == 5
    assert a.next_batch(True) is None


def test_overflow_defers_and_splits_never_drops():
    a = Admission(max_windows=8, slot_ids=100, pool_ids=300)
    for i in range(4):
        a.push(Pending(i, "select", win(), 0.0))
    b = a.next_batch(True)
    assert len(b.reqs) == 4
    # the device reported these per-window counts: total 240 > slot (100)
    a.overflowed(b, np.array([60, 60, 60, 60]))
    assert len(a) == 4
    b1 = a.next_batch(True)
    assert [r.rid for r in b1.reqs] == [0]           # 60 + 60 > 100: one per batch
    b2 = a.next_batch(True)
    assert [r.rid for r in b2.reqs] == [1]
    assert all(r.known_ids == 60 for r in b1.reqs + b2.reqs)


def test_oversized_request_goes_solo_when_idle():
    a = Admission(max_windows=8, slot_ids=100, pool_ids=300)
    a.push(Pending(7, "select", win(), 0.0))
    b = a.next_batch(True)
    a.overflowed(b, np.array([250]))
    assert a.queue[0].solo
    assert a.next_batch(all_idle=False) is None      # waits for every slot to drain
    b = a.next_batch(all_idle=True)
    assert b.whole_pool and [r.rid for r in b.reqs] == [7]


def test_request_larger_than_pool_is_an_error():
    a = Admission(max_windows=8, slot_ids=100, pool_ids=300)
    a.push(Pending(1, "select", win(), 0.0))
    b = a.next_batch(True)
    with pytest.raises(MemoryError):
        a.overflowed(b, np.array([301]))


def test_fake_clock_fifo_order():
    """Arrival order is preserved across batches (first come, first served)."""
    a = Admission(max_windows=3, slot_ids=10 ** 9, pool_ids=10 ** 9)
    t = 0.0
    order = []
    for i in range(11):
        t += 1e-4
        a.push(Pending(i, "select", win(), t))
    while len(a):
        b = a.next_batch(True)
        order += [r.rid for r in b.reqs]
    assert order == list(range(11))
