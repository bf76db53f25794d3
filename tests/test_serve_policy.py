"""CPU tests of the serving policy (pure host logic, no GPU): batch formation
in arrival order, joins alone, the size budget with known and estimated
sizes, re-queueing with exact sizes, and first-fit placement of batch outputs
in the id pool (live ranges never overlap)."""

import numpy as np
import pytest

from paper_2309_16913_amd.serve import Admission, IdPool, Pending


def win(k=1):
    return np.tile(np.array([[0.1, 0.1, 0.2, 0.2]], np.float32), (k, 1))


def test_packs_windows_up_to_limit():
    a = Admission(max_windows=4, budget_ids=100)
    for i in range(10):
        a.push(Pending(i, "select", win(), i * 1e-3))
    b = a.next_batch()
    assert [r.rid for r in b.reqs] == [0, 1, 2, 3] and b.windows.shape == (4, 4)
    assert len(a) == 6


def test_batches_hold_one_kind_in_arrival_order():
    a = Admission(max_windows=8, budget_ids=100)
    a.push(Pending(0, "select", win(), 0.0))
    a.push(Pending(1, "join", win(5), 0.0))
    a.push(Pending(2, "select", win(), 0.0))
    a.push(Pending(3, "join", win(3), 0.0))
    a.push(Pending(4, "join", win(2), 0.0))
    b1 = a.next_batch()
    # windows behind a waiting join are packed with the ones before it
    assert b1.kind == "select" and [r.rid for r in b1.reqs] == [0, 2]
    b2 = a.next_batch()
    # join probe sets are packed together up to the window limit (5 + 3 <= 8 < 5 + 3 + 2)
    assert b2.kind == "join" and [r.rid for r in b2.reqs] == [1, 3] and b2.windows.shape[0] == 8
    b3 = a.next_batch()
    assert b3.kind == "join" and [r.rid for r in b3.reqs] == [4]
    assert a.next_batch() is None


def test_estimates_are_kept_per_kind():
    a = Admission(max_windows=100, budget_ids=100)
    a.observe(total=500, nwin=10, kind="select")      # 50 ids per range window
    a.observe(total=1, nwin=100, kind="join")         # 0.01 pairs per probe window
    for i in range(3):
        a.push(Pending(i, "join", win(20), 0.0))
    assert len(a.next_batch().reqs) == 3              # 60 probe windows, ~0.6 pairs expected
    for i in range(3):
        a.push(Pending(10 + i, "select", win(), 0.0))
    assert len(a.next_batch().reqs) == 2              # 2 x 50 <= 100 < 3 x 50


def test_budget_with_known_and_estimated_sizes():
    a = Admission(max_windows=100, budget_ids=100)
    a.observe(total=300, nwin=10)                     # 30 ids per window so far
    for i in range(6):
        a.push(Pending(i, "select", win(), 0.0))
    b = a.next_batch()
    assert [r.rid for r in b.reqs] == [0, 1, 2]       # 3 x 30 <= 100 < 4 x 30
    # known sizes take precedence over the estimate; the first request of a
    # batch is taken whatever its size
    a.queue[0].known_ids = 250
    b = a.next_batch()
    assert [r.rid for r in b.reqs] == [3]
    a.queue[0].known_ids = 5
    a.queue[1].known_ids = 5
    b = a.next_batch()
    assert [r.rid for r in b.reqs] == [4, 5]


def test_requeue_records_exact_sizes_in_order():
    a = Admission(max_windows=8, budget_ids=100)
    for i in range(4):
        a.push(Pending(i, "select", win(2), 0.0))
    a.push(Pending(9, "select", win(), 1.0))
    b = a.next_batch()
    assert len(b.reqs) == 4
    a.requeue(b, np.array([10, 20, 30, 40, 50, 60, 70, 80]), pool_ids=400)
    assert [r.rid for r in a.queue] == [0, 1, 2, 3, 9]
    assert [r.known_ids for r in list(a.queue)[:4]] == [30, 70, 110, 150]
    b1 = a.next_batch()
    assert [r.rid for r in b1.reqs] == [0, 1]         # 30 + 70 <= 100 < + 110


def test_request_larger_than_pool_is_an_error():
    a = Admission(max_windows=8, budget_ids=100)
    a.push(Pending(1, "select", win(), 0.0))
    b = a.next_batch()
    with pytest.raises(MemoryError):
        a.requeue(b, np.array([301]), pool_ids=300)


def test_fifo_order_across_batches():
    a = Admission(max_windows=3, budget_ids=10 ** 9)
    t = 0.0
    for i in range(11):
        t += 1e-4
        a.push(Pending(i, "select", win(), t))
    order = []
    while len(a):
        order += [r.rid for r in a.next_batch().reqs]
    assert order == list(range(11))


def test_unbatched_mode_one_request_per_batch():
    a = Admission(max_windows=64, budget_ids=10 ** 9, one_per_batch=True)
    for i in range(3):
        a.push(Pending(i, "select", win(), 0.0))
    assert [len(a.next_batch().reqs) for _ in range(3)] == [1, 1, 1]


def test_pool_first_fit_never_overlaps():
    rng = np.random.default_rng(5)
    p = IdPool(1000)
    live = {}
    for step in range(3000):
        if live and (rng.random() < 0.5 or len(live) > 6):
            k = list(live)[rng.integers(len(live))]
            s, n = live.pop(k)
            p.free(s, n)
        else:
            n = int(rng.integers(0, 400))
            s = p.alloc(n)
            if s is None:
                # refused only when no gap of n exists
                ends = [0] + [e for _, e in sorted((a, a + b) for a, b in live.values())]
                starts = [a for a, _ in sorted(live.values())] + [1000]
                assert max(b - a for a, b in zip(ends, starts)) < n
                continue
            assert 0 <= s and s + n <= 1000
            for s2, n2 in live.values():
                assert s + n <= s2 or s2 + n2 <= s or n == 0 or n2 == 0
            if n:
                live[step] = (s, n)
        assert p.in_use() == sum(n for _, n in live.values())
