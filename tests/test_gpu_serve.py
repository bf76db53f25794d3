"""Served request stream: every result produced under continuous batching
(several batches in flight on several streams, count-first admission into a
small output pool: batches wait for room, get re-queued with exact sizes,
and single requests larger than a batch's share) equals the CPU oracle's
result for that request and the result of the request run alone."""

import sys

import numpy as np
import pytest

import oracle
import rtgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_served_results_equal_oracle_and_alone():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_16913_amd as rt
    from paper_2309_16913_amd.serve import Server
    o = oracle.get()
    big = rtgen.clustered_rects(400_000, 256, 0.005, 5e-5, 5101)
    jt = rtgen.uniform_rects(200_000, 5e-5, 5102)
    tb, tj = rt.build_str(big, 32, "soa"), rt.build_str(jt, 32, "soa")
    reqs = rtgen.c5_requests(3000, rate=3e5, seed_base=5100, join_frac=0.02, probe_n=2000)
    sel = [r for r in reqs if r.kind == "select"]
    wins = np.concatenate([r.payload for r in sel])
    # the oracle's answer for every range request
    woff, wids = o.select(o.build_str(big, 32), wins)
    counts = np.diff(woff.astype(np.int64))
    biggest = int(counts.max())
    # pool: 2.5 x the largest single result, so batches wait for room, the
    # first (unsized) batches exceed the whole pool and come back with exact
    # sizes, and the largest requests exceed one batch's share (pool / 3)
    pool = max(int(2.5 * biggest), 4096)
    say(f"case serve: {len(sel)} windows, biggest result {biggest}, pool {pool}")
    got = {}

    def sink(r, off, ids):
        got[r.rid] = (off.copy(), ids.copy())
    srv = Server(tb, tj, nslots=3, max_windows=2048, pool_ids=pool)
    # every request has arrived at the start (arrival times scaled to ~0): the
    # first batch is a full, unsized one of max_windows windows, whatever the
    # machine's launch latencies, so it exceeds the pool and is re-queued
    out = srv.run(reqs, sink=sink, time_scale=1e-9)
    say(f"case serve: {out}")
    assert len(got) == len(reqs)
    assert out["requeued_batches"] > 0, "the first batches were meant to exceed the pool"
    assert out["memory_waits"] > 0, "the pool was meant to make batches wait"
    assert out["oversized_batches"] > 0, "requests over a batch's share were meant to run"
    # range requests: identical to the oracle, and to the request run alone
    alone_off, alone_ids = rt.range_select(tb, wins)
    for k, r in enumerate(sel):
        off, ids = got[r.rid]
        want = wids[int(woff[k]):int(woff[k + 1])]
        assert off.tolist() == [0, want.shape[0]], f"request {r.rid} offsets"
        assert np.array_equal(ids, want), f"request {r.rid} differs from the oracle"
        alone = alone_ids[int(alone_off[k]):int(alone_off[k + 1])]
        assert np.array_equal(alone, want), f"request {r.rid} alone differs from the oracle"
    # join requests: index nested loop result == the oracle's join ==
    # the synchronized-traversal join on a probe tree
    oj = o.build_str(jt, 32)
    joins = [x for x in reqs if x.kind == "join"]
    assert joins
    for r in joins:
        off, ids = got[r.rid]
        pairs = np.stack([np.repeat(np.arange(r.payload.shape[0], dtype=np.uint32),
                                    np.diff(off.astype(np.int64))), ids], 1)
        assert np.array_equal(pairs, o.join(o.build_str(r.payload, 16), oj)), f"join request {r.rid} vs oracle"
        tp = rt.build_str(r.payload, 16, "soa")
        assert np.array_equal(pairs, rt.spatial_join(tp, tj)), f"join request {r.rid} vs rt_spatial_join"


def test_served_unbatched_and_large_pool():
    """The unbatched baseline (one request per launch) and a pool large
    enough that nothing waits give the same results as the oracle."""
    import torch
    assert torch.cuda.is_available()
    import paper_2309_16913_amd as rt
    from paper_2309_16913_amd.serve import Server
    o = oracle.get()
    big = rtgen.clustered_rects(200_000, 64, 0.01, 5e-5, 5111)
    jt = rtgen.uniform_rects(50_000, 5e-5, 5112)
    tb, tj = rt.build_str(big, 16, "aos"), rt.build_str(jt, 64, "d2")
    reqs = rtgen.c5_requests(400, rate=1e5, seed_base=5110, join_frac=0.02, probe_n=500)
    ot, oj = o.build_str(big, 16), o.build_str(jt, 16)
    for kw in (dict(nslots=1, one_per_batch=True), dict(nslots=4, pool_ids=1 << 24)):
        say(f"case serve {kw}")
        got = {}

        def sink(r, off, ids):
            got[r.rid] = (off.copy(), ids.copy())
        out = Server(tb, tj, max_windows=1024, **kw).run(reqs, sink=sink)
        assert len(got) == len(reqs) and out["requeued_batches"] == 0
        for r in reqs:
            off, ids = got[r.rid]
            wo, wi = o.select(ot if r.kind == "select" else oj, r.payload)
            assert np.array_equal(off.astype(np.uint64), wo) and np.array_equal(ids, wi), (kw, r.rid)
