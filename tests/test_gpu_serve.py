"""Served request stream: every result produced under continuous batching
(several batches in flight on several streams, deferral and splitting when the
output pool is short) is identical to the same request run alone."""

import sys

import numpy as np
import pytest

import oracle
import rtgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_served_results_equal_alone():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_16913_amd as rt
    from paper_2309_16913_amd.serve import Server
    big = rtgen.clustered_rects(400_000, 256, 0.005, 5e-5, 5101)
    jt = rtgen.uniform_rects(200_000, 5e-5, 5102)
    tb, tj = rt.build_str(big, 32, "soa"), rt.build_str(jt, 32, "soa")
    reqs = rtgen.c5_requests(3000, rate=3e5, seed_base=5100, join_frac=0.02, probe_n=2000)
    sel = [r for r in reqs if r.kind == "select"]
    wins = np.concatenate([r.payload for r in sel])
    off_all, ids_all = rt.range_select(tb, wins)
    counts = np.diff(off_all.astype(np.int64))
    biggest = int(counts.max())
    # pool: a few times the largest single result, so that batches overflow
    # their slot share and get split, and the largest requests run solo
    pool = max(4 * biggest, 4096)
    say(f"case serve: {len(sel)} windows, biggest result {biggest}, pool {pool}")
    got = {}

    def sink(r, off, ids):
        got[r.rid] = (off.copy(), ids.copy())
    srv = Server(tb, tj, nslots=3, max_windows=2048, pool_ids=pool)
    out = srv.run(reqs, sink=sink)
    say(f"case serve: {out}")
    assert len(got) == len(reqs)
    assert out["overflow_retries"] > 0, "the pool was meant to force deferrals"
    # range requests: identical to the alone results
    for k, r in enumerate(sel):
        off, ids = got[r.rid]
        want = ids_all[int(off_all[k]):int(off_all[k + 1])]
        assert np.array_equal(ids, want), f"request {r.rid}"
        alone = rt.range_select(tb, r.payload)
        assert np.array_equal(alone[1], want)
    # join requests: index nested loop result == synchronized-traversal join
    o = oracle.get()
    for j, r in enumerate([x for x in reqs if x.kind == "join"]):
        off, ids = got[r.rid]
        pairs = np.stack([np.repeat(np.arange(r.payload.shape[0], dtype=np.uint32),
                                    np.diff(off.astype(np.int64))), ids], 1)
        tp = rt.build_str(r.payload, 16, "soa")
        assert np.array_equal(pairs, rt.spatial_join(tp, tj)), f"join request {r.rid}"
        if j == 0:
            assert np.array_equal(pairs, o.join(o.build_str(r.payload, 16), o.build_str(jt, 32)))
