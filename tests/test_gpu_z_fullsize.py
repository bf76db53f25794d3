"""Full-size range select in the launch configuration the benchmark times:
10M rectangles (half uniform, half clustered), 1M windows with selectivity
log-uniform in [1e-6, 1e-3], device-pointer entry point, for fanout 32 SoA
(fill walking the tree), fanout 64 SoA and AoS (the configurations the
benchmark's tuner picks among) and fanout 16 in the third layout (fill
replaying the count pass's records, as the benchmark runs it).

The oracle computes a random sample of queries one by one (exact equality);
for every query the output is checked for properties that hold at any size:
ids strictly ascending within each query, every id intersects its window,
and the totals agree with the count-only entry point."""

import sys

import numpy as np
import pytest

import oracle
import rtgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c2_data():
    say("case fullsize: generating 10M rectangles, 1M windows")
    return rtgen.c2_rects(), rtgen.c2_queries()


@pytest.mark.parametrize("fanout,layout,nsample,replay", [(32, "soa", 2000, False), (64, "soa", 1000, True),
                                                          (64, "aos", 1000, True), (16, "d2", 500, True)])
def test_fullsize_select_bench_config(c2_data, fanout, layout, nsample, replay):
    import torch
    assert torch.cuda.is_available()
    import paper_2309_16913_amd as rt
    rects, queries = c2_data
    nq = queries.shape[0]
    say(f"case fullsize: F{fanout} {layout}")
    tree = rt.build_str(rects, fanout, layout)
    dq = torch.from_numpy(queries).cuda()
    counts = torch.empty(nq, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    wb0 = rt.select_workspace_bytes(nq, 0)
    work0 = torch.empty(wb0, dtype=torch.uint8, device="cuda")
    rt.range_count_device(tree, dq.data_ptr(), nq, counts.data_ptr(), work0.data_ptr(), wb0, s.cuda_stream)
    torch.cuda.synchronize()
    cap = int(counts.to(torch.int64).sum().item())
    del work0
    say(f"case fullsize: {cap} ids")
    off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    ids = torch.empty(cap, dtype=torch.int32, device="cuda")
    # the benchmark's workspace: with room for the count pass's records, the
    # fill replays them
    wb = (rt.select_replay_workspace_bytes if replay else rt.select_workspace_bytes)(nq, cap)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    st = torch.zeros(2, dtype=torch.int64, device="cuda")
    rt.range_select_device(tree, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), cap, work.data_ptr(), wb,
                           st.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    chunks, over = rt.select_replay_info(work.data_ptr())
    assert (chunks > 0 and not over) if replay else chunks == 0
    say(f"case fullsize: replay {replay}, {chunks} record chunks")
    del work
    stat = st.cpu().numpy()
    assert stat[0] == cap and stat[1] == 0
    # totals agree with the count-only pass, query by query
    assert torch.equal(off[1:] - off[:-1], counts.to(torch.int64))
    # properties over every id, on the GPU in chunks
    say("case fullsize: property checks")
    dr = torch.from_numpy(rects).cuda()
    lens = (off[1:] - off[:-1])
    qidx = torch.repeat_interleave(torch.arange(nq, device="cuda", dtype=torch.int32), lens)
    chunk = 1 << 24
    for c0 in range(0, cap, chunk):
        c1 = min(cap, c0 + chunk)
        i = ids[c0:c1].to(torch.int64)
        qq = qidx[c0:c1].to(torch.int64)
        assert int(i.min()) >= 0 and int(i.max()) < rects.shape[0]
        e = dr[i]
        w = dq[qq]
        ok = (e[:, 0] <= w[:, 2]) & (w[:, 0] <= e[:, 2]) & (e[:, 1] <= w[:, 3]) & (w[:, 1] <= e[:, 3])
        assert bool(ok.all()), "an id does not intersect its window"
        if c1 - c0 > 1:
            same = qq[1:] == qq[:-1]
            inc = i[1:] > i[:-1]
            assert bool((inc | ~same).all()), "ids not strictly ascending within a query"
        del i, qq, e, w, ok
    del qidx
    # exact equality with the oracle on a sample of queries
    say("case fullsize: oracle sample")
    o = oracle.get()
    ot = o.build_str(rects, fanout)
    g = np.random.Generator(np.random.PCG64(77 + fanout))
    sample = np.sort(g.choice(nq, size=nsample, replace=False))
    woff, wids = o.select(ot, queries[sample])
    hoff = off.cpu().numpy()
    for k, qi in enumerate(sample):
        a0, a1 = int(hoff[qi]), int(hoff[qi + 1])
        got = ids[a0:a1].cpu().numpy().view(np.uint32)
        want = wids[int(woff[k]):int(woff[k + 1])]
        assert np.array_equal(got, want), f"query {qi}: {got.size} vs {want.size} ids"
    tree.free()
