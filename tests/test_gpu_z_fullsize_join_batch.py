"""Full-size parity of the other benchmarked configurations, in the launch
configurations the benchmark times:

* the 2M uniform x 2M clustered spatial join (fanout 32, SoA, nodes sorted by
  low x): every pair against the oracle's join, and every expansion variant
  against the default;
* the 256-instance batch (sizes log-uniform in [1e3, 1e6], 4.0M windows),
  trees built with the fanout and layout chosen per size class, replayed
  from its graph: a seeded sample of windows of every tree against the
  oracle, and for all ids strict ascent per window and intersection with the
  window; the plain per-tree launches give the same bytes;
* the 50M-rectangle clustered serving tree (fanout 32, SoA): a sample of the
  served window mix against the oracle, all ids checked for ascent and
  intersection."""

import hashlib
import sys

import numpy as np
import pytest

import oracle
import rtgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_csr_properties(rects, windows, off, ids, what, chunk=1 << 24):
    """Every id intersects its window; ids strictly ascend within a window
    (checked over runs of whole windows of about `chunk` ids)."""
    off = off.astype(np.int64)
    nq = windows.shape[0]
    assert off[0] == 0 and off[-1] == ids.size and np.all(np.diff(off) >= 0), what
    if ids.size == 0:
        return
    assert int(ids.max()) < rects.shape[0], what
    q0 = 0
    while q0 < nq:
        q1 = int(np.searchsorted(off, off[q0] + chunk, side="right")) - 1
        q1 = min(max(q1, q0 + 1), nq)
        a, b = int(off[q0]), int(off[q1])
        part = ids[a:b]
        qi = np.repeat(np.arange(q0, q1), np.diff(off[q0:q1 + 1]))
        e = rects[part]
        w = windows[qi]
        ok = (e[:, 0] <= w[:, 2]) & (w[:, 0] <= e[:, 2]) & (e[:, 1] <= w[:, 3]) & (w[:, 1] <= e[:, 3])
        assert ok.all(), f"{what}: an id does not intersect its window"
        d = np.diff(part.astype(np.int64))
        same = qi[1:] == qi[:-1]
        assert np.all((d > 0) | ~same), f"{what}: ids not strictly ascending within a window"
        q0 = q1


def test_fullsize_join_c3():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_16913_amd as rt
    o = oracle.get()
    say("case fullsize join: 2M uniform x 2M clustered, F32 SoA sorted")
    a, b = rtgen.c3_join()
    ta = rt.build_str(a, 32, "soa", sort_lx=True)
    tb = rt.build_str(b, 32, "soa", sort_lx=True)
    want = o.join_mt(o.build_str(a, 32), o.build_str(b, 32), 8)
    say(f"case fullsize join: oracle {want.shape[0]} pairs")
    got = rt.spatial_join(ta, tb)
    assert np.array_equal(got, want), "host-output join differs from the oracle"
    n = rt.spatial_join_device(ta, tb, 0, 0)
    assert n == want.shape[0]
    buf = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    ref = torch.from_numpy(want.view(np.int32).reshape(-1)).cuda()
    for name, fl in [("default", None), ("tile", rt.JOIN_TILE), ("cand", 0), ("O3", rt.JOIN_O3),
                     ("O3+O4", rt.JOIN_O3 | rt.JOIN_O4), ("O3+O5", rt.JOIN_O3 | rt.JOIN_O5), ("O5", rt.JOIN_O5),
                     ("O3+O5+LB", rt.JOIN_O3 | rt.JOIN_O5 | rt.JOIN_LB)]:
        for rep in range(2):   # the second call of a repeated join replays its graph
            buf.fill_(-1)
            assert rt.spatial_join_device(ta, tb, buf.data_ptr(), n, fl) == n
            torch.cuda.synchronize()
            assert torch.equal(buf, ref), f"device join variant {name} (call {rep}) differs from the oracle"


def _digest(off, ids):
    h = hashlib.blake2b(digest_size=16)
    h.update(np.ascontiguousarray(off).tobytes())
    h.update(np.ascontiguousarray(ids).tobytes())
    return h.hexdigest()


def test_fullsize_batch_c4():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_16913_amd as rt
    o = oracle.get()
    say("case fullsize batch: 256 instances")
    inst = rtgen.c4_batch()
    # the benchmark's configuration: fanout and layout per size class, timed
    # in batch context
    from paper_2309_16913_amd.autotune import BatchTuner
    tuner = BatchTuner(reps=1)
    trees = tuner.build(inst, tuner.tune(inst))
    b = rt.Batch(trees, [x.queries for x in inst])
    b.run()
    torch.cuda.synchronize()
    total, flags = b.status()
    assert flags == 0
    chunks, over = b.replay_info()
    assert chunks > 0 and not over, "the graph's fill did not replay the count pass's records"
    g = np.random.Generator(np.random.PCG64(4242))
    digests = []
    seen = 0
    for i, x in enumerate(inst):
        off, ids = b.result(i)
        assert off.shape[0] == x.queries.shape[0] + 1
        seen += int(off[-1])
        _check_csr_properties(x.rects, x.queries, off, ids, f"tree {i}")
        k = min(16, x.queries.shape[0])
        pick = np.sort(g.choice(x.queries.shape[0], size=k, replace=False))
        woff, wids = o.select(o.build_str(x.rects, 16), x.queries[pick])
        for j, qi in enumerate(pick):
            got = ids[int(off[qi]):int(off[qi + 1])]
            want = wids[int(woff[j]):int(woff[j + 1])]
            assert np.array_equal(got, want), f"tree {i} window {qi}: {got.size} vs {want.size} ids"
        digests.append(_digest(off, ids))
    assert seen == total
    say(f"case fullsize batch: {total} ids checked; plain per-tree launches")
    b.run_plain()
    torch.cuda.synchronize()
    assert b.status() == (total, 0)
    for i in range(len(inst)):
        off, ids = b.result(i)
        assert _digest(off, ids) == digests[i], f"tree {i}: plain launches differ from the graph replay"


def test_fullsize_serving_tree_c5():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_16913_amd as rt
    o = oracle.get()
    say("case fullsize serving tree: 50M clustered, F32 SoA")
    big, _ = rtgen.c5_trees(n_join=1)
    t = rt.build_str(big, 32, "soa")
    t.set_split(16)   # the server's mapping
    q = rtgen.windows_loguniform(8_000, 1e-7, 1e-2, 5006)
    nq = q.shape[0]
    dq = torch.from_numpy(q).cuda()
    off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    dt = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert not rt.range_select_async(t, dq.data_ptr(), nq, off.data_ptr(), 0, 0, dt.data_ptr(), s)
    total = int(dt.item())
    ids = torch.empty(total, dtype=torch.int32, device="cuda")
    assert rt.range_select_async(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), total, dt.data_ptr(), s)
    torch.cuda.synchronize()
    assert int(dt.item()) == total
    hoff = off.cpu().numpy()
    hids = ids.cpu().numpy().view(np.uint32)
    say(f"case fullsize serving tree: {total} ids")
    _check_csr_properties(big, q, hoff, hids, "50M tree")
    # the one-call select with the record replay (the closed loop's path)
    # gives the same bytes
    wb = rt.select_replay_workspace_bytes(nq, total)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    st = torch.zeros(2, dtype=torch.int64, device="cuda")
    off2 = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    ids2 = torch.empty(total, dtype=torch.int32, device="cuda")
    rt.range_select_device(t, dq.data_ptr(), nq, off2.data_ptr(), ids2.data_ptr(), total, work.data_ptr(), wb,
                           st.data_ptr(), s)
    torch.cuda.synchronize()
    chunks, over = rt.select_replay_info(work.data_ptr())
    say(f"case fullsize serving tree: replay {chunks} record chunks, overflow {over}")
    assert chunks > 0 and not over and st.cpu().tolist() == [total, 0]
    assert torch.equal(off2, off) and torch.equal(ids2, ids)
    del work, off2, ids2
    g = np.random.Generator(np.random.PCG64(5055))
    pick = np.sort(g.choice(nq, size=400, replace=False))
    woff, wids = o.select(o.build_str(big, 32), q[pick])
    for j, qi in enumerate(pick):
        got = hids[int(hoff[qi]):int(hoff[qi + 1])]
        want = wids[int(woff[j]):int(woff[j + 1])]
        assert np.array_equal(got, want), f"window {qi}: {got.size} vs {want.size} ids"
