"""GPU parity of the stream-ordered boundary calls against the CPU oracle:
rt_range_select_async (library-held workspace, RT_ENOMEM without touching
the ids buffer), the two-stage device select (count stage, then fill stage
on the same workspace), and the library's own choice of fanout and layout
(fanout 0, RT_LAYOUT_AUTO)."""

import sys

import numpy as np
import pytest

import oracle
import rtgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    import paper_2309_16913_amd as m
    return m


@pytest.fixture(scope="module")
def ora():
    return oracle.get()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _csr_equal(go, gi, wo, wi, what):
    assert np.array_equal(go.astype(np.uint64), wo), f"{what}: offsets differ"
    assert np.array_equal(gi.view(np.uint32), wi), f"{what}: ids differ"


@pytest.mark.parametrize("fanout,layout,nq", [(16, "soa", 3000), (32, "aos", 9000), (64, "d2", 20000)])
def test_select_async_matches_oracle(rt, ora, fanout, layout, nq):
    import torch
    say(f"case select_async F={fanout} {layout} nq={nq}")
    r = rtgen.clustered_rects(150_000, 16, 0.02, 2e-3, 501 + fanout)
    q = rtgen.windows_loguniform(nq, 1e-7, 1e-3, 502 + fanout)
    t = rt.build_str(r, fanout, layout)
    wo, wi = ora.select(ora.build_str(r, fanout), q)
    total = int(wo[-1])
    dq = torch.from_numpy(q).cuda()
    off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    dt = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    # too small by one: refused, the ids buffer keeps its contents
    ids = torch.full((total + 8,), -7, dtype=torch.int32, device="cuda")
    ok = rt.range_select_async(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), total - 1, dt.data_ptr(),
                               s.cuda_stream)
    s.synchronize()
    assert not ok
    assert int(dt.item()) == total
    assert bool((ids == -7).all().item()), "the refused call wrote ids"
    assert np.array_equal(off.cpu().numpy().astype(np.uint64), wo), "offsets of the refused call"
    # exactly large enough, twice in a row on two streams
    s2 = torch.cuda.Stream()
    ids2 = torch.full((total + 8,), -7, dtype=torch.int32, device="cuda")
    off2 = torch.empty_like(off)
    dt2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert rt.range_select_async(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), total, dt.data_ptr(),
                                 s.cuda_stream)
    assert rt.range_select_async(t, dq.data_ptr(), nq, off2.data_ptr(), ids2.data_ptr(), total + 8,
                                 dt2.data_ptr(), s2.cuda_stream)
    s.synchronize()
    s2.synchronize()
    assert int(dt.item()) == total and int(dt2.item()) == total
    _csr_equal(off.cpu().numpy(), ids[:total].cpu().numpy(), wo, wi, "async stream 1")
    _csr_equal(off2.cpu().numpy(), ids2[:total].cpu().numpy(), wo, wi, "async stream 2")
    assert bool((ids2[total:] == -7).all().item()), "wrote past the result"


def test_select_async_empty_and_small(rt, ora):
    import torch
    r = rtgen.uniform_rects(5000, 1e-2, 511)
    t = rt.build_str(r, 8, "soa")
    off = torch.empty(1, dtype=torch.int64, device="cuda")
    dt = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    dq = torch.zeros((1, 4), dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    assert rt.range_select_async(t, dq.data_ptr(), 0, off.data_ptr(), 0, 0, dt.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    assert int(dt.item()) == 0 and int(off.item()) == 0
    # a window meeting nothing: a zero-capacity buffer is enough
    q = np.array([[5.0, 5.0, 6.0, 6.0]], np.float32)
    dq = torch.from_numpy(q).cuda()
    off = torch.empty(2, dtype=torch.int64, device="cuda")
    assert rt.range_select_async(t, dq.data_ptr(), 1, off.data_ptr(), 0, 0, dt.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    assert int(dt.item()) == 0 and off.cpu().tolist() == [0, 0]
    # growing workspaces: a small call, a large one, a small one again
    for nq in (10, 30000, 10):
        q = rtgen.windows_loguniform(nq, 1e-6, 1e-2, 512 + nq)
        wo, wi = ora.select(ora.build_str(r, 8), q)
        dq = torch.from_numpy(q).cuda()
        off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
        ids = torch.empty(max(int(wo[-1]), 1), dtype=torch.int32, device="cuda")
        assert rt.range_select_async(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), int(wo[-1]),
                                     dt.data_ptr(), s.cuda_stream)
        torch.cuda.synchronize()
        _csr_equal(off.cpu().numpy(), ids[:int(wo[-1])].cpu().numpy(), wo, wi, f"async nq={nq}")


@pytest.mark.parametrize("kmin", [0, 4])
def test_two_stage_select(rt, ora, kmin):
    """Count stage, host read of the total, fill stage into a buffer of
    exactly that size (the server's admission by output memory)."""
    import torch
    say(f"case two_stage kmin={kmin}")
    r = rtgen.clustered_rects(200_000, 8, 0.03, 1e-3, 521)
    q = rtgen.windows_loguniform(12_000, 1e-6, 1e-2, 522)
    t = rt.build_str(r, 32, "soa")
    t.set_split(kmin)
    nq = q.shape[0]
    wo, wi = ora.select(ora.build_str(r, 32), q)
    dq = torch.from_numpy(q).cuda()
    off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    wb0 = rt.select_workspace_bytes(nq, 0)
    total = int(wo[-1])
    wb = rt.select_workspace_bytes(nq, total)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    st = torch.zeros(2, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    rt.range_select_device_count(t, dq.data_ptr(), nq, off.data_ptr(), work.data_ptr(), wb0, s)
    got_total = int(off[nq].item())
    assert got_total == total
    ids = torch.empty(total, dtype=torch.int32, device="cuda")
    rt.range_select_device_fill(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), total, work.data_ptr(), wb,
                                st.data_ptr(), s)
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [total, 0]
    assert rt.select_replay_info(work.data_ptr()) == (0, False)   # no room to record: the fill walked
    _csr_equal(off.cpu().numpy(), ids.cpu().numpy(), wo, wi, f"two-stage kmin={kmin}")
    # the count stage given room past its layout records, the fill replays
    wr = rt.select_replay_workspace_bytes(nq, total)
    workr = torch.empty(wr, dtype=torch.uint8, device="cuda")
    for rep in range(2):
        ids.fill_(-1)
        rt.range_select_device_count(t, dq.data_ptr(), nq, off.data_ptr(), workr.data_ptr(), wr, s)
        rt.range_select_device_fill(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), total, workr.data_ptr(),
                                    wr, st.data_ptr(), s)
        torch.cuda.synchronize()
        assert st.cpu().tolist() == [total, 0]
        chunks, over = rt.select_replay_info(workr.data_ptr())
        assert chunks > 0 and not over, f"two-stage kmin={kmin}: the fill did not replay"
        _csr_equal(off.cpu().numpy(), ids.cpu().numpy(), wo, wi, f"two-stage replay kmin={kmin} rep {rep}")


def test_two_stage_replay_overflow(rt, ora):
    """Two-stage select whose count stage has room for only a few record
    chunks (tiny windows: about one record per id): the records overflow,
    the fill stage walks the tree, the results equal the oracle's."""
    import torch
    r = rtgen.c2_rects(200_000)
    q = rtgen.windows_loguniform(20_000, 1e-8, 1e-6, 541)
    t = rt.build_str(r, 16, "soa")
    nq = q.shape[0]
    wo, wi = ora.select(ora.build_str(r, 16), q)
    total = int(wo[-1])
    say(f"case two-stage replay overflow: {total} ids")
    dq = torch.from_numpy(q).cuda()
    off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    ids = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
    st = torch.zeros(2, dtype=torch.int64, device="cuda")
    # room for eight 256-record chunks past the count stage's layout; every
    # lane group that finds anything takes a chunk of its own
    wb = rt.select_workspace_bytes(nq, total) + 8 * (256 * 16 + 4) + 512
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    rt.range_select_device_count(t, dq.data_ptr(), nq, off.data_ptr(), work.data_ptr(), wb, s)
    rt.range_select_device_fill(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), total, work.data_ptr(), wb,
                                st.data_ptr(), s)
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [total, 0]
    chunks, over = rt.select_replay_info(work.data_ptr())
    assert chunks > 0 and over, f"{chunks} chunks, overflow {over}: the case was meant to overflow"
    _csr_equal(off.cpu().numpy(), ids[:total].cpu().numpy(), wo, wi, "two-stage replay overflow")


def test_library_chosen_fanout_and_layout(rt, ora, tmp_path):
    """fanout 0 / RT_LAYOUT_AUTO: the library times its candidates, keeps the
    fastest, caches the choice in the file named by RT_TUNE_CACHE, and the
    tree answers like any other (oracle parity)."""
    import os
    import torch
    cache = tmp_path / "tune.txt"
    os.environ["RT_TUNE_CACHE"] = str(cache)
    try:
        r = rtgen.clustered_rects(60_000, 8, 0.03, 2e-3, 531)
        q = rtgen.windows_loguniform(4000, 1e-6, 1e-2, 532)
        want = ora.brute_select(r, q)
        t = rt.build_str(r, 0, "auto")
        i = t.info()
        assert i.fanout in (16, 32, 64) and i.layout in (rt.LAYOUT_AOS, rt.LAYOUT_SOA, rt.LAYOUT_D2)
        go, gi = rt.range_select(t, q)
        _csr_equal(go, gi, want[0], want[1], "tuned F and layout")
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and lines[0].startswith("rt-tune-v2 ")
        assert lines[0].split()[2:4] == [str(i.fanout), str(i.layout)]
        # same key: the cached choice, no new timing line
        t2 = rt.build_str(r, 0, "auto")
        assert (t2.info().fanout, t2.info().layout) == (i.fanout, i.layout)
        assert len(cache.read_text().splitlines()) == 1
        # one of the two left to the library
        t3 = rt.build_str(r, 32, "auto")
        assert t3.info().fanout == 32 and t3.info().layout in (0, 1, 3)
        t4 = rt.build_str(r, 0, "soa")
        assert t4.info().layout == rt.LAYOUT_SOA and t4.info().fanout in (16, 32, 64)
        for tt, what in ((t3, "F32 auto"), (t4, "auto soa")):
            go, gi = rt.range_select(tt, q)
            _csr_equal(go, gi, want[0], want[1], what)
        assert len(cache.read_text().splitlines()) == 3
        # the device-input builder, with the low-x option (another key)
        d = torch.from_numpy(r).cuda()
        t5 = rt.build_str_device(d.data_ptr(), r.shape[0], 0, "auto", torch.cuda.current_stream().cuda_stream,
                                 sort_lx=True)
        assert t5.info().flags == rt.BUILD_SORT_LX
        go, gi = rt.range_select(t5, q)
        _csr_equal(go, gi, want[0], want[1], "device tuned, sorted")
        # an empty relation needs no timing
        e = rt.build_str(np.zeros((0, 4), np.float32), 0, "auto")
        assert e.info().n_objects == 0
    finally:
        del os.environ["RT_TUNE_CACHE"]
