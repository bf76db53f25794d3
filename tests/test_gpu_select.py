"""GPU parity of range select: the HIP path (through the C ABI) against the
CPU oracle, element by element, on seeded inputs."""

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


def assert_csr_equal(got, want, what=""):
    go, gi = got
    wo, wi = want
    assert go.shape == wo.shape, what
    if not np.array_equal(go, wo):
        k = int(np.nonzero(go != wo)[0][0])
        raise AssertionError(f"{what}: offsets differ first at {k}: {go[k]} vs {wo[k]}")
    if not np.array_equal(gi, wi):
        k = int(np.nonzero(gi != wi)[0][0])
        raise AssertionError(f"{what}: ids differ first at {k}: {gi[k]} vs {wi[k]}")


def test_select_plain_100k(rt, ora):
    """100k uniform rectangles, fanout 16 SoA, 1000 windows of side 0.01."""
    w = rtgen.c1_plain()
    say("case select_uniform_100k_q1k_f16_soa")
    t = rt.build_str(w.rects, w.fanout, w.layout)
    got = rt.range_select(t, w.queries)
    want = ora.select(ora.build_str(w.rects, 16), w.queries)
    assert_csr_equal(got, want, "c1")
    assert 10.0 < want[0][-1] / 1000 < 12.0


FANOUTS = [2, 3, 4, 7, 8, 15, 16, 17, 31, 32, 33, 63, 64]
LAYOUTS = ["aos", "soa", "d2"]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("fanout", FANOUTS)
def test_select_adversarial(rt, ora, fanout, layout):
    """Touching edges, points, segments, duplicates, infinite windows; sizes
    0, 1, F, F+1 and a few larger ones; every fanout width class."""
    for s, n in enumerate([0, 1, fanout, fanout + 1, 97, 1500, 6000]):
        say(f"case adversarial F={fanout} {layout} n={n}")
        r = rtgen.adversarial_rects(n, 1000 * fanout + s) if n else np.zeros((0, 4), np.float32)
        q = rtgen.adversarial_windows(64, 77 * fanout + s)
        t = rt.build_str(r, fanout, layout)
        got = rt.range_select(t, q)
        want = ora.brute_select(r, q)
        assert_csr_equal(got, want, f"F={fanout} {layout} n={n}")
        t.set_lookahead(True)
        assert_csr_equal(rt.range_select(t, q), want, f"lookahead F={fanout} {layout} n={n}")


def test_select_long_segments(rt, ora):
    """Windows whose results span several LDS sort tiles plus a ragged tail
    (the merge path of the segmented sort), on clustered data."""
    r = rtgen.clustered_rects(300_000, 6, 0.03, 1e-3, 31)
    q = np.concatenate([rtgen.windows_loguniform(200, 1e-3, 5e-2, 32),
                        np.array([[-np.inf, -np.inf, np.inf, np.inf]], np.float32)])
    for fanout, layout in [(16, "soa"), (32, "aos"), (64, "soa"), (32, "d2")]:
        say(f"case long segments F={fanout} {layout}")
        t = rt.build_str(r, fanout, layout)
        got = rt.range_select(t, q)
        want = ora.select(ora.build_str(r, 16), q)
        assert_csr_equal(got, want, f"long F={fanout} {layout}")
        assert int(np.diff(want[0].astype(np.int64)).max()) == r.shape[0]


SORT_CLASS_EDGES = [0, 1, 2, 3, 255, 256, 257, 1023, 1024, 1025, 4095, 4096, 4097, 16383, 16384, 16385,
                    32767, 32768, 32769, 65537, 150_000]


@pytest.mark.parametrize("permuted", [True, False])
def test_sort_class_edges(rt, ora, permuted):
    """Results of exactly the lengths that bound the segmented sort's size
    classes (one wave, the block shapes, the two-level pass): points on a
    line, windows covering runs of them.  Unpermuted, the ids of a window are
    one contiguous range, so the top-bit buckets are as uneven as they get
    and the bitonic and tile-and-merge fallbacks run."""
    n = 400_000
    x = np.arange(n, dtype=np.float32)
    r = np.stack([x, np.zeros(n, np.float32), x, np.zeros(n, np.float32)], axis=1)
    if permuted:
        r = rtgen.permute(r, 77)
    g = np.random.default_rng(78)
    q = []
    for c in SORT_CLASS_EDGES:
        a = int(g.integers(0, n - c))
        q.append([a - 0.5, -1.0, a + c - 0.5, 1.0])
    q = np.array(q, np.float32)
    want = ora.select(ora.build_str(r, 16), q)
    assert np.array_equal(np.diff(want[0].astype(np.int64)), SORT_CLASS_EDGES)
    for fanout, layout in [(16, "soa"), (64, "aos")]:
        say(f"case sort class edges permuted={permuted} F={fanout} {layout}")
        t = rt.build_str(r, fanout, layout)
        assert_csr_equal(rt.range_select(t, q), want, f"class edges F={fanout} {layout}")


def test_lookahead_parity(rt, ora):
    """Lookahead loads (on after every leaf) with Morton-ordered batches, the
    split mapping and every layout: results equal the oracle's."""
    r = rtgen.c2_rects(200_000)
    q = rtgen.c2_queries(20_000)
    want = ora.select(ora.build_str(r, 32), q)
    for fanout, layout, kmin in [(16, "soa", 0), (32, "aos", 2), (64, "d2", 0), (64, "soa", 16), (7, "aos", 0)]:
        say(f"case lookahead F={fanout} {layout} kmin={kmin}")
        t = rt.build_str(r, fanout, layout)
        t.set_split(kmin)
        t.set_lookahead(True)
        assert_csr_equal(rt.range_select(t, q), want, f"lookahead F={fanout} {layout} kmin={kmin}")
    with pytest.raises(rt.RTError):
        rt._check(rt._L.rt_tree_set_lookahead(t.h, 2))


def test_bulk_copy_parity(rt, ora):
    """Long contained runs (>= 2048 ids) deferred to the streaming copy after
    the fill pass, forced on a small tree, and kept in the pass: results
    equal the oracle's with windows of up to 0.3 of the space (contained runs
    of up to ~10^5 ids), for every layout, the split mapping and lookahead,
    through the host and the device entry points."""
    import torch
    r = rtgen.c2_rects(400_000)
    q = rtgen.windows_loguniform(1500, 1e-5, 0.3, 91)
    want = ora.select(ora.build_str(r, 32), q)
    say(f"case bulk copy: {want[1].size} ids")
    for fanout, layout, kmin, la, mode in [(16, "soa", 0, False, "on"), (32, "aos", 0, True, "on"),
                                           (64, "d2", 16, False, "on"), (64, "soa", 0, False, "on"),
                                           (64, "soa", 0, False, "off"), (32, "soa", 2, True, "auto")]:
        say(f"case bulk copy F={fanout} {layout} kmin={kmin} lookahead={la} mode={mode}")
        t = rt.build_str(r, fanout, layout)
        t.set_split(kmin)
        t.set_lookahead(la)
        t.set_bulk_copy(mode)
        assert_csr_equal(rt.range_select(t, q), want, f"bulk copy F={fanout} {layout} kmin={kmin} {mode}")
        # device entry point, resident queries, twice on one workspace
        nq, cap = q.shape[0], int(want[1].size)
        dq = torch.from_numpy(q).cuda()
        off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
        ids = torch.empty(cap, dtype=torch.int32, device="cuda")
        wb = rt.select_workspace_bytes(nq, cap)
        w = torch.empty(wb, dtype=torch.uint8, device="cuda")
        st = torch.zeros(2, dtype=torch.int64, device="cuda")
        s = torch.cuda.current_stream().cuda_stream
        for _ in range(2):
            ids.fill_(-1)
            rt.range_select_device(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), cap, w.data_ptr(), wb,
                                   st.data_ptr(), s)
            torch.cuda.synchronize()
            assert st.cpu().tolist() == [cap, 0]
            assert np.array_equal(off.cpu().numpy(), want[0].astype(np.int64))
            assert np.array_equal(ids.cpu().numpy().view(np.uint32), want[1])
        t.free()
    t = rt.build_str(r[:1000], 16, "soa")
    with pytest.raises(rt.RTError):
        rt._check(rt._L.rt_tree_set_bulk_copy(t.h, 3))


def _device_select(rt, t, q, cap, wb):
    """One-call device select on a fresh workspace of wb bytes; returns
    (offsets, ids, replay info), run twice on the same buffers."""
    import torch
    nq = q.shape[0]
    dq = torch.from_numpy(q).cuda()
    off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    ids = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    w = torch.empty(wb, dtype=torch.uint8, device="cuda")
    st = torch.zeros(2, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    out = []
    for _ in range(2):
        ids.fill_(-1)
        rt.range_select_device(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), cap, w.data_ptr(), wb,
                               st.data_ptr(), s)
        torch.cuda.synchronize()
        assert st.cpu().tolist() == [cap, 0]
        out.append((off.cpu().numpy().copy(), ids[:cap].cpu().numpy().view(np.uint32).copy(),
                    rt.select_replay_info(w.data_ptr())))
    return out


def test_replay_parity(rt, ora):
    """The fill replaying the count pass's records (leaf hit masks, contained
    leaf ranges) instead of walking the tree: results equal the oracle's for
    every layout, fanouts 7 to 64 (64: two records per leaf), the split
    mapping, lookahead and long deferred runs; an arena too small for the
    records falls back to the walk; replay switched off records nothing."""
    r = rtgen.c2_rects(300_000)
    q = np.concatenate([rtgen.c2_queries(20_000), rtgen.windows_loguniform(500, 1e-5, 0.1, 93)])
    want = ora.select(ora.build_str(r, 32), q)
    cap = int(want[1].size)
    wo = want[0].astype(np.int64)
    say(f"case replay: {q.shape[0]} windows, {cap} ids")
    nq = q.shape[0]
    full = rt.select_replay_workspace_bytes(nq, cap)
    base = rt.select_workspace_bytes(nq, cap)
    assert full > base
    for fanout, layout, kmin, la, bulk in [(16, "soa", 0, False, "auto"), (32, "aos", 0, True, "auto"),
                                           (64, "d2", 16, False, "auto"), (64, "soa", 0, False, "on"),
                                           (7, "aos", 0, False, "auto"), (64, "aos", 2, True, "auto"),
                                           (33, "soa", 0, False, "on")]:
        say(f"case replay F={fanout} {layout} kmin={kmin} lookahead={la} bulk={bulk}")
        t = rt.build_str(r, fanout, layout)
        t.set_split(kmin)
        t.set_lookahead(la)
        t.set_bulk_copy(bulk)
        for go, gi, (chunks, over) in _device_select(rt, t, q, cap, full):
            assert chunks > 0 and not over, f"F={fanout} {layout}: replay did not run ({chunks}, {over})"
            assert np.array_equal(go, wo) and np.array_equal(gi, want[1]), f"replay F={fanout} {layout} kmin={kmin}"
        # an arena of a few chunks overflows: the fill walks the tree
        for go, gi, (chunks, over) in _device_select(rt, t, q, cap, base + 64 * 4096):
            assert over, f"F={fanout} {layout}: a 64-chunk arena did not overflow"
            assert np.array_equal(go, wo) and np.array_equal(gi, want[1]), f"fallback F={fanout} {layout}"
        t.set_replay(False)
        for go, gi, (chunks, over) in _device_select(rt, t, q, cap, full):
            assert chunks == 0 and not over
            assert np.array_equal(go, wo) and np.array_equal(gi, want[1]), f"replay off F={fanout} {layout}"
        t.free()
    t = rt.build_str(r[:1000], 16, "soa")
    with pytest.raises(rt.RTError):
        rt._check(rt._L.rt_tree_set_replay(t.h, 2))
    # windows over the whole space: every root child is one range record of
    # tens of thousands of ids, every segment holds all 300k ids
    qa = np.array([[-1.0, -1.0, 2.0, 2.0]] * 8 + [[0.0, 0.0, 0.5, 1.0]] * 4, np.float32)
    wa = ora.select(ora.build_str(r, 32), qa)
    capa = int(wa[1].size)
    for fanout, layout in [(64, "soa"), (16, "d2")]:
        say(f"case replay whole-space windows F={fanout} {layout}: {capa} ids")
        t = rt.build_str(r, fanout, layout)
        for go, gi, (chunks, over) in _device_select(rt, t, qa, capa,
                                                     rt.select_replay_workspace_bytes(qa.shape[0], capa)):
            assert chunks > 0 and not over
            assert np.array_equal(go, wa[0].astype(np.int64)) and np.array_equal(gi, wa[1]), f"F={fanout} {layout}"
        t.free()


def test_select_all_windows(rt):
    """64 windows covering all 2M rectangles: 2M-id segments, whose
    sub-buckets hold 8192 ids each, sorted by the wide (1024 x 32) group
    sorts; every window gets every id, ascending."""
    n = 2_000_000
    r = rtgen.uniform_rects(n, 1e-4, 55)
    t = rt.build_str(r, 16, "soa")
    q = np.tile(np.array([[-np.inf, -np.inf, np.inf, np.inf]], np.float32), (64, 1))
    off, ids = rt.range_select(t, q)
    assert np.array_equal(off, np.arange(65, dtype=np.uint64) * n)
    want = np.arange(n, dtype=np.uint32)
    for k in range(64):
        assert np.array_equal(ids[k * n:(k + 1) * n], want), k


def test_select_empty_query_batch(rt):
    t = rt.build_str(rtgen.uniform_rects(100, 0.01, 1), 16, "soa")
    off, ids = rt.range_select(t, np.zeros((0, 4), np.float32))
    assert off.tolist() == [0] and ids.size == 0


def test_select_rejects_bad_queries(rt):
    t = rt.build_str(rtgen.uniform_rects(100, 0.01, 1), 16, "soa")
    with pytest.raises(rt.RTError):
        rt.range_select(t, np.array([[0.5, 0.5, 0.4, 0.6]], np.float32))
    with pytest.raises(rt.RTError):
        rt.range_select(t, np.array([[np.nan, 0.5, 0.4, 0.6]], np.float32))


def test_subnormal_coordinates(rt, ora):
    """Subnormal fp32 coordinates must compare exactly as on the CPU (the
    library is built without denormal flushing)."""
    tiny = np.float32(2.0 ** -140)
    r = np.array([[0, 0, tiny, tiny], [tiny, tiny, 2 * tiny, 2 * tiny], [-tiny, -tiny, 0, 0],
                  [3 * tiny, 0, 4 * tiny, tiny], [0, 0, 0, 0]], np.float32)
    q = np.array([[tiny, tiny, tiny, tiny], [np.float32(1.5) * tiny, 0, 2 * tiny, 0],
                  [-tiny, -tiny, -tiny, -tiny], [0, 0, 0, 0], [2.5 * tiny, 0, 2.75 * tiny, tiny]], np.float32)
    for F in (2, 4, 16):
        t = rt.build_str(r, F, "soa")
        assert_csr_equal(rt.range_select(t, q), ora.brute_select(r, q), f"subnormal F={F}")


def test_tree_invariants(rt, ora):
    """The library's tree read back from the device satisfies every invariant
    of the oracle's checker (MBR unions, one leaf entry per object with its own
    rectangle, levels, counts)."""
    for n, F, layout in [(0, 8, "soa"), (1, 16, "aos"), (64, 64, "soa"), (65, 64, "d2"),
                         (10_000, 16, "soa"), (50_000, 32, "aos"), (123_457, 7, "d2")]:
        r = rtgen.clustered_rects(n, 5, 0.05, 1e-3, n + F) if n else np.zeros((0, 4), np.float32)
        t = rt.build_str(r, F, layout)
        ex = t.export()
        ot = ora.tree_from_arrays(**ex)
        rc, msg = ora.check(ot, r)
        assert rc == 0, (n, F, layout, msg)
        # the kernels rely on contiguous children: entry e of an internal node
        # points at the node's first child + e
        for u in np.nonzero(ex["level"] > 0)[0]:
            f0, c = int(ex["first"][u]), int(ex["count"][u])
            p = ex["ptr"][f0:f0 + c].astype(np.int64)
            assert np.array_equal(p, p[0] + np.arange(c)), (n, F, layout, u)
        info = t.info()
        assert info.node_bytes == 20 * F


def test_deterministic(rt):
    r = rtgen.c2_rects(200_000)
    q = rtgen.c2_queries(5000)
    t = rt.build_str(r, 32, "soa")
    a = rt.range_select(t, q)
    b = rt.range_select(t, q)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_device_api_and_capacity(rt, ora):
    """Stream-ordered device-pointer select with torch buffers; an output
    capacity that is too small is reported in the status words and leaves the
    id buffer untouched."""
    import torch
    r = rtgen.c2_rects(200_000)
    q = rtgen.c2_queries(3000)
    t = rt.build_str(r, 16, "aos")
    want = ora.select(ora.build_str(r, 16), q)
    total = int(want[0][-1])
    dq = torch.from_numpy(q).cuda()
    off = torch.empty(q.shape[0] + 1, dtype=torch.int64, device="cuda")
    for cap, ok in [(total, True), (total + 1000, True), (total - 1, False)]:
        ids = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
        wb = rt.select_workspace_bytes(q.shape[0], cap)
        work = torch.empty(wb, dtype=torch.uint8, device="cuda")
        st = torch.zeros(2, dtype=torch.int64, device="cuda")
        s = torch.cuda.current_stream()
        rt.range_select_device(t, dq.data_ptr(), q.shape[0], off.data_ptr(), ids.data_ptr(), cap,
                               work.data_ptr(), wb, st.data_ptr(), s.cuda_stream)
        s.synchronize()
        stat = st.cpu().numpy()
        assert stat[0] == total
        if ok:
            assert stat[1] == 0
            got = (off.cpu().numpy().astype(np.uint64), ids.cpu().numpy().view(np.uint32)[:total])
            assert_csr_equal(got, want, f"device cap={cap}")
        else:
            assert stat[1] & 1
            assert bool((ids == -1).all())
    # count-only entry point
    counts = torch.empty(q.shape[0], dtype=torch.int32, device="cuda")
    wb = rt.select_workspace_bytes(q.shape[0], 0)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    rt.range_count_device(t, dq.data_ptr(), q.shape[0], counts.data_ptr(), work.data_ptr(), wb,
                          torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy().astype(np.int64), np.diff(want[0].astype(np.int64)))


def test_visit_stats(rt):
    """Visited-node statistics: every query visits at least the root; a
    select-all window contains every child of the root, so it visits only
    the root and takes all ids wholesale; a window away from the data visits
    only the root."""
    r = rtgen.uniform_rects(20_000, 1e-3, 5)
    t = rt.build_str(r, 16, "soa")
    root_entries = int(t.export()["count"][0])
    vn, ve, vc = rt.visit_stats(t, np.array([[-np.inf, -np.inf, np.inf, np.inf]], np.float32))
    assert (vn, ve, vc) == (1, root_entries, 20_000)
    vn, ve, vc = rt.visit_stats(t, np.array([[5, 5, 6, 6]], np.float32))
    assert (vn, vc) == (1, 0)


@pytest.mark.parametrize("fanout,layout", [(16, "soa"), (32, "aos"), (64, "d2"), (32, "soa")])
def test_select_ordered_batch(rt, ora, fanout, layout):
    """Batches of at least 8192 windows are processed in Morton order with
    per-XCD slices; the CSR must be identical to the oracle's."""
    r = rtgen.c2_rects(300_000, seed_base=2100)
    q = rtgen.c2_queries(20_011, seed_base=2100)
    say(f"case ordered batch F={fanout} {layout}")
    t = rt.build_str(r, fanout, layout)
    got = rt.range_select(t, q)
    want = ora.select(ora.build_str(r, fanout), q)
    assert_csr_equal(got, want, f"ordered F={fanout} {layout}")


@pytest.mark.parametrize("kmin", [0, 1, 2, 16])
@pytest.mark.parametrize("fanout,layout", [(16, "aos"), (32, "soa"), (8, "d2")])
def test_select_split_mapping(rt, ora, kmin, fanout, layout):
    """Queries split into (query, subtree) work items -- kmin = 1 splits every
    query that reaches a parents-of-leaves node -- give the same CSR as one
    lane group per query (kmin = 0) and as the oracle, for small and large
    batches (with and without the Morton order)."""
    r = rtgen.clustered_rects(250_000, 16, 0.02, 2e-3, 77)
    for nq, lo, hi in [(300, 1e-4, 0.3), (9000, 1e-6, 1e-2)]:
        q = rtgen.windows_loguniform(nq, lo, hi, 78 + nq)
        q = np.concatenate([q, np.array([[-np.inf, -np.inf, np.inf, np.inf]], np.float32)])
        say(f"case split kmin={kmin} F={fanout} {layout} nq={nq}")
        t = rt.build_str(r, fanout, layout)
        t.set_split(kmin)
        got = rt.range_select(t, q)
        want = ora.select(ora.build_str(r, fanout), q)
        assert_csr_equal(got, want, f"split kmin={kmin} F={fanout} {layout} nq={nq}")


def test_sort_dense_id_runs(rt):
    """9M points on a 4096-wide grid, numbered row by row, and windows over
    whole rows: each result is one run of consecutive ids (known in closed
    form).  The top-8-bit sub-buckets of such class-L segments hold up to
    65536 ids: runs that split into two halves of 24576 take the wide
    (1024 x 32) group sorts, longer ones the tile-and-merge fallback."""
    W, rows = 4096, 2198
    n = W * rows
    i = np.arange(n, dtype=np.int64)
    x = (i % W).astype(np.float32)
    y = (i // W).astype(np.float32)
    r = np.stack([x, y, x, y], axis=1)
    # (first row, rows): ids [first * W, (first + rows) * W)
    runs = [(250, 12), (0, 10), (250, 17), (700, 74), (1200, 489)]
    q = np.array([[-0.5, f - 0.5, W - 0.5, f + k - 0.5] for f, k in runs], np.float32)
    say("case dense id runs")
    t = rt.build_str(r, 32, "soa")
    off, ids = rt.range_select(t, q)
    assert np.array_equal(np.diff(off.astype(np.int64)), [k * W for _, k in runs])
    for j, (f, k) in enumerate(runs):
        assert np.array_equal(ids[off[j]:off[j + 1]], np.arange(f * W, (f + k) * W, dtype=np.uint32)), (f, k)
