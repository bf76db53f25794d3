"""GPU join over nodes sorted by low x with the pruning of section 4: outer
slicing (O3), one-to-many (O4) and many-to-many (O5) inner shrinking.  Every
variant returns exactly the oracle's pair set, and evaluates exactly as many
child-pair predicates as the oracle's pruned join does on the same trees
(which pins the GPU's slicing and flip indices, not only its results).  The
lower bound on the inner scan (LB, not in the paper) is held to the oracle's
pair set and to evaluating no more predicates than O3 + O5."""

import sys

import numpy as np
import pytest

import oracle
import rtgen
from str_shape import assert_export_equal, expected_export

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


def _flag_sets(rt):
    return [0, rt.JOIN_O3, rt.JOIN_O4, rt.JOIN_O5, rt.JOIN_O3 | rt.JOIN_O4, rt.JOIN_O3 | rt.JOIN_O5]


@pytest.mark.parametrize("n,F,layout", [(0, 8, "soa"), (1, 4, "aos"), (64, 64, "d2"), (5000, 7, "soa"),
                                        (60_000, 32, "aos"), (123_457, 16, "d2")])
def test_sorted_build_shape(rt, ora, n, F, layout):
    r = rtgen.adversarial_rects(n, 40 + n) if n else np.zeros((0, 4), np.float32)
    t = rt.build_str(r, F, layout, sort_lx=True)
    assert t.info().flags == rt.BUILD_SORT_LX
    ex = t.export()
    assert_export_equal(ex, expected_export(r, F, sort_lx=True), f"n={n} F={F} {layout}")
    for u in range(ex["level"].shape[0]):
        f0, c = int(ex["first"][u]), int(ex["count"][u])
        assert np.all(np.diff(ex["lx"][f0:f0 + c]) >= 0)
    assert ora.check(ora.tree_from_arrays(**ex), r)[0] == 0


JOIN_CASES = [
    # (name, A, Fa, layout a, B, Fb, layout b)
    ("adv-small", lambda: rtgen.adversarial_rects(700, 1), 4, "soa", lambda: rtgen.adversarial_rects(900, 2), 4, "aos"),
    ("uniform-clustered", lambda: rtgen.uniform_rects(40_000, 0.004, 3), 32, "soa",
     lambda: rtgen.clustered_rects(40_000, 8, 0.05, 0.004, 4), 32, "soa"),
    ("f64-f16", lambda: rtgen.uniform_rects(30_000, 0.005, 5), 64, "d2",
     lambda: rtgen.uniform_rects(2_000, 0.01, 6), 16, "aos"),
    ("unequal-height", lambda: rtgen.uniform_rects(50_000, 0.003, 7), 8, "soa",
     lambda: rtgen.uniform_rects(300, 0.02, 8), 32, "soa"),
    ("ragged", lambda: rtgen.clustered_rects(12_345, 5, 0.1, 0.01, 9), 7, "aos",
     lambda: rtgen.adversarial_rects(30_000, 10), 13, "d2"),
]


@pytest.mark.parametrize("case", JOIN_CASES, ids=lambda c: c[0])
def test_pruned_join_parity(rt, ora, case):
    name, fa, Fa, la, fb, Fb, lb = case
    A, B = fa(), fb()
    say("join", name, A.shape[0], B.shape[0])
    want = ora.join(ora.build_str(A, Fa), ora.build_str(B, Fb))
    ta, tb = rt.build_str(A, Fa, la, sort_lx=True), rt.build_str(B, Fb, lb, sort_lx=True)
    equal_h = ta.info().height == tb.info().height
    assert equal_h == (name != "unequal-height"), (name, ta.info().height, tb.info().height)
    oa = ora.tree_from_arrays(**ta.export())
    ob = ora.tree_from_arrays(**tb.export())
    for flags in _flag_sets(rt):
        got, tests = rt.spatial_join(ta, tb, flags, with_tests=True)
        assert np.array_equal(got, want), f"{name} flags {flags}: {got.shape} vs {want.shape}"
        if equal_h:
            p, otests = ora.join_opt(oa, ob, flags)
            assert np.array_equal(p, want)
            assert tests == otests, f"{name} flags {flags}: GPU evaluated {tests}, oracle {otests}"
    lb = rt.JOIN_O3 | rt.JOIN_O5 | rt.JOIN_LB
    got, tests_lb = rt.spatial_join(ta, tb, lb, with_tests=True)
    assert np.array_equal(got, want), f"{name} flags {lb}"
    assert tests_lb <= rt.spatial_join(ta, tb, rt.JOIN_O3 | rt.JOIN_O5, with_tests=True)[1]
    got = rt.spatial_join(ta, tb, rt.JOIN_TILE)
    assert np.array_equal(got, want)
    assert np.array_equal(rt.spatial_join(ta, tb), want)   # default: O3|O5|LB on sorted trees


def test_pruned_join_c3_sample(rt, ora):
    """C3-shaped relations (2M x 2M at full size; a 200k x 200k cut here):
    pruning removes most predicate evaluations and no pair."""
    A = rtgen.uniform_rects(200_000, 5e-4, 3001)
    B = rtgen.clustered_rects(200_000, 64, 0.01, 5e-4, 3002)
    ta, tb = rt.build_str(A, 32, "soa", sort_lx=True), rt.build_str(B, 32, "soa", sort_lx=True)
    want = ora.join(ora.build_str(A, 32), ora.build_str(B, 32))
    oa, ob = ora.tree_from_arrays(**ta.export()), ora.tree_from_arrays(**tb.export())
    assert ta.info().height == tb.info().height
    res = {}
    for flags in _flag_sets(rt):
        got, tests = rt.spatial_join(ta, tb, flags, with_tests=True)
        assert np.array_equal(got, want), flags
        assert tests == ora.join_opt(oa, ob, flags)[1], flags
        res[flags] = tests
    lb = rt.JOIN_O3 | rt.JOIN_O5 | rt.JOIN_LB
    got, res[lb] = rt.spatial_join(ta, tb, lb, with_tests=True)
    assert np.array_equal(got, want)
    say("tests per variant", res)
    assert res[lb] < res[rt.JOIN_O3 | rt.JOIN_O5] == res[rt.JOIN_O3 | rt.JOIN_O4] < res[rt.JOIN_O3] <= res[0]


def _edge_rects(n, seed):
    """Rectangles that stress the lower bound's margin: infinite and
    half-infinite extents, huge and tiny magnitudes, points, duplicates, and
    rectangles that touch exactly at the bound."""
    g = np.random.default_rng(seed)
    r = rtgen.adversarial_rects(n, seed, grid=64).astype(np.float32)
    k = g.integers(0, 64, size=n)
    inf = np.float32(np.inf)
    r[k == 0, 0] = -inf                                   # open to the left
    r[k == 1, 2] = inf                                    # open to the right
    r[g.integers(0, n, size=2)] = (-inf, -inf, inf, inf)  # whole plane
    big = g.uniform(-3e37, 3e37, size=(int((k == 3).sum()), 1)).astype(np.float32)
    r[k == 3] = np.hstack([big, big, big + np.abs(big) * np.float32(1e-6), big])
    tiny = g.integers(-40, 40, size=(int((k == 4).sum()), 2)).astype(np.float32) * np.float32(1e-40)
    r[k == 4] = np.hstack([tiny, tiny + np.float32(1e-40)])
    # a run of rectangles whose high x equals the next one's low x exactly
    e = np.flatnonzero(k == 5)
    x = np.float32(0.125) * np.arange(e.size, dtype=np.float32)
    r[e] = np.stack([x, np.zeros_like(x), x + np.float32(0.125), np.full_like(x, 0.01)], 1)
    return r


@pytest.mark.parametrize("n,F,seed", [(5_000, 8, 61), (40_000, 32, 62), (20_000, 64, 63)])
def test_join_lower_bound_edges(rt, ora, n, F, seed):
    """The lower bound never cuts a qualifying pair, with infinite extents
    (where the bound turns off), widths near the largest float, subnormal
    coordinates and pairs that touch exactly."""
    A, B = _edge_rects(n, seed), _edge_rects(n // 2 + 1, seed + 1000)
    say(f"case lower bound n={n} F={F} seed={seed}")
    want = ora.join(ora.build_str(A, F), ora.build_str(B, F))
    ta, tb = rt.build_str(A, F, "soa", sort_lx=True), rt.build_str(B, F, "aos", sort_lx=True)
    for flags in (rt.JOIN_O3 | rt.JOIN_O5 | rt.JOIN_LB, rt.JOIN_O3 | rt.JOIN_O5, None):
        got = rt.spatial_join(ta, tb, flags)
        assert np.array_equal(got, want), flags
        assert np.array_equal(rt.spatial_join(tb, ta, flags), want[np.lexsort((want[:, 0], want[:, 1]))][:, ::-1])


def test_pruning_needs_sorted_trees(rt):
    A = rtgen.uniform_rects(2000, 0.01, 11)
    ts, tu = rt.build_str(A, 16, "soa", sort_lx=True), rt.build_str(A, 16, "soa")
    assert tu.info().flags == 0
    for flags in (rt.JOIN_O3, rt.JOIN_O4, rt.JOIN_O5):
        with pytest.raises(rt.RTError):
            rt.spatial_join(ts, tu, flags)
    with pytest.raises(rt.RTError):
        rt.spatial_join(ts, ts, rt.JOIN_TILE | rt.JOIN_O3)
    with pytest.raises(rt.RTError):
        rt.spatial_join(ts, ts, 64)
    for flags in (rt.JOIN_LB, rt.JOIN_LB | rt.JOIN_O3, rt.JOIN_LB | rt.JOIN_O5,
                  rt.JOIN_LB | rt.JOIN_O3 | rt.JOIN_O4, rt.JOIN_LB | rt.JOIN_O3 | rt.JOIN_O4 | rt.JOIN_O5):
        with pytest.raises(rt.RTError):
            rt.spatial_join(ts, ts, flags)
    with pytest.raises(rt.RTError):
        rt.spatial_join(ts, tu, rt.JOIN_O3 | rt.JOIN_O5 | rt.JOIN_LB)
    # unsorted trees still join without pruning, in both kernels
    want = rt.spatial_join(ts, ts, rt.JOIN_O3 | rt.JOIN_O5)
    assert np.array_equal(rt.spatial_join(tu, tu, 0), want)
    assert np.array_equal(rt.spatial_join(tu, tu, rt.JOIN_TILE), want)
    assert np.array_equal(rt.spatial_join(tu, tu), want)


def test_join_device_output(rt, ora):
    """Device-output join: same pairs as the host API; too small a buffer is
    reported with the needed size and left untouched."""
    import torch
    A = rtgen.uniform_rects(30_000, 0.004, 21)
    B = rtgen.clustered_rects(30_000, 6, 0.05, 0.004, 22)
    want = ora.join(ora.build_str(A, 16), ora.build_str(B, 16))
    for sort_lx, flags in [(False, None), (True, None), (True, rt.JOIN_O3 | rt.JOIN_O4), (False, 0)]:
        ta, tb = rt.build_str(A, 16, "soa", sort_lx=sort_lx), rt.build_str(B, 32, "aos", sort_lx=sort_lx)
        small = torch.full((2 * 10,), 7, dtype=torch.int32, device="cuda")
        n = rt.spatial_join_device(ta, tb, small.data_ptr(), 10, flags)
        assert n == want.shape[0] and n > 10
        assert bool((small == 7).all())
        buf = torch.full((2 * n,), 7, dtype=torch.int32, device="cuda")
        s = torch.cuda.current_stream()
        assert rt.spatial_join_device(ta, tb, buf.data_ptr(), n, flags, s.cuda_stream) == n
        got = buf.cpu().numpy().view(np.uint32).reshape(-1, 2)
        assert np.array_equal(got, want), (sort_lx, flags)
    # empty relation
    te = rt.build_str(np.zeros((0, 4), np.float32), 16)
    assert rt.spatial_join_device(te, ta, 0, 0) == 0


def test_join_workspace_reuse(rt, ora):
    """Joins run in a sequence reuse one pooled workspace: a repeated join
    replays its levels with the sizes kept on the device, a smaller one
    replays inside the larger buffers, a larger one (or one with another
    level structure) outgrows them and runs level by level.  Every result
    equals the oracle's."""
    cases = [("big", 60_000, 32, 41), ("big again", 60_000, 32, 41), ("small", 3_000, 32, 42),
             ("larger", 120_000, 32, 43), ("other shape", 20_000, 8, 44), ("big last", 60_000, 32, 41)]
    for name, n, F, seed in cases:
        say(f"case workspace reuse {name} n={n} F={F}")
        A = rtgen.uniform_rects(n, 2e-3, seed)
        B = rtgen.clustered_rects(n, 16, 0.05, 2e-3, seed + 100)
        want = ora.join(ora.build_str(A, 16), ora.build_str(B, 16))
        ta = rt.build_str(A, F, "soa", sort_lx=True)
        tb = rt.build_str(B, F, "soa", sort_lx=True)
        assert np.array_equal(rt.spatial_join(ta, tb), want), name
        import torch
        m = rt.spatial_join_device(ta, tb, 0, 0)
        assert m == want.shape[0], name
        buf = torch.empty(2 * max(m, 1), dtype=torch.int32, device="cuda")
        assert rt.spatial_join_device(ta, tb, buf.data_ptr(), m) == m
        got = buf[:2 * m].cpu().numpy().view(np.uint32).reshape(-1, 2)
        assert np.array_equal(got, want), name


def test_join_key_sort_paths(rt, ora):
    """The pair keys are split into 2048 buckets by their top bits and every
    bucket is sorted in LDS; a bucket over the LDS cap (one object meeting
    20000 others) is sorted in runs merged through global memory, and a
    result over the bucketing limit (3.4M pairs) goes through the LSD radix
    sort instead.  Every path gives the oracle's pairs."""
    B = rtgen.uniform_rects(20_000, 0.01, 71)
    small = rtgen.uniform_rects(9_999, 0.01, 72)
    whole = np.array([[-1.0, -1.0, 2.0, 2.0]], np.float32)
    cases = [("lds buckets", small),
             ("bucket over the cap", np.concatenate([small[:5000], whole, small[5000:]])),
             ("over the bucketing limit", np.concatenate([np.repeat(whole, 170, 0), small[:100]]))]
    tb = rt.build_str(B, 32, "soa", sort_lx=True)
    ob = ora.build_str(B, 32)
    for name, A in cases:
        say(f"case key sort {name} nA={A.shape[0]}")
        want = ora.join(ora.build_str(A, 32), ob)
        ta = rt.build_str(A, 32, "soa", sort_lx=True)
        for flags in (None, rt.JOIN_TILE):
            got = rt.spatial_join(ta, tb, flags)
            assert np.array_equal(got, want), (name, flags, got.shape, want.shape)


def test_join_graph_replays(rt, ora):
    """A join repeated with the same trees is replayed from a captured graph
    (from its third run on); other joins in between, host- and device-output
    calls and a buffer that is too small all leave every result equal to the
    oracle's."""
    import torch
    A = rtgen.uniform_rects(80_000, 2e-3, 81)
    B = rtgen.clustered_rects(80_000, 16, 0.05, 2e-3, 82)
    C = rtgen.uniform_rects(5_000, 5e-3, 83)
    want = ora.join(ora.build_str(A, 32), ora.build_str(B, 32))
    want_c = ora.join(ora.build_str(C, 32), ora.build_str(B, 32))
    ta, tb = rt.build_str(A, 32, "soa", sort_lx=True), rt.build_str(B, 32, "soa", sort_lx=True)
    tc = rt.build_str(C, 32, "soa", sort_lx=True)
    n = want.shape[0]
    buf = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    for rep in range(6):
        say(f"case graph replay {rep}")
        buf.fill_(7)
        assert rt.spatial_join_device(ta, tb, buf.data_ptr(), n) == n
        got = buf.cpu().numpy().view(np.uint32).reshape(-1, 2)
        assert np.array_equal(got, want), rep
        assert np.array_equal(rt.spatial_join(ta, tb), want), rep
        if rep % 2:
            assert np.array_equal(rt.spatial_join(tc, tb), want_c), rep
        small = torch.full((2 * 10,), 7, dtype=torch.int32, device="cuda")
        assert rt.spatial_join_device(ta, tb, small.data_ptr(), 10) == n
        assert bool((small == 7).all())


def _walk_counts(ea, eb):
    """Node pairs, entry predicates and real entries of the synchronized
    traversal, walked on the host over two exported trees (the deeper tree
    descends alone against the other tree's bounding box until the levels
    meet)."""
    def entries(ex, u):
        f0, c = int(ex["first"][u]), int(ex["count"][u])
        return np.stack([ex["lx"][f0:f0 + c], ex["ly"][f0:f0 + c], ex["hx"][f0:f0 + c], ex["hy"][f0:f0 + c]], 1), \
            ex["ptr"][f0:f0 + c]

    def mbr(ex):
        e, _ = entries(ex, 0)
        return np.array([e[:, 0].min(), e[:, 1].min(), e[:, 2].max(), e[:, 3].max()], np.float32)

    la, lb = int(ea["height"]) - 1, int(eb["height"]) - 1
    fr = [(0, 0)]
    pairs = preds = ents = 0
    while fr:
        pairs += len(fr)
        nxt = []
        for u, v in fr:
            if la > lb or lb > la:
                deep, other, node = (ea, eb, u) if la > lb else (eb, ea, v)
                e, p = entries(deep, node)
                m = mbr(other)
                hit = (e[:, 0] <= m[2]) & (m[0] <= e[:, 2]) & (e[:, 1] <= m[3]) & (m[1] <= e[:, 3])
                preds += e.shape[0]
                ents += e.shape[0]
                nxt += [(int(c), v) if la > lb else (u, int(c)) for c in p[hit]]
            else:
                a, pa = entries(ea, u)
                b, pb = entries(eb, v)
                preds += a.shape[0] * b.shape[0]
                ents += a.shape[0] + b.shape[0]
                if la == 0:
                    continue
                hit = ((a[:, None, 0] <= b[None, :, 2]) & (b[None, :, 0] <= a[:, None, 2]) &
                       (a[:, None, 1] <= b[None, :, 3]) & (b[None, :, 1] <= a[:, None, 3]))
                ii, jj = np.nonzero(hit)
                nxt += list(zip(pa[ii].tolist(), pb[jj].tolist()))
        if la > lb:
            la -= 1
        elif lb > la:
            lb -= 1
        else:
            if la == 0:
                break
            la -= 1
            lb -= 1
        fr = nxt
    return pairs, preds, ents


@pytest.mark.parametrize("na,Fa,nb,Fb", [(3000, 8, 2500, 8), (4000, 16, 200, 4), (300, 32, 5000, 5)])
def test_join_visit_stats(rt, ora, na, Fa, nb, Fb):
    """The byte/operation model's counts of the plain traversal equal a host
    walk over the exported trees; at equal heights the tile expansion's
    predicate count equals the oracle's unpruned join count."""
    A = rtgen.uniform_rects(na, 0.02, 41)
    B = rtgen.clustered_rects(nb, 4, 0.05, 0.02, 42)
    ta, tb = rt.build_str(A, Fa, "soa", sort_lx=True), rt.build_str(B, Fb, "aos", sort_lx=True)
    got = rt.join_visit_stats(ta, tb)
    want = _walk_counts(ta.export(), tb.export())
    assert got == want, (got, want)
    if ta.info().height == tb.info().height:
        _, tile_tests = rt.spatial_join(ta, tb, rt.JOIN_TILE, with_tests=True)
        oa, ob = ora.tree_from_arrays(**ta.export()), ora.tree_from_arrays(**tb.export())
        assert tile_tests == ora.join_opt(oa, ob, 0)[1] == got[1]
