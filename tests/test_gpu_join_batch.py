"""GPU parity of the spatial join and of the batched (persistent, graph)
select, against the CPU oracle."""

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


def assert_pairs_equal(got, want, what):
    assert got.shape == want.shape, f"{what}: {got.shape} vs {want.shape}"
    if not np.array_equal(got, want):
        k = int(np.nonzero((got != want).any(1))[0][0])
        raise AssertionError(f"{what}: first difference at {k}: {got[k]} vs {want[k]}")


def test_join_uniform_vs_clustered(rt, ora):
    """Scaled-down join of a uniform and a clustered relation (fanout 32, SoA)."""
    a, b = rtgen.c3_join(100_000)
    say("case join 100k x 100k F32 soa")
    got = rt.spatial_join(rt.build_str(a, 32, "soa"), rt.build_str(b, 32, "soa"))
    want = ora.join(ora.build_str(a, 32), ora.build_str(b, 32))
    # E[pairs] = NA * NB * (E[wA] + E[wB])^2 = 1e10 * (5e-4)^2 = 2500
    assert 2000 < want.shape[0] < 3000
    assert_pairs_equal(got, want, "join")


@pytest.mark.parametrize("fa,fb,la,lb", [(4, 64, "soa", "aos"), (64, 3, "aos", "soa"), (16, 16, "d2", "soa"),
                                         (2, 33, "soa", "d2"), (32, 32, "aos", "aos")])
def test_join_unequal_heights_and_layouts(rt, ora, fa, fb, la, lb):
    for s, (na, nb) in enumerate([(0, 10), (1, 1), (5, 3000), (2500, 40), (3000, 3000)]):
        say(f"case join Fa={fa} Fb={fb} {la}/{lb} na={na} nb={nb}")
        A = rtgen.adversarial_rects(na, 10 * s + fa) if na else np.zeros((0, 4), np.float32)
        B = rtgen.adversarial_rects(nb, 10 * s + fb + 5) if nb else np.zeros((0, 4), np.float32)
        got = rt.spatial_join(rt.build_str(A, fa, la), rt.build_str(B, fb, lb))
        want = ora.brute_join(A, B)
        assert_pairs_equal(got, want, f"Fa={fa} Fb={fb} na={na} nb={nb}")


def test_join_swap_symmetry(rt):
    a, b = rtgen.c3_join(20_000, seed_base=3100)
    ta, tb = rt.build_str(a, 16, "soa"), rt.build_str(b, 64, "aos")
    j = rt.spatial_join(ta, tb)
    js = rt.spatial_join(tb, ta)[:, ::-1]
    js = js[np.lexsort((js[:, 1], js[:, 0]))]
    assert np.array_equal(j, js)


def _small_batch(scale=0.02, ntrees=24):
    return rtgen.c4_batch(ntrees=ntrees, scale=scale, seed_base=4400)


def test_batch_matches_oracle_and_plain(rt, ora):
    """Many uneven trees (mixed fanout and layout) in one persistent, graph-
    replayed launch: each instance's CSR equals the oracle's, with the fill
    replaying the count pass's records and with the walking fill; the plain
    per-tree launch sequence gives the same results."""
    inst = _small_batch()
    trees, qs, wants = [], [], []
    for k, x in enumerate(inst):
        F = [16, 32, 64][k % 3]
        lay = ["aos", "soa", "d2"][(k // 3) % 3]
        trees.append(rt.build_str(x.rects, F, lay))
        qs.append(x.queries)
        wants.append(ora.select(ora.build_str(x.rects, 16), x.queries))
    say(f"case batch {len(trees)} trees")
    b = rt.Batch(trees, qs)
    for rep in range(3):
        b.run()
        tot, flags = b.status()
        assert flags == 0, flags
        assert tot == sum(int(w[0][-1]) for w in wants)
        chunks, over = b.replay_info()
        assert chunks > 0 and not over, "the graph's fill did not replay the count pass's records"
        for i, w in enumerate(wants):
            got = b.result(i)
            assert np.array_equal(got[0], w[0]) and np.array_equal(got[1], w[1]), (rep, i)
    # the walking fill in the graph gives the same results
    b.set_replay(False)
    for rep in range(2):
        b.run()
        assert b.status() == (tot, 0) and b.replay_info() == (0, False)
        for i, w in enumerate(wants):
            got = b.result(i)
            assert np.array_equal(got[0], w[0]) and np.array_equal(got[1], w[1]), ("walk", rep, i)
    b.set_replay(True)
    b.run()
    assert b.status() == (tot, 0) and b.replay_info()[0] > 0
    with pytest.raises(rt.RTError):
        rt._check(rt._L.rt_batch_set_replay(b.h, 2))
    b.run_plain()
    tot, flags = b.status()
    assert flags == 0
    for i, w in enumerate(wants):
        got = b.result(i)
        assert np.array_equal(got[0], w[0]) and np.array_equal(got[1], w[1]), ("plain", i)
    outs = rt.range_select_batch(trees, qs)
    for i, w in enumerate(wants):
        assert np.array_equal(outs[i][0], w[0]) and np.array_equal(outs[i][1], w[1])


def test_batch_small_pool_flags_overflow(rt):
    inst = _small_batch(scale=0.01, ntrees=6)
    trees = [rt.build_str(x.rects, 32, "soa") for x in inst]
    full = rt.Batch(trees, [x.queries for x in inst])
    full.run()
    tot, _ = full.status()
    if tot < 2:
        pytest.skip("too few results to shrink the pool")
    small = rt.Batch(trees, [x.queries for x in inst], ids_capacity=tot - 1)
    small.run()
    t2, flags = small.status()
    assert t2 == tot and (flags & 1)


def test_autotuner_choice_is_valid_and_exact(rt, ora, tmp_path):
    """The autotuner times every candidate, caches its choice, and the tree it
    builds returns the oracle's CSR."""
    from paper_2309_16913_amd.autotune import Autotuner
    r = rtgen.c2_rects(120_000, seed_base=2300)
    q = rtgen.c2_queries(3000, seed_base=2300)
    cache = str(tmp_path / "tune.json")
    tu = Autotuner(cache_path=cache, fanouts=(16, 32), layouts=("aos", "soa"), kmins=(0, 4), sample=2000, reps=1)
    t, c = tu.build(r, q, "mixed")
    assert c["cached"] is False and len(c["timings_ms"]) == 8
    assert (c["fanout"], c["layout"], c["kmin"]) in {(F, L, K) for F in (16, 32) for L in ("aos", "soa")
                                                     for K in (0, 4)}
    got = rt.range_select(t, q)
    want = ora.select(ora.build_str(r, 16), q)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    tu2 = Autotuner(cache_path=cache, fanouts=(16, 32), layouts=("aos", "soa"), kmins=(0, 4), sample=2000, reps=1)
    c2 = tu2.tune(r, q, "mixed")
    assert c2["cached"] is True and c2["fanout"] == c["fanout"] and c2["layout"] == c["layout"]
