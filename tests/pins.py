"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code path.

Each pin takes an ``oracle.Oracle`` instance and raises AssertionError on a
mismatch, so the same pins can be run against deliberately broken oracle
builds (mutants) to show that they catch plausible mistakes.
"""

from __future__ import annotations

import math
import os

import numpy as np

import rtgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _f32(tok: str) -> np.float32:
    return np.float32(float(tok))


def load_handworked():
    rects, queries, expect = {}, [], []
    join_a = join_b = None
    pairs = None
    with open(os.path.join(GOLDEN, "select_handworked.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, _, tail = line.partition(":")
            tok = head.split()
            if tok[0] == "rect":
                rects[int(tok[1])] = [_f32(t) for t in tok[2:6]]
            elif tok[0] == "query":
                queries.append([_f32(t) for t in tok[2:6]])
                expect.append([int(t) for t in tail.split()])
            elif tok[0] == "joinA":
                join_a = [int(t) for t in tok[1:]]
            elif tok[0] == "joinB":
                join_b = [int(t) for t in tok[1:]]
            elif tok[0] == "pairs":
                pairs = [tuple(int(v) for v in p.split(",")) for p in tail.split()]
    R = np.array([rects[i] for i in sorted(rects)], dtype=np.float32)
    Q = np.array(queries, dtype=np.float32)
    return R, Q, expect, R[join_a], R[join_b], pairs


def segments(off, ids):
    return [ids[int(off[k]):int(off[k + 1])].tolist() for k in range(len(off) - 1)]


# ---------------------------------------------------------------------------
def pin_handworked(o, fanouts=(2, 3, 4)):
    """Hand-worked golden values (closed predicate, section 3 / 4.1)."""
    R, Q, expect, A, B, pairs = load_handworked()
    for F in fanouts:
        t = o.build_str(R, F)
        off, ids = o.select(t, Q)
        got = segments(off, ids)
        assert got == expect, f"F={F}: {got} != {expect}"
        ta, tb = o.build_str(A, F), o.build_str(B, F)
        p = [tuple(x) for x in o.join(ta, tb).tolist()]
        assert p == pairs, f"join F={F}: {p} != {pairs}"
    # brute force too: it is the definition written as nested loops
    off, ids = o.brute_select(R, Q)
    assert segments(off, ids) == expect
    assert [tuple(x) for x in o.brute_join(A, B).tolist()] == pairs


def pin_select_vs_brute(o, seeds=range(20), sizes=(0, 1, 2, 5, 16, 17, 64, 65, 300, 1500),
                        fanouts=(2, 3, 4, 8, 16, 32, 64)):
    """Tree search equals the nested-loop scan on adversarial inputs (touching
    edges, points, segments, duplicates, infinite windows)."""
    for s in seeds:
        for n in sizes:
            F = fanouts[(s + n) % len(fanouts)]
            r = rtgen.adversarial_rects(n, 100 + s) if n else np.zeros((0, 4), np.float32)
            q = rtgen.adversarial_windows(40, 500 + s)
            t = o.build_str(r, F)
            a = o.select(t, q)
            b = o.brute_select(r, q)
            assert np.array_equal(a[0], b[0]), f"seed {s} n {n} F {F}: counts differ"
            assert np.array_equal(a[1], b[1]), f"seed {s} n {n} F {F}: ids differ"


def pin_join_vs_brute(o, seeds=range(12)):
    """Synchronized traversal equals the nested-loop join, including trees of
    different heights and empty relations."""
    for s in seeds:
        na = [0, 1, 7, 40, 200, 900][s % 6]
        nb = [3, 0, 50, 700, 64, 65][(s * 5) % 6]
        Fa = [2, 4, 8, 16, 3, 32][s % 6]
        Fb = [5, 16, 2, 8, 64, 4][(s + 1) % 6]
        A = rtgen.adversarial_rects(na, 900 + s) if na else np.zeros((0, 4), np.float32)
        B = rtgen.adversarial_rects(nb, 950 + s) if nb else np.zeros((0, 4), np.float32)
        p = o.join(o.build_str(A, Fa), o.build_str(B, Fb))
        q = o.brute_join(A, B)
        assert np.array_equal(p, q), f"seed {s}: join != brute ({p.shape} vs {q.shape})"


def pin_join_is_union_of_selects(o, seed=3):
    """J(A,B) = union over a of {(a,b) : b in select_B(A[a])}, and
    J(A,B) = swap(J(B,A)): two routes independent of the join recursion."""
    A = rtgen.uniform_rects(3000, 0.01, seed)
    B = rtgen.clustered_rects(2500, 5, 0.05, 0.01, seed + 1)
    ta, tb = o.build_str(A, 8), o.build_str(B, 16)
    J = o.join(ta, tb)
    off, ids = o.select(tb, A)
    cnt = np.diff(off.astype(np.int64))
    U = np.stack([np.repeat(np.arange(A.shape[0], dtype=np.uint32), cnt), ids], axis=1)
    assert np.array_equal(J, U)
    Js = o.join(tb, ta)[:, ::-1]
    order = np.lexsort((Js[:, 1], Js[:, 0]))
    assert np.array_equal(J, Js[order])


def pin_closed_form_uniform(o):
    """Uniform rectangles with sides U[0,s] and square windows of side w inside
    the unit square: E[#hits] = N * (w + s/2)^2 (the window grows by the mean
    side on the low sides).  The same mean also checks the
    C1-sized tree: ~11.0 hits per query."""
    N, s, w = 100_000, 1e-3, 0.01
    r = rtgen.uniform_rects(N, s, 7)
    g = rtgen.rng(8)
    c = g.uniform(0.02, 0.98, size=(2, 4000))
    q = np.stack([c[0] - w / 2, c[1] - w / 2, c[0] + w / 2, c[1] + w / 2], 1).astype(np.float32)
    t = o.build_str(r, 16)
    off, ids = o.select(t, q)
    cnt = np.diff(off.astype(np.int64))
    expect = N * (w + s / 2) ** 2
    se = math.sqrt(expect / len(cnt))          # Poisson standard error of the mean
    assert abs(cnt.mean() - expect) < 5 * se, (cnt.mean(), expect)


def pin_closed_form_join(o):
    """Two uniform relations with sides U[0,s]: E[#pairs] = NA*NB*(E[wA]+E[wB])^2
    for objects away from the border; here (s/2 + s/2)^2 = s^2."""
    N, s = 20_000, 2e-3
    A = rtgen.uniform_rects(N, s, 11)
    B = rtgen.uniform_rects(N, s, 12)
    p = o.join(o.build_str(A, 16), o.build_str(B, 32))
    expect = N * N * s * s
    assert abs(p.shape[0] - expect) < 5 * math.sqrt(expect) + 0.01 * expect, (p.shape[0], expect)


def pin_tree_shape(o):
    """STR packs every level completely except possibly its last node:
    nodes per level = ceil(count / F) repeated until one node is left; every
    invariant of the checker holds."""
    for n, F in [(1, 4), (4, 4), (5, 4), (100, 2), (1000, 16), (4097, 64), (33, 32), (99_991, 16)]:
        r = rtgen.uniform_rects(n, 1e-3, n + F)
        t = o.build_str(r, F)
        rc, msg = o.check(t, r)
        assert rc == 0, (n, F, msg)
        A = t.arrays()
        levels = np.bincount(A["level"].astype(np.int64)).tolist()
        exp, c = [], n
        while c > F:
            c = -(-c // F)
            exp.append(c)
        exp.append(1)                   # the root
        assert levels == exp, (n, F, levels, exp)
        assert t.height == len(exp)


def pin_special_cases(o):
    """Empty relation, select-all window, identical rectangles, n = F and F+1."""
    q = np.array([[-np.inf, -np.inf, np.inf, np.inf], [0.5, 0.5, 0.5, 0.5]], np.float32)
    t = o.build_str(np.zeros((0, 4), np.float32), 8)
    off, ids = o.select(t, q)
    assert off.tolist() == [0, 0, 0] and ids.size == 0
    same = np.tile(np.array([[0.25, 0.25, 0.75, 0.75]], np.float32), (37, 1))
    for F in (2, 4, 36, 37, 38):
        t = o.build_str(same, F)
        off, ids = o.select(t, q)
        assert ids.tolist() == list(range(37)) * 2
    # degenerate windows on a coarse grid
    r = rtgen.adversarial_rects(500, 77)
    t = o.build_str(r, 4)
    off, ids = o.select(t, q[:1])
    assert ids.tolist() == list(range(500))


def pin_results_canonical(o):
    """Results are strictly ascending per query (sorted, duplicate-free) and every
    reported id intersects its window (soundness, checked per element)."""
    r = rtgen.clustered_rects(20_000, 8, 0.05, 5e-3, 21)
    q = rtgen.windows_loguniform(300, 1e-5, 1e-2, 22)
    t = o.build_str(r, 16)
    off, ids = o.select(t, q)
    for k in range(q.shape[0]):
        s = ids[int(off[k]):int(off[k + 1])]
        assert np.all(np.diff(s.astype(np.int64)) > 0)
        e = r[s]
        w = q[k]
        assert np.all((e[:, 0] <= w[2]) & (w[0] <= e[:, 2]) & (e[:, 1] <= w[3]) & (w[1] <= e[:, 3]))


# ---------------------------------------------------------------------------
# join over nodes sorted by low x (section 4.1 pruning, section 4.2 many-to-many)

def load_m2m_example():
    v = {}
    with open(os.path.join(GOLDEN, "m2m_worked_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            v[tok[0]] = tok[1:]
    return v


def pin_m2m_worked_example(o):
    """The index update printed in section 4.2: gather [2,2,2,2] with mask
    0b1001 gives flip [x,2,2,x] and next gather [3,1,1,3]; and the finished
    search on values that produce that mask ends at the hand-worked stops."""
    v = load_m2m_example()
    g, f = o.m2m_update(int(v["mask"][0], 0), int(v["step"][0]), int(v["n_pow"][0]),
                        [int(x) for x in v["gidx"]], [int(x) for x in v["flip"]])
    assert g.tolist() == [int(x) for x in v["gidx_next"]], g
    assert f.tolist() == [int(x) for x in v["flip_next"]], f
    lx = np.array([_f32(x) for x in v["in_lx"]], np.float32)
    hx = np.array([_f32(x) for x in v["out_hx"]], np.float32)
    mask = sum(1 << k for k in range(4) if hx[k] >= lx[2])
    assert mask == int(v["mask"][0], 0)
    assert o.m2m_flip(hx, lx).tolist() == [int(x) for x in v["flip_final"]]


def pin_m2m_flip_is_lower_bound(o, seed=11):
    """The finished many-to-many search equals the plain definition: the
    first inner position whose low x exceeds the outer high x (a binary
    search over the sorted low x values), for every inner size 0..64,
    with ties, touching values and infinities."""
    g = np.random.default_rng(seed)
    for n_in in range(0, 65):
        for rep in range(3):
            lx = np.sort(g.integers(0, 12, n_in).astype(np.float32) / 8)
            if n_in and rep == 2:
                lx[0] = -np.inf
            w = int(g.integers(1, 65))
            hx = g.integers(-2, 14, w).astype(np.float32) / 8
            hx[g.random(w) < 0.1] = np.inf
            hx[g.random(w) < 0.1] = -np.inf
            want = np.searchsorted(lx, hx, side="right")
            got = o.m2m_flip(hx, lx)
            assert np.array_equal(got, want), (n_in, rep, lx, hx, got, want)


def pin_join_pruned_vs_brute(o, seeds=range(10)):
    """Pruning never changes the pair set: every combination of O3, O4 and
    O5 over low-x-sorted nodes equals the nested-loop join; O4 and O5 stop the
    inner scan at the same place, and pruning only ever removes predicate
    evaluations."""
    for s in seeds:
        na = [1, 7, 40, 200, 900, 1500][s % 6]
        nb = [3, 50, 700, 64, 65, 1200][(s * 5) % 6]
        Fa = [2, 4, 8, 16, 3, 32][s % 6]
        Fb = [5, 16, 2, 8, 64, 4][(s + 1) % 6]
        A = rtgen.adversarial_rects(na, 1900 + s)
        B = rtgen.adversarial_rects(nb, 1950 + s)
        ta, tb = o.build_str(A, Fa), o.build_str(B, Fb)
        o.sort_entries_lx(ta)
        o.sort_entries_lx(tb)
        assert o.check(ta, A)[0] == 0 and o.check(tb, B)[0] == 0
        want = o.brute_join(A, B)
        tests = {}
        for flags in (0, o.O3, o.O4, o.O5, o.O3 | o.O4, o.O3 | o.O5):
            p, t = o.join_opt(ta, tb, flags)
            assert np.array_equal(p, want), f"seed {s} flags {flags}: {p.shape} vs {want.shape}"
            tests[flags] = t
        assert tests[o.O4] == tests[o.O5] and tests[o.O3 | o.O4] == tests[o.O3 | o.O5], tests
        assert tests[o.O3 | o.O5] <= tests[o.O3] <= tests[0], tests
        assert tests[o.O5] <= tests[0], tests
    # pruning needs sorted nodes: STR orders a node's entries by y-center, so
    # this unsorted tree is refused
    t = o.build_str(rtgen.uniform_rects(500, 0.05, 5), 8)
    try:
        o.join_opt(t, t, o.O3)
    except ValueError:
        pass
    else:
        raise AssertionError("pruned join accepted nodes not sorted by low x")


ALL_PINS = [pin_handworked, pin_select_vs_brute, pin_join_vs_brute, pin_join_is_union_of_selects,
            pin_closed_form_uniform, pin_closed_form_join, pin_tree_shape, pin_special_cases,
            pin_results_canonical, pin_m2m_worked_example, pin_m2m_flip_is_lower_bound,
            pin_join_pruned_vs_brute]


# ---------------------------------------------------------------------------
# the invariant checker rejects broken trees (section 2.3: a node holds up to
# F entries (MBR, ptr) plus its level and entry count; an internal entry's MBR
# bounds its child's entries)
# ---------------------------------------------------------------------------

def _corrupt_cases(A, rects):
    """(name, arrays, rects to check against, expected code) for one fault
    each, applied to the node/entry arrays A of a valid tree (height >= 3)."""
    def cp():
        return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in A.items()}
    lev, cnt, first, ptr = A["level"], A["count"], A["first"], A["ptr"]
    root = int(A["root"])
    r0 = int(first[root])                      # the root's first entry
    child = int(ptr[r0])                       # an internal child of the root
    assert lev[child] >= 1
    leaves = np.nonzero(lev == 0)[0]
    le = [int(first[u]) for u in leaves if cnt[u] >= 1]
    out = []

    B = cp()
    B["hx"][r0] = np.nextafter(B["hx"][r0], np.float32(np.inf))
    out.append(("parent MBR grown", B, rects, 15))
    B = cp()
    B["lx"][r0] = np.nextafter(B["lx"][r0], np.float32(np.inf))
    out.append(("parent MBR shrunk", B, rects, 15))
    B = cp()
    B["ptr"][le[1]] = B["ptr"][le[0]]
    out.append(("object twice", B, None, 9))
    B = cp()
    B["n_objects"] = int(A["n_objects"]) + 1
    out.append(("object missing (count claims one more)", B, rects, 16))
    # a real missing object: drop from a leaf an entry that lies strictly
    # inside the union of its siblings (so no MBR above changes)
    for u in leaves:
        f0, c = int(first[u]), int(cnt[u])
        if c < 3:
            continue
        E = np.stack([A["lx"][f0:f0 + c], A["ly"][f0:f0 + c], A["hx"][f0:f0 + c], A["hy"][f0:f0 + c]], 1)
        for j in range(c):
            o = np.delete(E, j, 0)
            if (E[j, 0] > o[:, 0].min() and E[j, 1] > o[:, 1].min() and E[j, 2] < o[:, 2].max()
                    and E[j, 3] < o[:, 3].max()):
                B = cp()
                last = f0 + c - 1
                for k in ("lx", "ly", "hx", "hy", "ptr"):
                    B[k][f0 + j], B[k][last] = B[k][last], B[k][f0 + j]
                B["count"][u] = c - 1
                out.append(("object missing (dropped from its leaf)", B, rects, 16))
                break
        else:
            continue
        break
    else:
        raise AssertionError("no leaf entry strictly inside its siblings' union")
    R = np.array(rects, np.float32, copy=True)
    k = int(ptr[le[2]])
    R[k, 2] = np.nextafter(R[k, 2], np.float32(np.inf))
    out.append(("leaf rectangle differs from the input", cp(), R, 10))
    B = cp()
    B["level"][child] += 1
    out.append(("child level", B, rects, 13))
    B = cp()
    B["level"][root] += 1
    out.append(("root level", B, rects, 3))
    B = cp()
    B["fanout"] = int(A["fanout"]) - 1
    out.append(("count > F", B, rects, 4))
    B = cp()
    B["count"][child] = 0
    out.append(("empty non-root node", B, rects, 14))
    B = cp()
    for k, v in (("level", 0), ("count", 1), ("first", 0)):
        B[k] = np.append(B[k], np.array([v], B[k].dtype))
    out.append(("unreachable node", B, rects, 17))
    B = cp()
    B["ptr"][r0 + 1] = B["ptr"][r0]
    out.append(("node reached twice", B, rects, 12))
    B = cp()
    B["ptr"][r0] = B["level"].shape[0]
    out.append(("child out of range", B, rects, 11))
    B = cp()
    B["lx"][r0] = np.float32(np.nan)
    out.append(("NaN entry", B, rects, 7))
    return out


def pin_checker_rejects_corruptions(o):
    """The invariant checker accepts the oracle's STR tree and the library's
    tree shape (the numpy statement in str_shape.py), and returns the
    distinct code of each single planted fault: parent MBR grown or shrunk,
    an object twice or missing, a leaf rectangle unlike the input, a wrong
    level, a node over F entries, an empty or unreachable node, a node
    reached twice, a child out of range, a NaN entry."""
    from str_shape import expected_export
    r = rtgen.uniform_rects(2000, 2e-2, 4242)
    trees = []
    t = o.build_str(r, 8)
    trees.append(("oracle STR", t.arrays()))
    ex = expected_export(r, 8)
    ex.update(root=0, fanout=8, n_objects=r.shape[0])
    trees.append(("library shape", ex))
    for what, A in trees:
        assert int(A["height"]) >= 3
        good = o.tree_from_arrays(**{k: A[k] for k in ("fanout", "height", "root", "n_objects", "level", "count",
                                                       "first", "lx", "ly", "hx", "hy", "ptr")})
        rc, msg = o.check(good, r)
        assert rc == 0, (what, msg)
        for name, B, rr, code in _corrupt_cases(A, r):
            bad = o.tree_from_arrays(**{k: B[k] for k in ("fanout", "height", "root", "n_objects", "level",
                                                          "count", "first", "lx", "ly", "hx", "hy", "ptr")})
            rc, msg = o.check(bad, rr)
            assert rc == code, f"{what}, {name}: checker returned {rc} ({msg}), expected {code}"


ALL_PINS.append(pin_checker_rejects_corruptions)


def pin_threaded_drivers_match(o):
    """The threaded select and join (timing baseline for all host cores)
    return exactly the single-thread results, for thread counts that do and
    do not divide the work, and on empty inputs."""
    r = rtgen.clustered_rects(30_000, 8, 0.05, 3e-3, 31)
    q = rtgen.windows_loguniform(777, 1e-6, 1e-2, 32)
    t = o.build_str(r, 16)
    off, ids = o.select(t, q)
    for nt in (1, 3, 8, 1000):
        off2, ids2 = o.select_mt(t, q, nt)
        assert np.array_equal(off, off2) and np.array_equal(ids, ids2), nt
    off2, ids2 = o.select_mt(t, q[:0], 4)
    assert off2.tolist() == [0] and ids2.size == 0
    A = rtgen.uniform_rects(8000, 4e-3, 33)
    B = rtgen.clustered_rects(9000, 4, 0.05, 4e-3, 34)
    for Fa, Fb in ((8, 8), (4, 32)):   # equal and unequal heights
        ta, tb = o.build_str(A, Fa), o.build_str(B, Fb)
        want = o.join(ta, tb)
        for nt in (1, 5, 64):
            assert np.array_equal(o.join_mt(ta, tb, nt), want), (Fa, Fb, nt)
    e = o.build_str(np.zeros((0, 4), np.float32), 8)
    assert o.join_mt(e, ta, 4).shape == (0, 2)


ALL_PINS.append(pin_threaded_drivers_match)
