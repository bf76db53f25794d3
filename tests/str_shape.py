"""Expected shape of the library's STR trees, written out in numpy for tests.

The library bulk-loads with Sort-Tile-Recursive (Leutenegger, Lopez,
Edgington 1997; the paper leaves construction open).  Its exact tree follows
from these rules, restated here independently of the library's code:

  * a level of c > F items gets P = ceil(c/F) nodes and S = ceil(sqrt(P))
    vertical slices of S*F items; the items are ranked by x-center, the item
    of x-rank p goes to slice p // (S*F); the packing order sorts by
    (slice, y-center, item index); consecutive runs of F items of it form the
    level's nodes, node k holding packing positions [kF, kF+F);
  * centers are the float32 value 0.5*lo + 0.5*hi (each operation rounded to
    float32), compared as numbers; x ties are broken by item index;
  * a level of c <= F items is the root, holding them in index order;
  * node MBRs (exact min/max of their items) are the next level's items;
  * numbering is breadth first from the root; the children of each node are
    stored contiguously in its entry order;
  * with the low-x option, the entries of every node are reordered by
    ascending low x (ties keep their order) before the numbering.

`expected_export` gives the same arrays as `Tree.export()`.
"""

from __future__ import annotations

import numpy as np


def _ceil_sqrt(p: int) -> int:
    s = int(np.sqrt(p))
    while s * s < p:
        s += 1
    while s > 1 and (s - 1) * (s - 1) >= p:
        s -= 1
    return s


def _centers(items: np.ndarray, lo: int, hi: int) -> np.ndarray:
    h = np.float32(0.5)
    with np.errstate(invalid="ignore"):   # -inf..+inf gives a NaN center, ordered last
        return (h * items[:, lo]).astype(np.float32) + (h * items[:, hi]).astype(np.float32)


def packing_order(items: np.ndarray, F: int) -> np.ndarray:
    c = items.shape[0]
    if c <= F:
        return np.arange(c, dtype=np.int64)
    P = -(-c // F)
    slice_len = _ceil_sqrt(P) * F
    idx = np.arange(c, dtype=np.int64)
    cx = _centers(items, 0, 2).astype(np.float64)
    xorder = np.lexsort((idx, cx))             # by x-center, then index
    xrank = np.empty(c, np.int64)
    xrank[xorder] = idx
    cy = _centers(items, 1, 3).astype(np.float64)
    return np.lexsort((idx, cy, xrank // slice_len))


def sort_runs_lx(items: np.ndarray, order: np.ndarray, F: int) -> np.ndarray:
    """Reorder each run of F packing positions (one node) by ascending low x,
    ties keeping their packing order."""
    out = order.copy()
    for k0 in range(0, order.shape[0], F):
        run = order[k0:k0 + F]
        out[k0:k0 + F] = run[np.argsort(items[run, 0], kind="stable")]
    return out


def expected_export(rects, F: int, sort_lx: bool = False) -> dict:
    items = np.ascontiguousarray(rects, np.float32).reshape(-1, 4)
    levels = []   # (items, packing order, node count), leaves first
    while True:
        c = items.shape[0]
        order = packing_order(items, F)
        if sort_lx:
            order = sort_runs_lx(items, order, F)
        P = -(-c // F) if c > F else 1
        mbr = np.full((P, 4), np.nan, np.float32)
        for k in range(P):
            grp = items[order[k * F:(k + 1) * F]]
            if grp.shape[0]:
                mbr[k] = (grp[:, 0].min(), grp[:, 1].min(), grp[:, 2].max(), grp[:, 3].max())
        levels.append((items, order, P))
        if c <= F:
            break
        items = mbr
    H = len(levels)
    # stored order of every level, root first
    stored = [None] * H
    stored[H - 1] = np.zeros(1, np.int64)
    for l in range(H - 1, 0, -1):
        it, order, P = levels[l]
        stored[l - 1] = np.concatenate([order[k * F:(k + 1) * F] for k in stored[l]]) if P else np.zeros(0, np.int64)
    first_node = {}
    g = 0
    for l in range(H - 1, -1, -1):
        first_node[l] = g
        g += len(stored[l])
    glob = []
    for l in range(H):
        a = np.empty(len(stored[l]), np.int64)
        a[stored[l]] = first_node[l] + np.arange(len(stored[l]))
        glob.append(a)
    lev, cnt, first, ent, ptr = [], [], [], [], []
    e = 0
    for l in range(H - 1, -1, -1):
        it, order, P = levels[l]
        for k in stored[l]:
            sel = order[k * F:(k + 1) * F]
            lev.append(l)
            cnt.append(len(sel))
            first.append(e)
            e += len(sel)
            ent.append(it[sel])
            ptr.append(sel if l == 0 else glob[l - 1][sel])
    ent = np.concatenate(ent) if ent else np.zeros((0, 4), np.float32)
    ptr = np.concatenate(ptr) if ptr else np.zeros(0, np.int64)
    return dict(level=np.array(lev, np.uint32), count=np.array(cnt, np.uint32), first=np.array(first, np.uint64),
                lx=ent[:, 0].copy(), ly=ent[:, 1].copy(), hx=ent[:, 2].copy(), hy=ent[:, 3].copy(),
                ptr=ptr.astype(np.uint32), height=H)


def assert_export_equal(got: dict, want: dict, what: str = ""):
    assert int(got["height"]) == int(want["height"]), what
    for k in ("level", "count", "first", "ptr"):
        assert got[k].shape == want[k].shape, (what, k)
        if not np.array_equal(got[k], want[k]):
            i = int(np.nonzero(got[k] != want[k])[0][0])
            raise AssertionError(f"{what}: {k} differs first at {i}: {got[k][i]} vs {want[k][i]}")
    for k in ("lx", "ly", "hx", "hy"):   # compared as numbers: -0.0 == +0.0
        assert np.array_equal(got[k], want[k]), (what, k)
