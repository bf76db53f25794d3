"""The numpy statement of the library's STR tree shape (tests/str_shape.py)
produces valid R-trees: the oracle's checker accepts them (MBR unions, one
leaf entry per object with its own rectangle, levels, counts), children are
contiguous, and the slice/run rules hold."""

import numpy as np
import pytest

import oracle
import rtgen
from str_shape import expected_export, packing_order


@pytest.fixture(scope="module")
def ora():
    return oracle.get()


@pytest.mark.parametrize("n,F", [(0, 8), (1, 16), (16, 16), (17, 16), (1000, 4), (5000, 7), (20000, 64)])
def test_expected_export_is_valid_tree(ora, n, F):
    r = rtgen.clustered_rects(n, 4, 0.05, 1e-3, 100 + n) if n else np.zeros((0, 4), np.float32)
    ex = expected_export(r, F)
    t = ora.tree_from_arrays(**ex, root=0, fanout=F, n_objects=n)
    rc, msg = ora.check(t, r)
    assert rc == 0, msg
    for u in np.nonzero(ex["level"] > 0)[0]:
        f0, c = int(ex["first"][u]), int(ex["count"][u])
        p = ex["ptr"][f0:f0 + c].astype(np.int64)
        assert np.array_equal(p, p[0] + np.arange(c))
    # every node but the last-created of its level is full
    for l in range(int(ex["height"])):
        cnt = ex["count"][ex["level"] == l]
        assert int((cnt < F).sum()) <= 1


def test_packing_order_slices():
    """Brute-force restatement on a tiny level: positions inside one slice
    are ordered by y-center, and the slices are ordered by x-center."""
    r = rtgen.uniform_rects(300, 0.01, 7)
    F = 4
    order = packing_order(r, F)
    P = -(-300 // F)
    S = int(np.ceil(np.sqrt(P)))
    L = S * F
    h = np.float32(0.5)
    cx = h * r[:, 0] + h * r[:, 2]
    cy = h * r[:, 1] + h * r[:, 3]
    assert cx.dtype == np.float32
    for s0 in range(0, 300, L):
        sl = order[s0:s0 + L]
        assert np.all(np.diff(cy[sl]) >= 0)
        if s0 + L < 300:
            nxt = order[s0 + L:s0 + 2 * L]
            assert cx[sl].max() <= cx[nxt].min()
