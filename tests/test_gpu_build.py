"""GPU STR bulk load: the device builder (through rt_build_str with host
rectangles and rt_build_str_device with device rectangles) produces exactly
the tree that the STR rules give (tests/str_shape.py), a tree that the
oracle's checker accepts, and selects on it match the oracle."""

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


def _cases():
    z = np.zeros((0, 4), np.float32)
    inf = np.float32(np.inf)
    special = np.array([[-inf, -inf, inf, inf], [-0.0, -0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0],
                        [-inf, 0.25, 0.5, 0.5], [0.1, -inf, 0.2, 0.3], [0.5, 0.5, inf, inf]] * 40, np.float32)
    return [
        ("empty", z, 8, "soa"),
        ("one", rtgen.uniform_rects(1, 0.1, 1), 16, "aos"),
        ("full-root", rtgen.uniform_rects(64, 0.1, 2), 64, "soa"),
        ("root+1", rtgen.uniform_rects(65, 0.1, 3), 64, "d2"),
        ("F2", rtgen.uniform_rects(1000, 0.01, 4), 2, "soa"),
        ("clustered", rtgen.clustered_rects(50_000, 5, 0.05, 1e-3, 5), 32, "aos"),
        ("ragged", rtgen.clustered_rects(123_457, 9, 0.02, 1e-3, 6), 7, "d2"),
        ("adversarial", rtgen.adversarial_rects(20_000, 7), 16, "soa"),
        ("inf-zero", special, 5, "aos"),
        ("c2-like", rtgen.c2_rects(200_000), 64, "soa"),
    ]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_build_matches_str_rules(rt, ora, case):
    import torch
    name, r, F, layout = case
    say("build", name, r.shape[0], F, layout)
    want = expected_export(r, F)
    t = rt.build_str(r, F, layout)
    assert_export_equal(t.export(), want, f"{name} host input")
    t.free()
    d = torch.from_numpy(np.ascontiguousarray(r)).cuda() if r.shape[0] else torch.zeros(1, 4, device="cuda")
    s = torch.cuda.current_stream()
    td = rt.build_str_device(d.data_ptr(), r.shape[0], F, layout, s.cuda_stream)
    ex = td.export()
    assert_export_equal(ex, want, f"{name} device input")
    ot = ora.tree_from_arrays(**ex)
    rc, msg = ora.check(ot, r)
    assert rc == 0, (name, msg)
    td.free()


def test_device_build_select_parity(rt, ora):
    import torch
    r = rtgen.c2_rects(300_000)
    q = rtgen.c2_queries(20_000)
    want = ora.select(ora.build_str(r, 32), q)
    d = torch.from_numpy(r).cuda()
    for F, layout in [(16, "aos"), (32, "soa"), (64, "d2")]:
        t = rt.build_str_device(d.data_ptr(), r.shape[0], F, layout, torch.cuda.current_stream().cuda_stream)
        off, ids = rt.range_select(t, q)
        assert np.array_equal(off, want[0]) and np.array_equal(ids, want[1]), (F, layout)
        t.free()


def test_device_build_rejects_bad_rects(rt):
    import torch
    r = rtgen.uniform_rects(5000, 0.01, 9)
    for bad in ("nan", "flip"):
        x = r.copy()
        if bad == "nan":
            x[4321, 1] = np.nan
        else:
            x[17, 0], x[17, 2] = 0.9, 0.1
        d = torch.from_numpy(x).cuda()
        with pytest.raises(rt.RTError) as e:
            rt.build_str_device(d.data_ptr(), x.shape[0], 16, "soa", 0)
        assert e.value.code == rt.RT_EINVAL
        with pytest.raises(rt.RTError):
            rt.build_str(x, 16, "soa")
    # misaligned pointer
    d = torch.from_numpy(np.concatenate([np.zeros(1, np.float32), r.ravel()])).cuda()
    with pytest.raises(rt.RTError):
        rt.build_str_device(d.data_ptr() + 4, r.shape[0], 16, "soa", 0)
