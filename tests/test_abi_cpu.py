"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/rt.h declares, and rejects bad arguments before touching a GPU."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "rt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2309_16913_amd as rt
    lib = C.CDLL(rt.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(rt.exported_symbols())


def test_version_string():
    import paper_2309_16913_amd as rt
    assert "gfx950" in rt.version()


@pytest.mark.parametrize("bad", [
    np.array([[0, 0, np.nan, 1]], np.float32),
    np.array([[1, 0, 0, 1]], np.float32),       # lx > hx
    np.array([[0, 1, 1, 0]], np.float32),       # ly > hy
])
def test_build_rejects_invalid_rectangles(bad):
    import paper_2309_16913_amd as rt
    with pytest.raises(rt.RTError) as ei:
        rt.build_str(bad, 16, "soa")
    assert ei.value.code == rt.RT_EINVAL


@pytest.mark.parametrize("fanout", [1, 65, 1000])
def test_build_rejects_bad_fanout(fanout):
    import paper_2309_16913_amd as rt
    with pytest.raises(rt.RTError) as ei:
        rt.build_str(np.zeros((4, 4), np.float32), fanout, "soa")
    assert ei.value.code == rt.RT_EINVAL


def test_build_rejects_bad_layout():
    import paper_2309_16913_amd as rt
    lib = rt._L
    h = C.c_void_p()
    r = np.zeros((4, 4), np.float32)
    rc = lib.rt_build_str(r.ctypes.data_as(C.POINTER(C.c_float)), 4, 16, 7, C.byref(h))
    assert rc == rt.RT_EINVAL and not h.value
    assert "layout" in lib.rt_last_error().decode()


def test_null_arguments_rejected():
    import paper_2309_16913_amd as rt
    lib = rt._L
    assert lib.rt_build_str(None, 5, 16, 1, None) == rt.RT_EINVAL
    h = C.c_void_p()
    assert lib.rt_build_str(None, 5, 16, 1, C.byref(h)) == rt.RT_EINVAL
    p = C.POINTER(rt._Ids)()
    assert lib.rt_range_select(None, None, 0, C.byref(p)) == rt.RT_EINVAL
    q = C.POINTER(rt._Pairs)()
    assert lib.rt_spatial_join(None, None, C.byref(q)) == rt.RT_EINVAL
    assert lib.rt_spatial_join_ex(None, None, rt.JOIN_O3 | rt.JOIN_O5, C.byref(q), None) == rt.RT_EINVAL
    lib.rt_free(None)   # no-op
    assert lib.rt_tree_stats(None, None) == rt.RT_EINVAL
    assert lib.rt_select_workspace_bytes(1000, 0) > 1000 * 4
    # the replay workspace: the plain layout plus room for 256-record chunks
    # (cap/16 + 16 nq records and more), growing with both arguments
    for nq, cap in [(1, 0), (1000, 0), (1000, 10**6), (10**6, 1_416_539_337)]:
        plain = lib.rt_select_workspace_bytes(nq, cap)
        full = lib.rt_select_replay_workspace_bytes(nq, cap)
        assert full - plain >= 16 * (cap // 16 + 16 * nq), (nq, cap)
    assert lib.rt_select_replay_workspace_bytes(1000, 2 * 10**6) > lib.rt_select_replay_workspace_bytes(1000, 10**6)
    assert lib.rt_select_replay_workspace_bytes(2000, 10**6) > lib.rt_select_replay_workspace_bytes(1000, 10**6)
    # the knobs reject a NULL tree
    assert lib.rt_tree_set_replay(None, 1) == rt.RT_EINVAL
    assert lib.rt_tree_set_bulk_copy(None, 0) == rt.RT_EINVAL
    c, o = C.c_uint32(0), C.c_uint32(0)
    assert lib.rt_select_replay_info(None, C.byref(c), C.byref(o)) == rt.RT_EINVAL
    assert lib.rt_batch_set_replay(None, 1) == rt.RT_EINVAL
    assert lib.rt_batch_replay_info(None, C.byref(c), C.byref(o)) == rt.RT_EINVAL


def test_stack_bound_formula():
    # the kernels size their LDS stacks by (h-1)(F-1)+1 (depth-first walk
    # popping one node and pushing its qualifying children); check the bound
    # against the worst case of a complete F-ary tree on the CPU
    for F in (2, 3, 16, 32, 64):
        for h in range(1, 6):
            # DFS on a complete tree where every entry qualifies
            stack = [(h - 1, 0)]
            peak = 1
            while stack:
                lvl, _ = stack.pop()
                if lvl > 0:
                    stack.extend((lvl - 1, k) for k in range(F))
                    peak = max(peak, len(stack))
                if F ** h > 20000:
                    break
            if F ** h <= 20000:
                assert peak == (1 if h == 1 else (h - 1) * (F - 1) + 1), (F, h, peak)
