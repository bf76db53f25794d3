"""Python binding of the MI355X R-tree range-select / spatial-join library.

Argument marshalling only: every step of a select or join runs in the HIP
kernels of ``librt_mi355x.so`` behind the C ABI declared in ``include/rt.h``.
There is no CPU fallback; importing this package without the built library
raises immediately.

Host-array calls (numpy in, numpy out):
    build_str(rects, fanout, layout)  -> Tree
    range_select(tree, queries)       -> (offsets uint64[nq+1], ids uint32[...])
    spatial_join(tree_a, tree_b)      -> pairs uint32[n, 2]
Device-pointer calls (for resident data, e.g. torch tensors' data_ptr()):
    range_select_device(...), range_count_device(...)
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt_mi355x.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE = 0, -1, -2, -3
BUILD_SORT_LX = 0x100
JOIN_O3, JOIN_O4, JOIN_O5, JOIN_TILE, JOIN_LB, JOIN_DEFAULT = 1, 2, 4, 8, 16, -1
LAYOUT_AOS, LAYOUT_SOA, LAYOUT_AUTO, LAYOUT_D2 = 0, 1, 2, 3
_LAYOUTS = {"aos": LAYOUT_AOS, "soa": LAYOUT_SOA, "auto": LAYOUT_AUTO, "d2": LAYOUT_D2,
            LAYOUT_AOS: LAYOUT_AOS, LAYOUT_SOA: LAYOUT_SOA, LAYOUT_AUTO: LAYOUT_AUTO, LAYOUT_D2: LAYOUT_D2}


class RTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rt error {code}: {msg}")
        self.code = code


try:  # load torch's HIP runtime first so the process holds a single copy of it
    import torch  # noqa: F401
except Exception:  # pragma: no cover - the library itself does not need torch
    pass

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(the library has no CPU fallback)")

_L = C.CDLL(LIB_PATH)


class TreeInfo(C.Structure):
    _fields_ = [("n_objects", C.c_uint64), ("n_entries", C.c_uint64), ("device_bytes", C.c_uint64),
                ("n_nodes", C.c_uint32), ("height", C.c_uint32), ("fanout", C.c_uint32),
                ("layout", C.c_uint32), ("node_bytes", C.c_uint32), ("first_leaf", C.c_uint32),
                ("device", C.c_int32), ("flags", C.c_uint32)]


class _Ids(C.Structure):
    _fields_ = [("nq", C.c_uint64), ("offsets", C.POINTER(C.c_uint64)), ("ids", C.POINTER(C.c_uint32))]


class _Pairs(C.Structure):
    _fields_ = [("n", C.c_uint64), ("pairs", C.POINTER(C.c_uint32))]


_vp, _u64, _u32, _fp = C.c_void_p, C.c_uint64, C.c_uint32, C.POINTER(C.c_float)
_sig = {
    "rt_build_str": ([_fp, _u64, _u32, _u32, C.POINTER(_vp)], C.c_int),
    "rt_build_str_device": ([_vp, _u64, _u32, _u32, _vp, C.POINTER(_vp)], C.c_int),
    "rt_range_select": ([_vp, _fp, _u64, C.POINTER(C.POINTER(_Ids))], C.c_int),
    "rt_spatial_join": ([_vp, _vp, C.POINTER(C.POINTER(_Pairs))], C.c_int),
    "rt_spatial_join_ex": ([_vp, _vp, C.c_int32, C.POINTER(C.POINTER(_Pairs)), C.POINTER(_u64)], C.c_int),
    "rt_spatial_join_device": ([_vp, _vp, C.c_int32, _vp, _u64, C.POINTER(_u64), _vp], C.c_int),
    "rt_join_visit_stats": ([_vp, _vp, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64)], C.c_int),
    "rt_free": ([_vp], None),
    "rt_select_workspace_bytes": ([_u64, _u64], _u64),
    "rt_select_replay_workspace_bytes": ([_u64, _u64], _u64),
    "rt_range_select_device": ([_vp, _vp, _u64, _vp, _vp, _u64, _vp, _u64, _vp, _vp], C.c_int),
    "rt_range_select_device_timed": ([_vp, _vp, _u64, _vp, _vp, _u64, _vp, _u64, _vp, _vp, _vp], C.c_int),
    "rt_range_count_device": ([_vp, _vp, _u64, _vp, _vp, _u64, _vp], C.c_int),
    "rt_range_select_device_count": ([_vp, _vp, _u64, _vp, _vp, _u64, _vp], C.c_int),
    "rt_range_select_device_fill": ([_vp, _vp, _u64, _vp, _vp, _u64, _vp, _u64, _vp, _vp], C.c_int),
    "rt_range_select_async": ([_vp, _vp, _u64, _vp, _vp, _u64, _vp, _vp], C.c_int),
    "rt_range_select_device_noalloc": ([_vp, _vp, _u64, _vp, _vp, _u64, _vp, _vp], C.c_int),
    "rt_range_select_batch": ([C.POINTER(_vp), _u32, C.POINTER(_fp), C.POINTER(_u64),
                               C.POINTER(C.POINTER(_Ids))], C.c_int),
    "rt_batch_create": ([C.POINTER(_vp), _u32, C.POINTER(_fp), C.POINTER(_u64), _u64,
                         C.POINTER(_vp)], C.c_int),
    "rt_batch_run": ([_vp, _vp], C.c_int),
    "rt_batch_run_plain": ([_vp, _vp], C.c_int),
    "rt_batch_status": ([_vp, C.POINTER(_u64), C.POINTER(_u64)], C.c_int),
    "rt_batch_set_replay": ([_vp, _u32], C.c_int),
    "rt_batch_replay_info": ([_vp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)], C.c_int),
    "rt_batch_result": ([_vp, _u32, C.POINTER(C.POINTER(_Ids))], C.c_int),
    "rt_tree_stats": ([_vp, C.POINTER(TreeInfo)], C.c_int),
    "rt_tree_set_split": ([_vp, _u32], C.c_int),
    "rt_tree_set_lookahead": ([_vp, _u32], C.c_int),
    "rt_tree_set_bulk_copy": ([_vp, _u32], C.c_int),
    "rt_tree_set_replay": ([_vp, _u32], C.c_int),
    "rt_select_replay_info": ([_vp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)], C.c_int),
    "rt_tree_export": ([_vp] + [_vp] * 8, C.c_int),
    "rt_select_visit_stats": ([_vp, _fp, _u64, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64)], C.c_int),
    "rt_last_error": ([], C.c_char_p),
    "rt_version": ([], C.c_char_p),
}
for _name, (_a, _r) in _sig.items():
    _f = getattr(_L, _name)
    _f.argtypes = _a
    _f.restype = _r


def exported_symbols():
    return list(_sig)


def _check(rc):
    if rc != RT_OK:
        raise RTError(rc, _L.rt_last_error().decode())


def _rects(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a.reshape(-1, 4)


def _f(a):
    return a.ctypes.data_as(_fp)


def version() -> str:
    return _L.rt_version().decode()


class Tree:
    """A device-resident R-tree (immutable)."""

    def __init__(self, handle):
        self.h = _vp(handle)

    def info(self) -> TreeInfo:
        i = TreeInfo()
        _check(_L.rt_tree_stats(self.h, C.byref(i)))
        return i

    def export(self) -> dict:
        i = self.info()
        nn, ne = i.n_nodes, i.n_entries
        out = dict(level=np.zeros(nn, np.uint32), count=np.zeros(nn, np.uint32), first=np.zeros(nn, np.uint64),
                   lx=np.zeros(ne, np.float32), ly=np.zeros(ne, np.float32), hx=np.zeros(ne, np.float32),
                   hy=np.zeros(ne, np.float32), ptr=np.zeros(ne, np.uint32))
        args = [out[k].ctypes.data_as(_vp) for k in ("level", "count", "first", "lx", "ly", "hx", "hy", "ptr")]
        _check(_L.rt_tree_export(self.h, *args))
        out.update(root=0, height=i.height, fanout=i.fanout, n_objects=i.n_objects)
        return out

    def set_split(self, kmin: int):
        """Work mapping knob (never changes results): split queries that reach
        at least kmin parents-of-leaves nodes; 0 = one lane group per query."""
        _check(_L.rt_tree_set_split(self.h, int(kmin)))

    def set_lookahead(self, on: bool):
        """Load the next node ahead after a leaf in later selects (never
        changes results)."""
        _check(_L.rt_tree_set_lookahead(self.h, 1 if on else 0))

    def set_bulk_copy(self, mode: str):
        """Where the fill pass copies long contained runs (never changes
        results): "auto" (a streaming kernel after the pass on trees of at
        least 2^25 objects), "on" (always) or "off" (in the pass)."""
        _check(_L.rt_tree_set_bulk_copy(self.h, {"auto": 0, "on": 1, "off": 2}[mode]))

    def set_replay(self, on: bool):
        """Let one-call selects replay the count pass's records in the fill
        (given a workspace of select_replay_workspace_bytes) instead of
        walking the tree again (never changes results)."""
        _check(_L.rt_tree_set_replay(self.h, 1 if on else 0))

    def free(self):
        if self.h is not None and self.h.value:
            _L.rt_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _layout_arg(layout, sort_lx: bool) -> int:
    return _LAYOUTS[layout] | (BUILD_SORT_LX if sort_lx else 0)


def build_str(rects, fanout: int = 32, layout="soa", sort_lx: bool = False) -> Tree:
    """STR tree over host rectangles (built on the device).  sort_lx: entries
    of every node in ascending low x (needed by the join pruning)."""
    r = _rects(rects)
    h = _vp()
    _check(_L.rt_build_str(_f(r), r.shape[0], int(fanout), _layout_arg(layout, sort_lx), C.byref(h)))
    return Tree(h.value)


def build_str_device(d_rects: int, n: int, fanout: int = 32, layout="soa", stream: int = 0,
                     sort_lx: bool = False) -> Tree:
    h = _vp()
    _check(_L.rt_build_str_device(_vp(d_rects), int(n), int(fanout), _layout_arg(layout, sort_lx), _vp(stream),
                                  C.byref(h)))
    return Tree(h.value)


def _take_ids(p):
    r = p.contents
    nq = int(r.nq)
    off = np.ctypeslib.as_array(r.offsets, shape=(nq + 1,)).copy()
    tot = int(off[-1])
    ids = np.ctypeslib.as_array(r.ids, shape=(tot,)).copy() if tot else np.zeros(0, np.uint32)
    _L.rt_free(C.cast(p, _vp))
    return off, ids


def range_select(tree: Tree, queries):
    q = _rects(queries)
    p = C.POINTER(_Ids)()
    _check(_L.rt_range_select(tree.h, _f(q), q.shape[0], C.byref(p)))
    return _take_ids(p)


def spatial_join(a: Tree, b: Tree, flags: int | None = None, with_tests: bool = False):
    """All intersecting (a, b) as an (n, 2) uint32 array in lexicographic
    order.  flags: JOIN_O3 | JOIN_O4 | JOIN_O5, JOIN_O3 | JOIN_O5 | JOIN_LB,
    JOIN_TILE, 0, or None for the library default.  with_tests: also return
    the number of child-pair predicates evaluated."""
    p = C.POINTER(_Pairs)()
    tests = _u64(0)
    if flags is None and not with_tests:
        _check(_L.rt_spatial_join(a.h, b.h, C.byref(p)))
    else:
        _check(_L.rt_spatial_join_ex(a.h, b.h, JOIN_DEFAULT if flags is None else int(flags), C.byref(p),
                                     C.byref(tests) if with_tests else None))
    n = int(p.contents.n)
    out = np.ctypeslib.as_array(p.contents.pairs, shape=(2 * n,)).copy().reshape(n, 2) if n else \
        np.zeros((0, 2), np.uint32)
    _L.rt_free(C.cast(p, _vp))
    return (out, int(tests.value)) if with_tests else out


def spatial_join_device(a: Tree, b: Tree, d_pairs: int, capacity: int, flags: int | None = None,
                        stream: int = 0) -> int:
    """Join into caller device memory (2 * capacity uint32 at d_pairs).
    Returns the number of pairs; if it exceeds capacity nothing was written
    and the call can be repeated with a larger buffer."""
    n = _u64(0)
    rc = _L.rt_spatial_join_device(a.h, b.h, JOIN_DEFAULT if flags is None else int(flags), _vp(d_pairs),
                                   int(capacity), C.byref(n), _vp(stream))
    if rc == RT_ENOMEM and n.value > capacity:
        return int(n.value)
    _check(rc)
    return int(n.value)


def join_visit_stats(a: Tree, b: Tree):
    """(node pairs visited, entry predicates, real entries loaded) of the
    plain synchronized-traversal join of a and b."""
    n, p, e = _u64(), _u64(), _u64()
    _check(_L.rt_join_visit_stats(a.h, b.h, C.byref(n), C.byref(p), C.byref(e)))
    return int(n.value), int(p.value), int(e.value)


def visit_stats(tree: Tree, queries):
    """(visited nodes, visited entries, ids taken wholesale from subtrees that
    lie inside their window) summed over the queries."""
    q = _rects(queries)
    vn, ve, vc = _u64(), _u64(), _u64()
    _check(_L.rt_select_visit_stats(tree.h, _f(q), q.shape[0], C.byref(vn), C.byref(ve), C.byref(vc)))
    return int(vn.value), int(ve.value), int(vc.value)


def select_workspace_bytes(nq: int, ids_capacity: int) -> int:
    return int(_L.rt_select_workspace_bytes(int(nq), int(ids_capacity)))


def select_replay_info(d_work: int):
    """(record chunks taken, overflowed) of the last one-call select on the
    workspace d_work (after its stream has been synchronized)."""
    c, o = C.c_uint32(0), C.c_uint32(0)
    _check(_L.rt_select_replay_info(_vp(d_work), C.byref(c), C.byref(o)))
    return int(c.value), bool(o.value)


def select_replay_workspace_bytes(nq: int, ids_capacity: int) -> int:
    """Workspace with room for the count pass's records (the fill replays
    them instead of walking the tree again)."""
    return int(_L.rt_select_replay_workspace_bytes(int(nq), int(ids_capacity)))


def range_select_device(tree: Tree, d_queries: int, nq: int, d_offsets: int, d_ids: int, ids_capacity: int,
                        d_work: int, work_bytes: int, d_status: int, stream: int = 0):
    _check(_L.rt_range_select_device(tree.h, _vp(d_queries), int(nq), _vp(d_offsets), _vp(d_ids),
                                     int(ids_capacity), _vp(d_work), int(work_bytes), _vp(d_status),
                                     _vp(stream)))


def range_select_device_timed(tree: Tree, d_queries: int, nq: int, d_offsets: int, d_ids: int,
                              ids_capacity: int, d_work: int, work_bytes: int, d_status: int, stream: int,
                              events):
    """events: sequence of 5 hipEvent_t handles (ints) or None."""
    ev = (_vp * 5)(*[_vp(x) for x in events]) if events is not None else None
    _check(_L.rt_range_select_device_timed(tree.h, _vp(d_queries), int(nq), _vp(d_offsets), _vp(d_ids),
                                           int(ids_capacity), _vp(d_work), int(work_bytes), _vp(d_status),
                                           _vp(stream), ev))


def range_select_device_count(tree: Tree, d_queries: int, nq: int, d_offsets: int, d_work: int, work_bytes: int,
                              stream: int = 0):
    """Count stage of a device select: offsets (with the total at [nq]) and
    the plan in the workspace; nothing waits."""
    _check(_L.rt_range_select_device_count(tree.h, _vp(d_queries), int(nq), _vp(d_offsets), _vp(d_work),
                                           int(work_bytes), _vp(stream)))


def range_select_device_fill(tree: Tree, d_queries: int, nq: int, d_offsets: int, d_ids: int, ids_capacity: int,
                             d_work: int, work_bytes: int, d_status: int, stream: int = 0):
    """Fill stage after range_select_device_count on the same workspace."""
    _check(_L.rt_range_select_device_fill(tree.h, _vp(d_queries), int(nq), _vp(d_offsets), _vp(d_ids),
                                          int(ids_capacity), _vp(d_work), int(work_bytes), _vp(d_status),
                                          _vp(stream)))


NOALLOC_SCRATCH_BYTES = 32 << 20


def range_select_device_noalloc(tree: Tree, d_queries: int, nq: int, d_offsets: int, d_ids: int,
                                ids_capacity: int, d_status: int, stream: int = 0):
    """range_select_device with the library's fixed device scratch as its
    workspace (allocates nothing; calls overlapping on one device race)."""
    _check(_L.rt_range_select_device_noalloc(tree.h, _vp(d_queries), int(nq), _vp(d_offsets), _vp(d_ids),
                                             int(ids_capacity), _vp(d_status), _vp(stream)))


def range_select_async(tree: Tree, d_queries: int, nq: int, d_offsets: int, d_ids: int, ids_capacity: int,
                       d_total: int, stream: int = 0) -> bool:
    """Select into caller device buffers (library-held workspace).  Returns
    False (RT_ENOMEM, ids untouched) when the result exceeds ids_capacity;
    the size is then in d_total.  True: the fill runs on `stream`."""
    rc = _L.rt_range_select_async(tree.h, _vp(d_queries), int(nq), _vp(d_offsets), _vp(d_ids), int(ids_capacity),
                                  _vp(d_total), _vp(stream))
    if rc == RT_ENOMEM:
        return False
    _check(rc)
    return True


def range_count_device(tree: Tree, d_queries: int, nq: int, d_counts: int, d_work: int, work_bytes: int,
                       stream: int = 0):
    _check(_L.rt_range_count_device(tree.h, _vp(d_queries), int(nq), _vp(d_counts), _vp(d_work),
                                    int(work_bytes), _vp(stream)))


class Batch:
    """A prepared device-resident batch of (tree, queries) instances."""

    def __init__(self, trees, queries, ids_capacity: int = 0):
        self.trees = list(trees)
        self.q = [_rects(x) for x in queries]
        n = len(self.trees)
        th = (_vp * n)(*[t.h for t in self.trees])
        qp = (_fp * n)(*[_f(x) for x in self.q])
        nq = (_u64 * n)(*[x.shape[0] for x in self.q])
        h = _vp()
        _check(_L.rt_batch_create(th, n, qp, nq, int(ids_capacity), C.byref(h)))
        self.h = h

    def run(self, stream: int = 0):
        _check(_L.rt_batch_run(self.h, _vp(stream)))

    def run_plain(self, stream: int = 0):
        _check(_L.rt_batch_run_plain(self.h, _vp(stream)))

    def set_replay(self, on: bool):
        """Recapture the graph with the replayed (True) or walking fill."""
        _check(_L.rt_batch_set_replay(self.h, 1 if on else 0))

    def replay_info(self):
        """(record chunks taken, overflowed) of the last graph run."""
        c, o = C.c_uint32(0), C.c_uint32(0)
        _check(_L.rt_batch_replay_info(self.h, C.byref(c), C.byref(o)))
        return int(c.value), bool(o.value)

    def status(self):
        t, f = _u64(), _u64()
        _check(_L.rt_batch_status(self.h, C.byref(t), C.byref(f)))
        return int(t.value), int(f.value)

    def result(self, i: int):
        p = C.POINTER(_Ids)()
        _check(_L.rt_batch_result(self.h, int(i), C.byref(p)))
        return _take_ids(p)

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _L.rt_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def range_select_batch(trees, queries):
    n = len(trees)
    qs = [_rects(x) for x in queries]
    th = (_vp * n)(*[t.h for t in trees])
    qp = (_fp * n)(*[_f(x) for x in qs])
    nq = (_u64 * n)(*[x.shape[0] for x in qs])
    outs = (C.POINTER(_Ids) * n)()
    _check(_L.rt_range_select_batch(th, n, qp, nq, outs))
    return [_take_ids(outs[i]) for i in range(n)]
