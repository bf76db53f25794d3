"""Python access to the scalar CPU oracle (``rtree_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  The GPU library and its Python binding never
import this package.

The oracle computes range select and spatial join from their plain
definitions: ``select(q) = ascending {i : overlap(rect[i], q)}`` and
``join(A, B) = lexicographic {(a, b) : overlap(A[a], B[b])}`` with the closed
four-comparison overlap test of the paper's select (section 3) and join
(section 4.1, step 3) predicates.  See ``rtree_oracle.c`` for the steps.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rtree_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()


def build(out_path: str = LIB_PATH, mutant: int = 0) -> str:
    """Compile the oracle with gcc (plain C99, -O2, no vector intrinsics)."""
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-pthread", "-D_GNU_SOURCE",
           f"-DORA_MUTANT={int(mutant)}", _SRC, "-o", out_path + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out_path + ".tmp", out_path)
    return out_path


class _Tree(C.Structure):
    _fields_ = [
        ("fanout", C.c_uint32), ("height", C.c_uint32), ("n_nodes", C.c_uint32),
        ("root", C.c_uint32), ("n_objects", C.c_uint64), ("n_entries", C.c_uint64),
        ("level", C.POINTER(C.c_uint32)), ("count", C.POINTER(C.c_uint32)),
        ("first", C.POINTER(C.c_uint64)),
        ("lx", C.POINTER(C.c_float)), ("ly", C.POINTER(C.c_float)),
        ("hx", C.POINTER(C.c_float)), ("hy", C.POINTER(C.c_float)),
        ("ptr", C.POINTER(C.c_uint32)),
    ]


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _u64ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _rects(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 4:
        a = a.reshape(-1, 4)
    return a


class Oracle:
    def __init__(self, path: str | None = None):
        path = path or LIB_PATH
        if path == LIB_PATH:
            with _lock:
                if (not os.path.exists(path)
                        or os.path.getmtime(path) < os.path.getmtime(_SRC)):
                    build(path)
        L = C.CDLL(path)
        T = C.POINTER(_Tree)
        L.ora_build_str.argtypes = [C.POINTER(C.c_float), C.c_uint64, C.c_uint32, T]
        L.ora_free_tree.argtypes = [T]
        L.ora_select.argtypes = [T, C.POINTER(C.c_float), C.c_uint64, C.POINTER(C.c_uint64),
                                 C.POINTER(C.POINTER(C.c_uint32)), C.POINTER(C.c_uint64)]
        L.ora_join.argtypes = [T, T, C.POINTER(C.POINTER(C.c_uint32)), C.POINTER(C.c_uint64)]
        L.ora_select_mt.argtypes = [T, C.POINTER(C.c_float), C.c_uint64, C.c_int, C.POINTER(C.c_uint64),
                                    C.POINTER(C.POINTER(C.c_uint32)), C.POINTER(C.c_uint64)]
        L.ora_join_mt.argtypes = [T, T, C.c_int, C.POINTER(C.POINTER(C.c_uint32)), C.POINTER(C.c_uint64)]
        L.ora_brute_select.argtypes = [C.POINTER(C.c_float), C.c_uint64, C.POINTER(C.c_float),
                                       C.c_uint64, C.POINTER(C.c_uint64),
                                       C.POINTER(C.POINTER(C.c_uint32)), C.POINTER(C.c_uint64)]
        L.ora_brute_join.argtypes = [C.POINTER(C.c_float), C.c_uint64, C.POINTER(C.c_float),
                                     C.c_uint64, C.POINTER(C.POINTER(C.c_uint32)),
                                     C.POINTER(C.c_uint64)]
        L.ora_join_opt.argtypes = [T, T, C.c_int, C.POINTER(C.POINTER(C.c_uint32)), C.POINTER(C.c_uint64),
                                   C.POINTER(C.c_uint64)]
        L.ora_sort_entries_lx.argtypes = [T]
        L.ora_m2m_update.argtypes = [C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32),
                                     C.POINTER(C.c_uint32)]
        L.ora_m2m_update.restype = None
        L.ora_m2m_flip.argtypes = [C.c_uint32, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_uint32,
                                   C.POINTER(C.c_uint32)]
        L.ora_m2m_flip.restype = None
        L.ora_check_tree.argtypes = [T, C.POINTER(C.c_float), C.c_char_p, C.c_int]
        L.ora_free_buf.argtypes = [C.c_void_p]
        self.L = L

    # -- tree -------------------------------------------------------------
    def build_str(self, rects, fanout: int) -> "OraTree":
        r = _rects(rects)
        t = _Tree()
        rc = self.L.ora_build_str(_fptr(r), r.shape[0], fanout, C.byref(t))
        if rc != 0:
            raise ValueError(f"oracle STR build rejected input (rc={rc})")
        return OraTree(self, t)

    # -- select -----------------------------------------------------------
    def _take_ids(self, pids, total):
        n = int(total.value)
        ids = np.ctypeslib.as_array(pids, shape=(max(n, 1),))[:n].copy() if n else \
            np.zeros(0, np.uint32)
        self.L.ora_free_buf(C.cast(pids, C.c_void_p))
        return ids

    def select(self, tree: "OraTree", queries):
        q = _rects(queries)
        off = np.zeros(q.shape[0] + 1, dtype=np.uint64)
        pids = C.POINTER(C.c_uint32)()
        total = C.c_uint64()
        rc = self.L.ora_select(C.byref(tree.t), _fptr(q), q.shape[0], _u64ptr(off),
                               C.byref(pids), C.byref(total))
        if rc:
            raise MemoryError("oracle select failed")
        return off, self._take_ids(pids, total)

    def select_mt(self, tree: "OraTree", queries, nthreads: int):
        """select() with the queries cut into nthreads contiguous parts, one
        host thread each (a timing baseline; same result as select())."""
        q = _rects(queries)
        off = np.zeros(q.shape[0] + 1, dtype=np.uint64)
        pids = C.POINTER(C.c_uint32)()
        total = C.c_uint64()
        rc = self.L.ora_select_mt(C.byref(tree.t), _fptr(q), q.shape[0], int(nthreads), _u64ptr(off),
                                  C.byref(pids), C.byref(total))
        if rc:
            raise MemoryError("oracle select failed")
        return off, self._take_ids(pids, total)

    def brute_select(self, rects, queries):
        r, q = _rects(rects), _rects(queries)
        off = np.zeros(q.shape[0] + 1, dtype=np.uint64)
        pids = C.POINTER(C.c_uint32)()
        total = C.c_uint64()
        rc = self.L.ora_brute_select(_fptr(r), r.shape[0], _fptr(q), q.shape[0], _u64ptr(off),
                                     C.byref(pids), C.byref(total))
        if rc:
            raise MemoryError("oracle brute select failed")
        return off, self._take_ids(pids, total)

    # -- join -------------------------------------------------------------
    def _take_pairs(self, pp, n):
        k = int(n.value)
        out = np.ctypeslib.as_array(pp, shape=(max(2 * k, 1),))[:2 * k].copy().reshape(k, 2) \
            if k else np.zeros((0, 2), np.uint32)
        self.L.ora_free_buf(C.cast(pp, C.c_void_p))
        return out

    def join(self, a: "OraTree", b: "OraTree") -> np.ndarray:
        pp = C.POINTER(C.c_uint32)()
        n = C.c_uint64()
        if self.L.ora_join(C.byref(a.t), C.byref(b.t), C.byref(pp), C.byref(n)):
            raise MemoryError("oracle join failed")
        return self._take_pairs(pp, n)

    def join_mt(self, a: "OraTree", b: "OraTree", nthreads: int) -> np.ndarray:
        """join() with the intersecting root-entry pairs dealt to nthreads host
        threads (a timing baseline; same result as join())."""
        pp = C.POINTER(C.c_uint32)()
        n = C.c_uint64()
        if self.L.ora_join_mt(C.byref(a.t), C.byref(b.t), int(nthreads), C.byref(pp), C.byref(n)):
            raise MemoryError("oracle join failed")
        return self._take_pairs(pp, n)

    def brute_join(self, A, B) -> np.ndarray:
        a, b = _rects(A), _rects(B)
        pp = C.POINTER(C.c_uint32)()
        n = C.c_uint64()
        if self.L.ora_brute_join(_fptr(a), a.shape[0], _fptr(b), b.shape[0], C.byref(pp), C.byref(n)):
            raise MemoryError("oracle brute join failed")
        return self._take_pairs(pp, n)

    # -- join over nodes sorted by low x (section 4 pruning) ---------------
    O3, O4, O5 = 1, 2, 4

    def sort_entries_lx(self, tree: "OraTree") -> None:
        """Reorder every node's entries by ascending low x (in place)."""
        if self.L.ora_sort_entries_lx(C.byref(tree.t)):
            raise ValueError("oracle could not sort the tree's nodes")

    def join_opt(self, a: "OraTree", b: "OraTree", flags: int):
        """(pairs, tests): the join with O3 / O4 / O5 pruning (flags 1 / 2 / 4)
        and the number of pair predicates it evaluated."""
        pp = C.POINTER(C.c_uint32)()
        n = C.c_uint64()
        tests = C.c_uint64()
        rc = self.L.ora_join_opt(C.byref(a.t), C.byref(b.t), int(flags), C.byref(pp), C.byref(n), C.byref(tests))
        if rc == -1:
            raise ValueError("pruned join needs nodes sorted by low x and fanout <= 64")
        if rc:
            raise MemoryError("oracle join failed")
        return self._take_pairs(pp, n), int(tests.value)

    def m2m_update(self, mask: int, step: int, n_pow: int, gidx, flip):
        """One many-to-many index update; returns the new (gidx, flip)."""
        g = np.ascontiguousarray(gidx, np.uint32).copy()
        f = np.ascontiguousarray(flip, np.uint32).copy()
        assert g.shape == f.shape and g.size <= 64
        u32p = C.POINTER(C.c_uint32)
        self.L.ora_m2m_update(g.size, int(mask), int(step), int(n_pow), g.ctypes.data_as(u32p),
                              f.ctypes.data_as(u32p))
        return g, f

    def m2m_flip(self, out_hx, in_lx):
        """Flip index of each outer high x (at most 64) against the sorted
        inner low x values."""
        o = np.ascontiguousarray(out_hx, np.float32)
        i = np.ascontiguousarray(in_lx, np.float32)
        assert o.size <= 64 and i.size <= 64
        f = np.zeros(o.size, np.uint32)
        self.L.ora_m2m_flip(o.size, _fptr(o), _fptr(i) if i.size else None, i.size,
                            f.ctypes.data_as(C.POINTER(C.c_uint32)))
        return f

    # -- invariants -------------------------------------------------------
    def check(self, tree: "OraTree", rects=None):
        buf = C.create_string_buffer(256)
        rp = None
        if rects is not None:
            rects = _rects(rects)
            rp = _fptr(rects)
        rc = self.L.ora_check_tree(C.byref(tree.t), rp, buf, 256)
        return rc, buf.value.decode()

    def tree_from_arrays(self, *, fanout, height, root, n_objects, level, count, first,
                         lx, ly, hx, hy, ptr) -> "OraTree":
        """Wrap a tree given as flat arrays (for instance one read back from the
        GPU library) so that the invariant checker can inspect it."""
        keep = dict(level=np.ascontiguousarray(level, np.uint32),
                    count=np.ascontiguousarray(count, np.uint32),
                    first=np.ascontiguousarray(first, np.uint64),
                    lx=np.ascontiguousarray(lx, np.float32), ly=np.ascontiguousarray(ly, np.float32),
                    hx=np.ascontiguousarray(hx, np.float32), hy=np.ascontiguousarray(hy, np.float32),
                    ptr=np.ascontiguousarray(ptr, np.uint32))
        t = _Tree()
        t.fanout, t.height, t.root = int(fanout), int(height), int(root)
        t.n_nodes = keep["level"].shape[0]
        t.n_objects = int(n_objects)
        t.n_entries = keep["lx"].shape[0]
        for k in ("level", "count", "ptr"):
            setattr(t, k, keep[k].ctypes.data_as(C.POINTER(C.c_uint32)))
        t.first = keep["first"].ctypes.data_as(C.POINTER(C.c_uint64))
        for k in ("lx", "ly", "hx", "hy"):
            setattr(t, k, keep[k].ctypes.data_as(C.POINTER(C.c_float)))
        return OraTree(self, t, owned=False, keep=keep)


class OraTree:
    def __init__(self, o: Oracle, t: _Tree, owned: bool = True, keep=None):
        self.o, self.t, self.owned, self.keep = o, t, owned, keep

    @property
    def height(self):
        return self.t.height

    @property
    def n_nodes(self):
        return self.t.n_nodes

    def arrays(self):
        """Copies of the node and entry arrays (for tests)."""
        t = self.t
        nn, ne = t.n_nodes, t.n_entries

        def grab(p, n, dt):
            return np.ctypeslib.as_array(p, shape=(max(n, 1),))[:n].astype(dt, copy=True)
        return dict(level=grab(t.level, nn, np.uint32), count=grab(t.count, nn, np.uint32),
                    first=grab(t.first, nn, np.uint64), lx=grab(t.lx, ne, np.float32),
                    ly=grab(t.ly, ne, np.float32), hx=grab(t.hx, ne, np.float32),
                    hy=grab(t.hy, ne, np.float32), ptr=grab(t.ptr, ne, np.uint32),
                    root=t.root, height=t.height, fanout=t.fanout, n_objects=t.n_objects)

    def __del__(self):
        if self.owned and self.t is not None and self.t.n_nodes:
            try:
                self.o.L.ora_free_tree(C.byref(self.t))
            except Exception:
                pass
            self.t = None


_default = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
