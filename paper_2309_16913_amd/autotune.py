"""Autotuner for range select: picks the fanout, the node layout and the work
mapping for a dataset and its query mix by timing the device select on the
GPU, and remembers the choice in a JSON cache.

Candidates (all give identical results; only speed differs):
  fanout   16, 32, 64                     (entries per node, one lane each)
  layout   "aos" (D0), "soa" (D1), optionally "d2"
  mapping  split kmin 0 (one lane group per query) or k > 0 (windows that
           reach >= k parents-of-leaves run as one work item per subtree)

Cache key: (log2 of the object count, a caller-given distribution tag, the
decade of the median window selectivity measured against the data's MBR,
the candidate set).  A later tune() with the same key returns the cached
choice without timing anything.
"""

from __future__ import annotations

import json
import math
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(_HERE, "autotune_cache.json")


def selectivity_decade(rects: np.ndarray, queries: np.ndarray) -> int:
    if rects.shape[0] == 0 or queries.shape[0] == 0:
        return 0
    lo = rects[:, :2].min(0).astype(np.float64)
    hi = rects[:, 2:].max(0).astype(np.float64)
    area = float(np.prod(np.maximum(hi - lo, 1e-30)))
    q = queries.astype(np.float64)
    wa = np.clip((q[:, 2] - q[:, 0]) * (q[:, 3] - q[:, 1]), 1e-30, None) / area
    return int(math.floor(math.log10(float(np.median(wa)))))


class Autotuner:
    def __init__(self, cache_path: str | None = DEFAULT_CACHE, fanouts=(16, 32, 64), layouts=("aos", "soa"),
                 kmins=(0, 16), sample: int = 16384, reps: int = 3, replay: bool = True):
        import paper_2309_16913_amd as rt
        import torch
        self.rt, self.torch = rt, torch
        self.cache_path = cache_path
        self.fanouts, self.layouts, self.kmins = tuple(fanouts), tuple(layouts), tuple(kmins)
        self.sample, self.reps, self.replay = sample, reps, replay
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def key(self, n: int, tag: str, rects, queries) -> str:
        cand = (f"F{'-'.join(map(str, self.fanouts))}_L{'-'.join(self.layouts)}_K{'-'.join(map(str, self.kmins))}"
                + ("_R" if self.replay else ""))
        return f"n2^{int(math.log2(max(n, 1)))}_{tag}_sel1e{selectivity_decade(rects, queries)}_{cand}"

    def _time_select(self, tree, dq, nq):
        """Median wall time of a complete device select (count, scan, fill,
        sort) on resident queries."""
        rt, torch = self.rt, self.torch
        s = torch.cuda.current_stream()
        counts = torch.empty(max(nq, 1), dtype=torch.int32, device="cuda")
        wb0 = rt.select_workspace_bytes(nq, 0)
        w0 = torch.empty(wb0, dtype=torch.uint8, device="cuda")
        rt.range_count_device(tree, dq.data_ptr(), nq, counts.data_ptr(), w0.data_ptr(), wb0, s.cuda_stream)
        torch.cuda.synchronize()
        cap = int(counts[:nq].to(torch.int64).sum().item())
        off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
        # with room for the count pass's records, as a one-call select would
        # normally be given
        wb = rt.select_replay_workspace_bytes(nq, cap) if self.replay else rt.select_workspace_bytes(nq, cap)
        w = torch.empty(wb, dtype=torch.uint8, device="cuda")
        st = torch.zeros(2, dtype=torch.int64, device="cuda")
        times = []
        for r in range(self.reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rt.range_select_device(tree, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), cap, w.data_ptr(), wb,
                                   st.data_ptr(), s.cuda_stream)
            torch.cuda.synchronize()
            if r:
                times.append(time.perf_counter() - t0)
        assert int(st[1].item()) == 0
        return float(np.median(times))

    def tune(self, rects, queries, tag: str = "") -> dict:
        """Return {"fanout", "layout", "kmin", "timings_ms", "cached"}."""
        rects = np.ascontiguousarray(rects, np.float32).reshape(-1, 4)
        queries = np.ascontiguousarray(queries, np.float32).reshape(-1, 4)
        k = self.key(rects.shape[0], tag, rects, queries)
        if k in self.cache:
            out = dict(self.cache[k])
            out["cached"] = True
            return out
        sample = queries[: self.sample]
        dq = self.torch.from_numpy(sample).cuda()
        timings = {}
        for F in self.fanouts:
            for lay in self.layouts:
                t = self.rt.build_str(rects, F, lay)
                for km in self.kmins:
                    t.set_split(km)
                    timings[f"{F}/{lay}/{km}"] = self._time_select(t, dq, sample.shape[0]) * 1e3
                t.free()
        best = min(timings, key=timings.get)
        F, lay, km = best.split("/")
        out = {"fanout": int(F), "layout": lay, "kmin": int(km), "timings_ms": timings}
        self.cache[k] = out
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)
        out = dict(out)
        out["cached"] = False
        return out

    def build(self, rects, queries, tag: str = ""):
        """Tune (or look up) and build the tree with the chosen configuration."""
        c = self.tune(rects, queries, tag)
        t = self.rt.build_str(rects, c["fanout"], c["layout"])
        t.set_split(c["kmin"])
        return t, c


class BatchTuner:
    """Per-size-class choice of fanout and layout for a batch of independent
    trees, timed in batch context: the instances are grouped by the binary
    order of magnitude of their object count, every candidate configuration
    is built for one class's trees and that class's batch (persistent
    kernels replayed from its graph) is timed; each class keeps its fastest
    configuration.  The persistent batch kernel serves trees of different
    fanout and layout in one launch, so the classes' choices combine.

    instances: objects with .rects and .queries (numpy, n x 4 float32)."""

    def __init__(self, fanouts=(16, 32, 64), layouts=("aos", "soa", "d2"), reps: int = 2):
        import paper_2309_16913_amd as rt
        import torch
        self.rt, self.torch = rt, torch
        self.fanouts, self.layouts, self.reps = tuple(fanouts), tuple(layouts), reps

    @staticmethod
    def size_class(n: int) -> int:
        return int(math.log2(max(n, 1)))

    def _time_batch(self, trees, queries) -> float:
        rt, torch = self.rt, self.torch
        b = rt.Batch(trees, queries)
        b.run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(self.reps):
            t0 = time.perf_counter()
            b.run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        _, flags = b.status()
        b.free()
        assert flags == 0
        return float(np.median(ts))

    def tune(self, instances) -> dict:
        """{size class: {"fanout", "layout", "timings_ms"}}."""
        classes = {}
        for k, x in enumerate(instances):
            classes.setdefault(self.size_class(x.rects.shape[0]), []).append(k)
        out = {}
        for c, members in sorted(classes.items()):
            timings = {}
            for F in self.fanouts:
                for lay in self.layouts:
                    trees = [self.rt.build_str(instances[k].rects, F, lay) for k in members]
                    timings[f"{F}/{lay}"] = self._time_batch(trees, [instances[k].queries for k in members]) * 1e3
                    for t in trees:
                        t.free()
            best = min(timings, key=timings.get)
            F, lay = best.split("/")
            out[c] = {"fanout": int(F), "layout": lay, "trees": len(members), "timings_ms": timings}
        return out

    def build(self, instances, choice: dict):
        """Trees with each instance's class choice."""
        trees = []
        for x in instances:
            ch = choice[self.size_class(x.rects.shape[0])]
            trees.append(self.rt.build_str(x.rects, ch["fanout"], ch["layout"]))
        return trees
