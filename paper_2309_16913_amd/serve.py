"""Continuous-batching server for range-select and join requests on resident
R-trees (one GPU).

Requests arrive over time (open loop: each has a scheduled arrival time).
The loop keeps up to `nslots` batches in flight, one per HIP stream.  A free
slot takes the waiting requests of one kind -- range windows packed
together into one select on the range tree, or join requests (probe sets of
rectangles, answered as an index nested loop: every probe rectangle is a
window on the join tree) packed together into one select on the join tree
-- and runs it in two stages:

1. the count stage of the device select (every window's exact result size,
   the CSR offsets);
2. once the batch's exact total is known, it is given a contiguous range of
   that many ids in the output pool (first fit; ranges of batches in flight
   never overlap), and the fill stage writes the ids there and copies them to
   the same range of a pinned host pool.

Admission is thereby bounded by output-buffer memory with exact sizes: a
batch waits after its count stage until its range is free, and no result is
ever truncated, dropped or recomputed because it did not fit.  Batches are
formed so that about `nslots` of them fit in the pool at once (sizes known
from earlier count stages, others estimated from the running mean of ids per
window); a batch larger than the whole pool (only possible while sizes are
unknown) is re-queued with its exact per-request sizes, and a single request
larger than the pool is an error.  Requests that arrive while batches run
wait for the next free slot, so work of several batches overlaps on the
device.

Latency of a request = time its result is in pinned host memory - its
scheduled arrival.  All GPU work goes through the library's device-pointer
entry points; torch supplies device memory, pinned host memory, streams and
events only.
"""

from __future__ import annotations

import gc
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# pure host policy (no GPU): which waiting requests form the next batch, and
# where a batch's output goes
# ---------------------------------------------------------------------------

@dataclass
class Pending:
    rid: int
    kind: str                    # "select" or "join"
    windows: np.ndarray          # (m, 4) float32
    t_arrival: float
    known_ids: int = -1          # exact result size once a count stage has reported it


@dataclass
class Batch:
    kind: str
    reqs: list
    windows: np.ndarray


class Admission:
    """Forms batches from the waiting queue, in arrival order.

    * a batch holds requests of one kind (range windows on the range tree,
      or join probe sets on the join tree), the kind of the oldest waiting
      request; requests of the other kind keep their place in the queue;
    * requests are packed up to `max_windows` windows and while the batch's
      expected size stays within `budget_ids` (a request's known size, else
      its windows times the running estimate of ids per window of its kind);
      the first request of a batch is always taken, whatever its size."""

    def __init__(self, max_windows: int, budget_ids: int, one_per_batch: bool = False):
        self.max_windows = max_windows
        self.budget_ids = budget_ids
        self.one_per_batch = one_per_batch   # the unbatched baseline: one request per launch
        self.queue: deque = deque()
        self.per_window = {"select": 0.0, "join": 0.0}   # running estimates, from count stages

    def push(self, p: Pending):
        self.queue.append(p)

    def push_front(self, ps):
        for p in reversed(ps):
            self.queue.appendleft(p)

    def __len__(self):
        return len(self.queue)

    @property
    def ids_per_window(self) -> float:
        return self.per_window["select"]

    def expected(self, p: Pending) -> float:
        return p.known_ids if p.known_ids >= 0 else self.per_window[p.kind] * p.windows.shape[0]

    def next_batch(self):
        if not self.queue:
            return None
        kind = self.queue[0].kind
        reqs, size, nwin = [], 0.0, 0
        skipped = []   # requests of the other kind passed over (they keep their place)
        q = self.queue
        while q:
            p = q[0]
            if p.kind != kind:
                skipped.append(q.popleft())
                continue
            if (nwin + p.windows.shape[0] > self.max_windows or (reqs and size + self.expected(p) > self.budget_ids)
                    or (self.one_per_batch and reqs)):
                break
            reqs.append(q.popleft())
            nwin += p.windows.shape[0]
            size += self.expected(p)
        for p in reversed(skipped):
            q.appendleft(p)
        return Batch(kind, reqs, np.concatenate([r.windows for r in reqs]))

    def observe(self, total: int, nwin: int, kind: str = "select"):
        """A count stage reported `total` ids for `nwin` windows of `kind`."""
        if nwin:
            m = total / nwin
            old = self.per_window[kind]
            self.per_window[kind] = m if old == 0.0 else 0.8 * old + 0.2 * m

    def sizes_known(self, batch: Batch, counts: np.ndarray):
        """Record every request's exact size from per-window counts."""
        at = 0
        for r in batch.reqs:
            m = r.windows.shape[0]
            r.known_ids = int(counts[at:at + m].sum())
            at += m

    def requeue(self, batch: Batch, counts: np.ndarray, pool_ids: int):
        """A batch too large for the whole pool: back to the front of the
        queue with exact sizes (the next batches are packed to fit)."""
        self.sizes_known(batch, counts)
        for r in batch.reqs:
            if r.known_ids > pool_ids:
                raise MemoryError(f"request {r.rid} needs {r.known_ids} ids, more than the whole pool ({pool_ids})")
        self.push_front(batch.reqs)


class IdPool:
    """First-fit placement of batch outputs in one buffer of `size` ids: a
    batch gets a contiguous range [start, start + n) and keeps it until its
    results have been delivered; live ranges never overlap."""

    def __init__(self, size: int):
        self.size = size
        self.live = []           # sorted (start, end) of ranges in use

    def alloc(self, n: int):
        if n == 0:
            return 0
        prev = 0
        for i, (s, e) in enumerate(self.live):
            if s - prev >= n:
                self.live.insert(i, (prev, prev + n))
                return prev
            prev = e
        if self.size - prev >= n:
            self.live.append((prev, prev + n))
            return prev
        return None

    def free(self, start: int, n: int):
        if n == 0:
            return
        self.live.remove((start, start + n))

    def in_use(self) -> int:
        return sum(e - s for s, e in self.live)


# ---------------------------------------------------------------------------
# GPU server
# ---------------------------------------------------------------------------

@dataclass
class Stats:
    lat_select: list = field(default_factory=list)
    lat_join: list = field(default_factory=list)
    batches: int = 0
    requeued_batches: int = 0     # batches larger than the whole pool (sizes then known)
    oversized_batches: int = 0    # batches over the per-batch budget (a single large request)
    memory_waits: int = 0         # batches that waited after their count stage for pool room
    windows: int = 0
    ids: int = 0
    gpu_count_ms: float = 0.0     # device time of the count stages
    gpu_fill_ms: float = 0.0      # device time of the fill stages (fill pass + sort)
    gpu_copy_ms: float = 0.0      # device time of the result copies to pinned memory

    def summary(self, wall: float, nreq: int) -> dict:
        def pct(v, q):
            return float(np.percentile(np.array(v) * 1e3, q)) if v else None
        return {
            "requests": nreq, "wall_s": wall, "throughput_req_per_s": nreq / wall if wall > 0 else None,
            "windows_per_s": self.windows / wall if wall > 0 else None,
            "select_p50_ms": pct(self.lat_select, 50), "select_p99_ms": pct(self.lat_select, 99),
            "join_p50_ms": pct(self.lat_join, 50), "join_p99_ms": pct(self.lat_join, 99),
            "batches": self.batches, "requeued_batches": self.requeued_batches,
            "oversized_batches": self.oversized_batches, "memory_waits": self.memory_waits, "ids": self.ids,
            "gpu_count_ms": self.gpu_count_ms, "gpu_fill_ms": self.gpu_fill_ms, "gpu_copy_ms": self.gpu_copy_ms,
        }


IDLE, COUNTING, WAITING, FILLING = 0, 1, 2, 3


class _Slot:
    def __init__(self, torch, rt, max_windows, work_bytes):
        self.stream = torch.cuda.Stream()
        self.dq = torch.empty((max_windows, 4), dtype=torch.float32, device="cuda")
        self.off = torch.empty(max_windows + 1, dtype=torch.int64, device="cuda")
        self.status = torch.zeros(2, dtype=torch.int64, device="cuda")
        self.hq = torch.empty((max_windows, 4), dtype=torch.float32).pin_memory()
        self.hoff = torch.empty(max_windows + 1, dtype=torch.int64).pin_memory()
        self.hstat = torch.empty(2, dtype=torch.int64).pin_memory()
        self.wb = work_bytes
        self.work = torch.empty(work_bytes, dtype=torch.uint8, device="cuda")
        self.stage = IDLE
        self.batch = None
        self.ev = None
        self.start = 0
        self.total = 0


class Server:
    def __init__(self, range_tree, join_tree, *, nslots: int = 3, max_windows: int = 16384,
                 pool_ids: int = 1 << 27, one_per_batch: bool = False, split_kmin: int | None = 16):
        import torch

        import paper_2309_16913_amd as rt
        self.torch, self.rt = torch, rt
        self.trees = {"select": range_tree, "join": join_tree}
        if split_kmin is not None:
            # served windows span up to 1e-2 of the space: large ones are split
            # over many lane groups so one window does not serialize a batch
            for t in (range_tree, join_tree):
                t.set_split(split_kmin)
        self.nslots = nslots
        self.one_per_batch = one_per_batch
        self.max_windows = max_windows
        self.pool_ids = pool_ids
        # one id pool on the device and its pinned host mirror; a batch owns
        # the same range of both while it is in flight
        self.pool = torch.empty(max(pool_ids, 1), dtype=torch.int32, device="cuda")
        self.hpool = torch.empty(max(pool_ids, 1), dtype=torch.int32).pin_memory()
        # every slot can fill a batch as large as the whole pool
        wb = rt.select_workspace_bytes(max_windows, pool_ids)
        self.slots = [_Slot(torch, rt, max_windows, wb) for _ in range(nslots)]

    # -- stages --------------------------------------------------------------
    def _launch_count(self, sl: _Slot, b: Batch):
        torch, rt = self.torch, self.rt
        m = b.windows.shape[0]
        sl.hq[:m].copy_(torch.from_numpy(b.windows))
        with torch.cuda.stream(sl.stream):
            sl.dq[:m].copy_(sl.hq[:m], non_blocking=True)
            sl.ev_c0 = torch.cuda.Event(enable_timing=True)
            sl.ev_c0.record(sl.stream)
            rt.range_select_device_count(self.trees[b.kind], sl.dq.data_ptr(), m, sl.off.data_ptr(),
                                         sl.work.data_ptr(), sl.wb, sl.stream.cuda_stream)
            sl.ev_c1 = torch.cuda.Event(enable_timing=True)
            sl.ev_c1.record(sl.stream)
            sl.hoff[:m + 1].copy_(sl.off[:m + 1], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(sl.stream)
        sl.batch, sl.ev, sl.stage = b, ev, COUNTING

    def _counted(self, sl: _Slot, adm: Admission, st: Stats):
        """Count stage done: the exact size is known."""
        b = sl.batch
        st.gpu_count_ms += sl.ev_c0.elapsed_time(sl.ev_c1)
        m = b.windows.shape[0]
        off = sl.hoff[:m + 1].numpy()
        sl.total = int(off[m])
        adm.observe(sl.total, m, b.kind)
        if sl.total > self.pool_ids:
            st.requeued_batches += 1
            adm.requeue(b, np.diff(off), self.pool_ids)
            sl.stage, sl.batch = IDLE, None
            return
        if sl.total > adm.budget_ids:
            st.oversized_batches += 1
        sl.stage = WAITING
        sl.waited = False

    def _try_fill(self, sl: _Slot, pool: IdPool, st: Stats) -> bool:
        torch, rt = self.torch, self.rt
        start = pool.alloc(sl.total)
        if start is None:
            if not sl.waited:
                st.memory_waits += 1
                sl.waited = True
            return False
        b = sl.batch
        m = b.windows.shape[0]
        sl.start = start
        tot = sl.total
        with torch.cuda.stream(sl.stream):
            sl.ev_f0 = torch.cuda.Event(enable_timing=True)
            sl.ev_f0.record(sl.stream)
            ids_ptr = self.pool[start:].data_ptr() if tot else 0
            rt.range_select_device_fill(self.trees[b.kind], sl.dq.data_ptr(), m, sl.off.data_ptr(), ids_ptr, tot,
                                        sl.work.data_ptr(), sl.wb, sl.status.data_ptr(), sl.stream.cuda_stream)
            sl.ev_f1 = torch.cuda.Event(enable_timing=True)
            sl.ev_f1.record(sl.stream)
            sl.hstat.copy_(sl.status, non_blocking=True)
            if tot:
                self.hpool[start:start + tot].copy_(self.pool[start:start + tot], non_blocking=True)
            sl.ev = torch.cuda.Event(enable_timing=True)
            sl.ev.record(sl.stream)
        sl.stage = FILLING
        return True

    def _delivered(self, sl: _Slot, pool: IdPool, now: float, st: Stats, sink):
        b = sl.batch
        st.gpu_fill_ms += sl.ev_f0.elapsed_time(sl.ev_f1)
        st.gpu_copy_ms += sl.ev_f1.elapsed_time(sl.ev)
        tot, flags = int(sl.hstat[0]), int(sl.hstat[1])
        if flags or tot != sl.total:
            raise RuntimeError(f"device reported status {tot}/{flags} for a batch of {sl.total} ids")
        m = b.windows.shape[0]
        off = sl.hoff[:m + 1].numpy().copy()
        # views into the pinned pool: valid until the range is given to a
        # later batch, so a sink that keeps results must copy them
        ids = (self.hpool[sl.start:sl.start + tot].numpy().view(np.uint32) if tot
               else np.zeros(0, np.uint32))
        at = 0
        for r in b.reqs:
            k = r.windows.shape[0]
            lo, hi = int(off[at]), int(off[at + k])
            (st.lat_join if r.kind == "join" else st.lat_select).append(now - r.t_arrival)
            if sink is not None:
                sink(r, off[at:at + k + 1] - lo, ids[lo:hi])
            at += k
        pool.free(sl.start, tot)
        st.batches += 1
        st.windows += m
        st.ids += tot
        sl.stage, sl.batch = IDLE, None

    # -- the loop ------------------------------------------------------------
    def run(self, requests, sink=None, time_scale: float = 1.0) -> dict:
        """Serve `requests` (objects with t_arrival, kind, payload, rid) in
        real time.  `sink(req, offsets, ids)` receives every result as views
        into pinned staging memory that later batches reuse (copy what must
        be kept)."""
        # no garbage collection pass while serving: a full pass over the
        # loop's objects stalls every request in flight for milliseconds
        gc_was_on = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, sink, time_scale)
        finally:
            if gc_was_on:
                gc.enable()

    def _run(self, requests, sink, time_scale: float) -> dict:
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        budget = max(1, self.pool_ids // self.nslots)
        adm = Admission(self.max_windows, budget, self.one_per_batch)
        pool = IdPool(self.pool_ids)
        st = Stats()
        n = len(reqs)
        nxt = 0
        t0 = time.perf_counter()
        done_count = [0]

        def counted_sink(r, off, ids):
            done_count[0] += 1
            if sink is not None:
                sink(r, off, ids)
        while done_count[0] < n:
            now = (time.perf_counter() - t0) / time_scale
            # admit what has arrived (a bounded number per pass, so that a
            # burst does not hold back the launches)
            stop = min(n, nxt + 4096)
            while nxt < stop and reqs[nxt].t_arrival <= now:
                r = reqs[nxt]
                w = r.payload
                if not (isinstance(w, np.ndarray) and w.dtype == np.float32 and w.ndim == 2 and w.shape[1] == 4
                        and w.flags.c_contiguous):
                    w = np.ascontiguousarray(w, np.float32).reshape(-1, 4)
                if w.shape[0] > self.max_windows:
                    raise ValueError(f"request {r.rid} has more windows than a batch holds")
                adm.push(Pending(r.rid, r.kind, w, r.t_arrival))
                nxt += 1
            progressed = False
            for sl in self.slots:
                if sl.stage in (COUNTING, FILLING) and sl.ev.query():
                    if sl.stage == COUNTING:
                        self._counted(sl, adm, st)
                    else:
                        self._delivered(sl, pool, (time.perf_counter() - t0) / time_scale, st, counted_sink)
                    progressed = True
            # batches waiting for pool room, oldest first
            waiting = [sl for sl in self.slots if sl.stage == WAITING]
            waiting.sort(key=lambda s: s.batch.reqs[0].t_arrival)
            for sl in waiting:
                if self._try_fill(sl, pool, st):
                    progressed = True
                else:
                    break   # keep arrival order: later batches do not overtake
            for sl in self.slots:
                if sl.stage == IDLE and len(adm):
                    b = adm.next_batch()
                    if b is None:
                        break
                    self._launch_count(sl, b)
                    progressed = True
            if not progressed and nxt < n and not len(adm) and all(s.stage == IDLE for s in self.slots):
                # nothing to do until the next arrival
                wait = reqs[nxt].t_arrival - now
                if wait > 2e-4:
                    time.sleep(min(wait, 1e-3) * time_scale)
        wall = (time.perf_counter() - t0) / time_scale
        out = st.summary(wall, done_count[0])
        out["nslots"] = self.nslots
        out["max_windows"] = self.max_windows
        out["pool_ids"] = self.pool_ids
        out["batch_budget_ids"] = budget
        return out
