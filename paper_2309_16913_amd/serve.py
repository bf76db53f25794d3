"""Continuous-batching server for range-select and join requests on resident
R-trees (one GPU).

Requests arrive over time (open loop: each has a scheduled arrival time).
The loop keeps `nslots` batches in flight, one per HIP stream.  Whenever a
slot is free it admits the requests that have arrived and are waiting --
range windows are packed together into one select on the range tree, a join
request (a probe set of rectangles, answered as an index nested loop: every
probe rectangle is a window on the join tree) runs as its own batch -- and
launches the whole device select (count, scan, fill, sort) on that slot's
stream.  Requests that arrive while batches are running wait for the next
free slot, so work from several batches overlaps on the device.

Admission is bounded by output-buffer memory: every slot owns a fixed share
of the id pool.  A batch whose result does not fit is not truncated and not
dropped: its exact size is known from the status words, so it is split and
re-admitted (a single request bigger than a slot waits until every slot is
idle and then runs with the whole pool).

Latency of a request = time its result is in pinned host memory - its
scheduled arrival.  All GPU work goes through the library's device-pointer
entry point; torch supplies device memory, pinned host memory, streams and
events only.
"""

from __future__ import annotations

import gc
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# pure host policy (no GPU): which waiting requests form the next batch
# ---------------------------------------------------------------------------

@dataclass
class Pending:
    rid: int
    kind: str                    # "select" or "join"
    windows: np.ndarray          # (m, 4) float32
    t_arrival: float
    known_ids: int = -1          # exact result size once a run has reported it
    solo: bool = False           # too big for one slot: run alone with the pool


@dataclass
class Batch:
    kind: str
    reqs: list
    windows: np.ndarray
    whole_pool: bool = False


class Admission:
    """Forms batches from the waiting queue.

    * joins run one per batch; range windows are packed up to `max_windows`;
    * a request whose known size exceeds the slot share is marked solo and
      waits until every slot is idle (then it gets the whole pool);
    * requests with a known size are packed only while their sizes fit the
      slot share; unknown sizes are admitted optimistically (the device
      reports an overflow without writing past the buffer)."""

    def __init__(self, max_windows: int, slot_ids: int, pool_ids: int, one_per_batch: bool = False):
        self.max_windows = max_windows
        self.slot_ids = slot_ids
        self.pool_ids = pool_ids
        self.one_per_batch = one_per_batch   # the unbatched baseline: one request per launch
        self.queue: deque = deque()

    def push(self, p: Pending):
        self.queue.append(p)

    def push_front(self, ps):
        for p in reversed(ps):
            self.queue.appendleft(p)

    def __len__(self):
        return len(self.queue)

    def next_batch(self, all_idle: bool):
        if not self.queue:
            return None
        head = self.queue[0]
        if head.solo:
            if not all_idle:
                return None
            self.queue.popleft()
            return Batch(head.kind, [head], head.windows, whole_pool=True)
        if head.kind == "join":
            self.queue.popleft()
            return Batch("join", [head], head.windows)
        # pack waiting range windows in arrival order; join requests and solo
        # requests stay queued in place (they form batches of their own)
        reqs, known, nwin = [], 0, 0
        rest = deque()
        while self.queue:
            p = self.queue.popleft()
            take = (p.kind == "select" and not p.solo and nwin + p.windows.shape[0] <= self.max_windows
                    and not (p.known_ids >= 0 and reqs and known + p.known_ids > self.slot_ids)
                    and not (self.one_per_batch and reqs))
            if take:
                reqs.append(p)
                nwin += p.windows.shape[0]
                if p.known_ids >= 0:
                    known += p.known_ids
            else:
                rest.append(p)
                if nwin >= self.max_windows or (self.one_per_batch and reqs):
                    break
        rest.extend(self.queue)
        self.queue = rest
        if not reqs:
            return None
        return Batch("select", reqs, np.concatenate([r.windows for r in reqs]))

    def overflowed(self, batch: Batch, counts: np.ndarray):
        """Re-queue an overflowed batch at the front with exact sizes known:
        split it so that each part fits a slot; a single request larger than
        a slot becomes solo."""
        per_req = []
        at = 0
        for r in batch.reqs:
            m = r.windows.shape[0]
            r.known_ids = int(counts[at:at + m].sum())
            at += m
            if r.known_ids > self.pool_ids:
                raise MemoryError(f"request {r.rid} needs {r.known_ids} ids, more than the whole pool")
            if r.known_ids > self.slot_ids or batch.whole_pool:
                r.solo = True
            per_req.append(r)
        self.push_front(per_req)


# ---------------------------------------------------------------------------
# GPU server
# ---------------------------------------------------------------------------

@dataclass
class Stats:
    lat_select: list = field(default_factory=list)
    lat_join: list = field(default_factory=list)
    batches: int = 0
    overflows: int = 0
    windows: int = 0
    ids: int = 0
    gpu_select_ms: float = 0.0    # device time of the selects (incl. overflowed attempts)
    gpu_copy_ms: float = 0.0      # device time of the result copies to pinned memory

    def summary(self, wall: float, nreq: int) -> dict:
        def pct(v, q):
            return float(np.percentile(np.array(v) * 1e3, q)) if v else None
        return {
            "requests": nreq, "wall_s": wall, "throughput_req_per_s": nreq / wall if wall > 0 else None,
            "windows_per_s": self.windows / wall if wall > 0 else None,
            "select_p50_ms": pct(self.lat_select, 50), "select_p99_ms": pct(self.lat_select, 99),
            "join_p50_ms": pct(self.lat_join, 50), "join_p99_ms": pct(self.lat_join, 99),
            "batches": self.batches, "overflow_retries": self.overflows, "ids": self.ids,
            "gpu_select_ms": self.gpu_select_ms, "gpu_copy_ms": self.gpu_copy_ms,
        }


class _Slot:
    def __init__(self, torch, rt, max_windows, cap_ids):
        self.stream = torch.cuda.Stream()
        self.dq = torch.empty((max_windows, 4), dtype=torch.float32, device="cuda")
        self.off = torch.empty(max_windows + 1, dtype=torch.int64, device="cuda")
        self.status = torch.zeros(2, dtype=torch.int64, device="cuda")
        self.hq = torch.empty((max_windows, 4), dtype=torch.float32).pin_memory()
        self.hoff = torch.empty(max_windows + 1, dtype=torch.int64).pin_memory()
        self.hstat = torch.empty(2, dtype=torch.int64).pin_memory()
        self.cap = cap_ids
        self.ids = None
        self.hids = None
        self.work = None
        self.wb = 0
        self.batch = None
        self.done_ev = None
        self.stage = 0          # 0 idle, 1 running select, 2 copying results


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
        self.slot_ids = pool_ids // nslots
        self.slots = [_Slot(torch, rt, max_windows, self.slot_ids) for _ in range(nslots)]
        # one id pool; every slot views its share, a solo batch uses all of it
        self.pool = torch.empty(pool_ids, dtype=torch.int32, device="cuda")
        self.hpool = torch.empty(pool_ids, dtype=torch.int32).pin_memory()
        wb = rt.select_workspace_bytes(max_windows, pool_ids)
        self.work = torch.empty(wb, dtype=torch.uint8, device="cuda")
        self.wb_full = wb
        for k, sl in enumerate(self.slots):
            sl.ids = self.pool[k * self.slot_ids:(k + 1) * self.slot_ids]
            sl.hids = self.hpool[k * self.slot_ids:(k + 1) * self.slot_ids]
            sl.wb = rt.select_workspace_bytes(max_windows, self.slot_ids)
            sl.work = torch.empty(sl.wb, dtype=torch.uint8, device="cuda")

    # -- one batch ---------------------------------------------------------
    def _launch(self, sl: _Slot, b: Batch):
        torch, rt = self.torch, self.rt
        m = b.windows.shape[0]
        ids, hids, cap, work, wb = sl.ids, sl.hids, sl.cap, sl.work, sl.wb
        if b.whole_pool:
            ids, hids, cap, work, wb = self.pool, self.hpool, self.pool_ids, self.work, self.wb_full
        sl.cur = (ids, hids, cap)
        sl.hq[:m].copy_(torch.from_numpy(b.windows))
        with torch.cuda.stream(sl.stream):
            sl.dq[:m].copy_(sl.hq[:m], non_blocking=True)
            sl.ev0 = torch.cuda.Event(enable_timing=True)
            sl.ev0.record(sl.stream)
            rt.range_select_device(self.trees[b.kind], sl.dq.data_ptr(), m, sl.off.data_ptr(), ids.data_ptr(),
                                   cap, work.data_ptr(), wb, sl.status.data_ptr(), sl.stream.cuda_stream)
            sl.hstat.copy_(sl.status, non_blocking=True)
            sl.hoff[:m + 1].copy_(sl.off[:m + 1], non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(sl.stream)
        sl.batch, sl.done_ev, sl.stage = b, ev, 1

    def _finish_stage1(self, sl: _Slot, adm: Admission, st: Stats):
        """Select done: on overflow re-queue, else start the copy of the ids."""
        torch = self.torch
        b = sl.batch
        st.gpu_select_ms += sl.ev0.elapsed_time(sl.done_ev)
        sl.ev1 = sl.done_ev
        tot, flags = int(sl.hstat[0]), int(sl.hstat[1])
        m = b.windows.shape[0]
        if flags & 2:
            raise RuntimeError("device reported an internal error while serving")
        if flags & 1:
            st.overflows += 1
            off = sl.hoff[:m + 1].numpy()
            adm.overflowed(b, np.diff(off))
            sl.stage, sl.batch = 0, None
            return
        ids, hids, _ = sl.cur
        with torch.cuda.stream(sl.stream):
            if tot:
                hids[:tot].copy_(ids[:tot], non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(sl.stream)
        sl.total, sl.done_ev, sl.stage = tot, ev, 2

    def _finish_stage2(self, sl: _Slot, now: float, st: Stats, sink):
        b = sl.batch
        st.gpu_copy_ms += sl.ev1.elapsed_time(sl.done_ev)
        m = b.windows.shape[0]
        off = sl.hoff[:m + 1].numpy().copy()
        _, hids, _ = sl.cur
        # views into the slot's pinned buffer: valid until the slot is reused,
        # so a sink that keeps results must copy them
        ids = hids[:sl.total].numpy().view(np.uint32) if sl.total else np.zeros(0, np.uint32)
        at = 0
        for r in b.reqs:
            k = r.windows.shape[0]
            lo, hi = int(off[at]), int(off[at + k])
            lat = now - r.t_arrival
            (st.lat_join if r.kind == "join" else st.lat_select).append(lat)
            if sink is not None:
                sink(r, off[at:at + k + 1] - lo, ids[lo:hi])
            at += k
        st.batches += 1
        st.windows += m
        st.ids += sl.total
        sl.stage, sl.batch = 0, None

    # -- the loop ------------------------------------------------------------
    def run(self, requests, sink=None, time_scale: float = 1.0) -> dict:
        """Serve `requests` (objects with t_arrival, kind, payload, rid) in
        real time.  `sink(req, offsets, ids)` receives every result as views
        into pinned staging memory that is reused by later batches (copy what
        must be kept)."""
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
        adm = Admission(self.max_windows, self.slot_ids, self.pool_ids, self.one_per_batch)
        st = Stats()
        n = len(reqs)
        nxt, finished = 0, 0
        t0 = time.perf_counter()
        done_count = [0]

        def counted_sink(r, off, ids):
            done_count[0] += 1
            if sink is not None:
                sink(r, off, ids)
        while done_count[0] < n:
            now = (time.perf_counter() - t0) / time_scale
            while nxt < n and reqs[nxt].t_arrival <= now:
                r = reqs[nxt]
                if np.asarray(r.payload).size // 4 > self.max_windows:
                    raise ValueError(f"request {r.rid} has more windows than a batch holds")
                adm.push(Pending(r.rid, r.kind, np.ascontiguousarray(r.payload, np.float32).reshape(-1, 4),
                                 r.t_arrival))
                nxt += 1
            progressed = False
            for sl in self.slots:
                if sl.stage and sl.done_ev.query():
                    if sl.stage == 1:
                        self._finish_stage1(sl, adm, st)
                    else:
                        self._finish_stage2(sl, (time.perf_counter() - t0) / time_scale, st, counted_sink)
                    progressed = True
            all_idle = all(s.stage == 0 for s in self.slots)
            for sl in self.slots:
                if sl.stage == 0 and len(adm):
                    b = adm.next_batch(all_idle)
                    if b is None:
                        break
                    self._launch(sl, b)
                    all_idle = False
                    progressed = True
            if not progressed and nxt < n and not len(adm) and all(s.stage == 0 for s in self.slots):
                # nothing to do until the next arrival
                wait = reqs[nxt].t_arrival - now
                if wait > 2e-4:
                    time.sleep(min(wait, 1e-3) * time_scale)
        wall = (time.perf_counter() - t0) / time_scale
        finished = done_count[0]
        out = st.summary(wall, finished)
        out["nslots"] = self.nslots
        out["max_windows"] = self.max_windows
        out["pool_ids"] = self.pool_ids
        return out
