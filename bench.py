#!/usr/bin/env python3
"""Benchmark: batched R-tree range select (and join / batched / served legs)
on one MI355X.

Default workload (the "step"): one complete range select -- count pass,
scan, fill pass, segmented sort -- of 1,000,000 query windows (selectivity
log-uniform in [1e-6, 1e-3]) against a 10,000,000-rectangle tree (half
uniform, half in 64 Gaussian clusters, sides U[0, 1e-4]), fanout, node layout
and work mapping chosen by the autotuner on that workload, with queries,
tree and output buffers resident in device memory before timing starts.
Prints one JSON line.

Extra legs (same JSON line, under "legs"): device STR build; spatial join of
two 2M-rectangle relations; the 256-instance batched select (persistent +
graph vs plain per-tree launches); the served request stream (open loop at
five offered rates, closed loop, unbatched baseline); the same serving tree
selected device-side in one closed-loop batch with the results left in HBM;
and the scalar CPU oracle timed on bounded samples of the select and join
workloads on one thread and on all host cores ("cpu_baseline").

`--pmc-summary` turns two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) of
this script into the traffic summaries that the roofline entries read from
profiles/ (no GPU needed for that step).
"""

from __future__ import annotations

import argparse
import csv
import ctypes as C
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_LANE_OPS_PER_S = 256 * 64 * 2.4e9   # 256 CUs x 64 lanes x 2.4 GHz, one lane-op per lane per clock
METRIC = "range queries/s and join pairs/s on 1 GPU (bit-exact), % HBM peak; p99 latency"
SERVE_RATES = [1e4, 3e4, 1e5, 3e5, 1e6]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles through the HIP runtime already loaded in-process."""

    def __init__(self):
        self.h = C.CDLL("libamdhip64.so.7")
        self.h.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.h.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.h.hipEventDestroy.argtypes = [C.c_void_p]
        self.h.hipEventSynchronize.argtypes = [C.c_void_p]
        self.h.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]

    def create(self, n):
        out = []
        for _ in range(n):
            e = C.c_void_p()
            assert self.h.hipEventCreate(C.byref(e)) == 0
            out.append(e.value)
        return out

    def record(self, e, stream):
        assert self.h.hipEventRecord(C.c_void_p(e), C.c_void_p(stream)) == 0

    def ms(self, a, b):
        f = C.c_float()
        assert self.h.hipEventSynchronize(C.c_void_p(b)) == 0
        assert self.h.hipEventElapsedTime(C.byref(f), C.c_void_p(a), C.c_void_p(b)) == 0
        return float(f.value)


# ---------------------------------------------------------------------------
# HBM traffic summaries (profiles/<tag>_traffic.txt)
# ---------------------------------------------------------------------------

PHASE_SOURCES = {"count": ("select.hip", "rt_internal.h"), "fill": ("select.hip", "rt_internal.h"),
                 "sort": ("segsort.hip", "rt_internal.h"), "batch": ("batch_kernels.hip", "rt_internal.h")}


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2309_16913_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_phase(name: str):
    """Which phase of a select step a kernel belongs to (None: not timed)."""
    m = re.search(r"select_kernel<\d+, \d+, (\d), \d(?:, \d)?>", name)
    if m:
        return {"0": "count", "1": "fill"}.get(m.group(1))
    if "batch_replay_kernel" in name:   # the batch graph's replayed fill
        return "batch"
    if "bulk_copy_kernel" in name or "replay_kernel" in name:   # the fill stage's other kernels
        return "fill"
    if "segsort" in name or "seg_classify" in name:
        return "sort"
    m = re.search(r"batch_kernel<(\d)(?:, \d)?>", name)
    if m:
        return "batch_count" if m.group(1) == "0" else "batch"
    return None


def read_traffic(tag):
    """HBM bytes per launch, per phase, from a committed counter summary whose
    kernels still have the source they were measured on; {} if none."""
    p = os.path.join(ROOT, "profiles", f"{tag}_traffic.txt")
    if not os.path.exists(p):
        return {}
    vals = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    out = {}
    for ph, srcs in PHASE_SOURCES.items():
        if f"{ph}_bytes_per_launch" in vals and vals.get(f"{ph}_source_hash") == source_hash(*srcs):
            out[ph] = float(vals[f"{ph}_bytes_per_launch"])
            out[ph + "_ms"] = float(vals.get(f"{ph}_ms_per_launch", "nan"))
    if out:
        out["file"] = os.path.relpath(p, ROOT)
    return out


def _counter_rows(d):
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *counter_collection.csv under {d}")
    return rows


def _per_dispatch(rows, counter):
    """{dispatch id: (kernel name, value summed over the counter's instances,
    start, end)}."""
    out = {}
    for r in rows:
        cn = r.get("Counter_Name", "")
        if cn != counter:
            continue
        did = int(r.get("Dispatch_Id") or r.get("Correlation_Id"))
        v = float(r["Counter_Value"])
        name = r.get("Kernel_Name", "")
        s, e = int(r.get("Start_Timestamp", 0) or 0), int(r.get("End_Timestamp", 0) or 0)
        if did in out:
            out[did] = (name, out[did][1] + v, s, e)
        else:
            out[did] = (name, v, s, e)
    return out


def pmc_summary(args):
    """Write profiles/<tag>_traffic.txt from a FETCH_SIZE run and a WRITE_SIZE
    run of this script (both with --calib-copy-mib, so that the first copies
    calibrate the counters against a copy of known size)."""
    fetch = _per_dispatch(_counter_rows(args.fetch_dir), "FETCH_SIZE")
    write = _per_dispatch(_counter_rows(args.write_dir), "WRITE_SIZE")
    calib_bytes = args.calib_copy_mib << 20

    def calib(d):
        ids = sorted(k for k, v in d.items() if "copyBuffer" in v[0] or "copy" in v[0].lower())[:3]
        if len(ids) < 3:
            raise SystemExit("calibration copies not found")
        return sum(d[k][1] for k in ids) * 1024.0 / 3.0, set(ids)
    fk, fids = calib(fetch)
    wk, wids = calib(write)
    fetch_scale = calib_bytes / fk      # FETCH_SIZE of a copy reads 1/scale of its bytes
    write_scale = calib_bytes / wk
    # phase -> kernel name -> [(dispatch id, bytes)] per counter, and durations
    phases = {}
    for d, scale, skip, key in ((fetch, fetch_scale, fids, "fetch"), (write, write_scale, wids, "write")):
        for did, (name, v, s, e) in sorted(d.items()):
            if did in skip:
                continue
            ph = kernel_phase(name)
            if ph is None:
                continue
            k = phases.setdefault(ph, {}).setdefault(name, {"fetch": [], "write": [], "ms": []})
            k[key].append((did, v * 1024.0 * scale))
            if key == "fetch" and e > s:
                k["ms"].append((did, (e - s) / 1e6))
    # --last N: only the last N steps, which start at the N-th last launch of
    # the step's first phase
    thr = {"fetch": 0, "write": 0}
    if args.last:
        first = "batch_count" if "batch_count" in phases else "count"
        for key in thr:
            ids = sorted(did for k in phases.get(first, {}).values() for did, _ in k[key])
            thr[key] = ids[-args.last] if len(ids) >= args.last else 0
    lines = [f"# {args.title}",
             "# Two counter runs of the same command (FETCH_SIZE, then WRITE_SIZE):",
             f"#   cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d <fetch> -o run "
             f"-- python3 /root/repo/bench.py {args.bench_args}",
             f"#   cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv -d <write> -o run "
             f"-- python3 /root/repo/bench.py {args.bench_args}",
             f"#   python3 bench.py --pmc-summary --fetch-dir <fetch> --write-dir <write> --tag {args.tag} "
             f"--calib-copy-mib {args.calib_copy_mib}" + (f" --last {args.last}" if args.last else ""),
             "# FETCH_SIZE / WRITE_SIZE: KiB per dispatch between L2 and the fabric (Infinity Cache hits",
             "# included, so an upper bound on DRAM bytes), scaled by the first three copies of",
             f"# {args.calib_copy_mib} MiB: fetch_scale {fetch_scale:.4f}, write_scale {write_scale:.4f}.",
             "# Per phase: the bytes of one step of the phase (average over launches of each of its",
             "# kernels, summed over the kernels; the sort sums its kernels per step), and its kernel",
             "# time per step under the counter run."]
    nsteps = args.last or max(1, args.steps_in_run)
    for ph, kernels in sorted(phases.items()):
        fb = wb = ms = 0.0
        launches = 0
        for name, k in kernels.items():
            kf = [v for did, v in k["fetch"] if did >= thr["fetch"]]
            kw = [v for did, v in k["write"] if did >= thr["write"]]
            km = [v for did, v in k["ms"] if did >= thr["fetch"]]
            if not kf or not kw:
                continue
            # the sort launches a varying number of kernels per step: its
            # sums go per step; any other kernel runs once per step of its phase
            pf, pw = (nsteps, nsteps) if ph == "sort" else (len(kf), len(kw))
            fb += sum(kf) / pf
            wb += sum(kw) / pw
            ms += sum(km) / (nsteps if ph == "sort" else max(1, len(km))) if km else float("nan")
            launches += len(kf)
        if not launches:
            continue
        src = PHASE_SOURCES.get(ph if ph != "batch_count" else "batch")
        lines += [f"{ph}_fetch_bytes_per_launch: {fb:.0f}", f"{ph}_write_bytes_per_launch: {wb:.0f}",
                  f"{ph}_bytes_per_launch: {fb + wb:.0f}", f"{ph}_ms_per_launch: {ms:.4f}",
                  f"{ph}_launches: {launches}"]
        if src:
            lines.append(f"{ph}_source_hash: {source_hash(*src)}")
    lines += [f"fetch_scale: {fetch_scale:.4f}", f"write_scale: {write_scale:.4f}"]
    out = os.path.join(ROOT, "profiles", f"{args.tag}_traffic.txt")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def pmc_table(args):
    """Per-kernel averages of the counters of one rocprofv3 --pmc run of
    this script (weighted by dispatch duration), as a markdown table in
    profiles/<tag>.md."""
    rows = _counter_rows(args.fetch_dir)
    per = {}
    for r in rows:
        did = int(r.get("Dispatch_Id") or r.get("Correlation_Id"))
        d = per.setdefault(did, {"name": r.get("Kernel_Name", ""), "t": 0.0, "c": {}})
        s_, e_ = int(r.get("Start_Timestamp", 0) or 0), int(r.get("End_Timestamp", 0) or 0)
        d["t"] = max(d["t"], (e_ - s_) / 1e6)
        d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    agg = {}
    for d in per.values():
        a = agg.setdefault(d["name"], {"n": 0, "t": 0.0, "c": {}})
        a["n"] += 1
        a["t"] += d["t"]
        for k, v in d["c"].items():
            a["c"][k] = a["c"].get(k, 0.0) + v * d["t"]
    names = sorted({k for a in agg.values() for k in a["c"]})
    pat = re.compile(args.kernel_regex) if args.kernel_regex else None
    lines = [f"# {args.title}",
             f"# Command: cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc {' '.join(names)} --output-format csv "
             f"-d <out> -o run -- python3 /root/repo/bench.py {args.bench_args}",
             f"# Summary: python3 bench.py --pmc-table --fetch-dir <out> --tag {args.tag}"
             + (f" --kernel-regex '{args.kernel_regex}'" if args.kernel_regex else ""),
             "# Per kernel: dispatches, total ms under the counter run, and each counter averaged over the",
             "# dispatches weighted by their duration (derived metrics such as VALUBusy are percentages).", "",
             "| kernel | dispatches | total ms | " + " | ".join(names) + " |",
             "|---|---|---|" + "---|" * len(names)]
    for name, a in sorted(agg.items(), key=lambda kv: -kv[1]["t"]):
        if pat and not pat.search(name):
            continue
        vals = [a["c"].get(k, 0.0) / a["t"] if a["t"] > 0 else 0.0 for k in names]
        lines.append(f"| `{name[:80]}` | {a['n']} | {a['t']:.2f} | " + " | ".join(f"{v:.4g}" for v in vals) + " |")
    out = os.path.join(ROOT, "profiles", f"{args.tag}.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def stats_table(args):
    """profiles/<tag>.md from a rocprofv3 --kernel-trace --stats run of this
    script (its *kernel_stats.csv): calls, average and total time per kernel."""
    files = sorted(glob.glob(os.path.join(args.fetch_dir, "**", "*kernel_stats.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no *kernel_stats.csv under {args.fetch_dir}")
    rows = list(csv.DictReader(open(files[0], newline="")))
    lines = [f"# {args.title}",
             f"# Command: cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
             f"-d <out> -o run -- python3 /root/repo/bench.py {args.bench_args}",
             f"# Summary: python3 bench.py --stats-table --fetch-dir <out> --tag {args.tag}", "",
             "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows[:args.top]:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    out = os.path.join(ROOT, "profiles", f"{args.tag}.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def roofline_entry(kernel, live_ms, compulsory_bytes, visit_bytes, traffic):
    """Roofline of one kernel launch.  frac = measured HBM bytes (counter
    profile of the current source) / live duration / peak; without a current
    profile, the compulsory bytes (what must cross HBM at least once: the
    tree, the windows, the output) stand in.  effective_frac counts every
    visited node as if read from HBM (L2 / Infinity Cache hits included), so
    it is not bounded by 1."""
    t = live_ms / 1e3
    out = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "kernel": kernel, "time_ms": live_ms,
           "compulsory_bytes": compulsory_bytes, "compulsory_frac": compulsory_bytes / t / 1e9 / HBM_PEAK_GBS,
           "algorithmic_bytes": visit_bytes, "effective_frac": visit_bytes / t / 1e9 / HBM_PEAK_GBS}
    if traffic is not None:
        out.update(achieved=traffic / t / 1e9, traffic=traffic,
                   basis="measured HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated) / live kernel time")
    else:
        out.update(achieved=compulsory_bytes / t / 1e9, traffic=None,
                   basis="compulsory bytes / live kernel time (no counter profile of the current source)")
    out["frac"] = out["achieved"] / HBM_PEAK_GBS
    return out


# ---------------------------------------------------------------------------
# legs
# ---------------------------------------------------------------------------

def select_leg(rt, torch, ev, args, rects, queries, kmin=0):
    t0 = time.time()
    tree = rt.build_str(rects, args.fanout, args.layout)
    tree.set_split(kmin)
    build_s = time.time() - t0
    info = tree.info()
    nq = queries.shape[0]
    dq = torch.from_numpy(queries).cuda()
    off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    # size the output with the count-only entry point
    counts = torch.empty(nq, dtype=torch.int32, device="cuda")
    wb0 = rt.select_workspace_bytes(nq, 0)
    work0 = torch.empty(wb0, dtype=torch.uint8, device="cuda")
    rt.range_count_device(tree, dq.data_ptr(), nq, counts.data_ptr(), work0.data_ptr(), wb0, stream.cuda_stream)
    torch.cuda.synchronize()
    cap = int(counts.to(torch.int64).sum().item())
    del work0, counts
    ids = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    # room for the count pass's records: the fill replays them
    wb = (rt.select_replay_workspace_bytes if args.replay else rt.select_workspace_bytes)(nq, cap)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    status = torch.zeros(2, dtype=torch.int64, device="cuda")
    events = [ev.create(5) for _ in range(args.steps)]

    def step(e=None):
        rt.range_select_device_timed(tree, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), cap, work.data_ptr(),
                                     wb, status.data_ptr(), stream.cuda_stream, e)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = status.cpu().numpy()
    assert st[1] == 0 and st[0] == cap, f"select status {st} (cap {cap})"
    rec_chunks, rec_over = rt.select_replay_info(work.data_ptr())
    replay = {"workspace_bytes": wb, "record_chunks": rec_chunks, "overflowed": rec_over,
              "replayed": bool(args.replay and rec_chunks and not rec_over)}
    lookahead = None
    if args.lookahead:
        # the lookahead variant (loads one node ahead after each leaf), timed
        # the same way on the same buffers, then switched off again
        tree.set_lookahead(True)
        la_ev = ev.create(5)
        step()
        step(la_ev)
        torch.cuda.synchronize()
        tree.set_lookahead(False)
        lookahead = {"count": ev.ms(la_ev[0], la_ev[1]), "fill": ev.ms(la_ev[2], la_ev[3]),
                     "step": ev.ms(la_ev[0], la_ev[4])}
    phases = {"count": [], "scan": [], "fill": [], "sort": []}
    for e in events:
        phases["count"].append(ev.ms(e[0], e[1]))
        phases["scan"].append(ev.ms(e[1], e[2]))
        phases["fill"].append(ev.ms(e[2], e[3]))
        phases["sort"].append(ev.ms(e[3], e[4]))
    avg = {k: float(np.mean(v)) for k, v in phases.items()}
    vn, ve, vc = rt.visit_stats(tree, queries)
    tree_bytes = int(info.device_bytes)
    # visit-based (section 8(d) model: every visited node's entries + header)
    node_bytes = 20 * ve + 8 * vn
    visit = {"count": 16 * nq + node_bytes,
             "fill": 16 * nq + node_bytes + 4 * cap + 4 * vc + 8 * (nq + 1),
             "sort": 8 * cap + 8 * (nq + 1)}
    # compulsory: the tree once, the windows, what the phase must write/read
    comp = {"count": 16 * nq + tree_bytes + 4 * nq,
            "fill": 16 * nq + tree_bytes + 8 * (nq + 1) + 4 * cap,
            "sort": 8 * cap + 8 * (nq + 1)}
    if replay["replayed"]:
        # the count pass also writes its records (16 B each, at most 256 per
        # chunk taken); the fill reads them and each hit id once, and writes
        # the ids, without visiting nodes
        rb = 16 * 256 * rec_chunks
        visit["count"] += rb
        comp["count"] += rb
        visit["fill"] = rb + 8 * (nq + 1) + 8 * cap
        comp["fill"] = rb + 8 * (nq + 1) + 4 * cap + min(tree_bytes, 4 * cap)
    return dict(tree=tree, info=info, build_s=build_s, cap=cap, wall=wall, avg=avg, vn=vn, ve=ve, vc=vc,
                visit=visit, comp=comp, off=off, ids=ids, lookahead=lookahead, replay=replay)


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    # the host share of one GPU on a shared machine (OMP_NUM_THREADS is set to it)
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = min(nproc, share) if share > 0 else nproc
    return model, nproc, threads


def cpu_baseline(args, rects, queries, gpu_off, gpu_ids, join=None):
    """The oracle (plain scalar C, test infrastructure) on bounded samples of
    the timed workloads: 1 thread and all host cores (static partition),
    query phase only; every sampled result is compared with the GPU's."""
    import oracle
    o = oracle.get()
    model, nproc, threads = cpu_info()
    t0 = time.time()
    ot = o.build_str(rects, 16)
    build_s = time.time() - t0

    def check(done, woff, wids):
        g0, g1 = int(gpu_off[done]), int(gpu_off[done + woff.shape[0] - 1])
        goff = gpu_off[done:done + woff.shape[0]] - g0
        return (np.array_equal(goff, woff.astype(np.int64)) and
                np.array_equal(gpu_ids[g0:g1].view(np.uint32), wids))

    def run(nthreads, budget_s, chunk, start):
        done, spent, bad = 0, 0.0, 0
        while spent < budget_s and start + done < queries.shape[0]:
            q = queries[start + done:start + done + chunk]
            t1 = time.perf_counter()
            woff, wids = o.select(ot, q) if nthreads == 1 else o.select_mt(ot, q, nthreads)
            spent += time.perf_counter() - t1
            if not check(start + done, woff, wids):
                bad += 1
            done += q.shape[0]
        return done, spent, bad

    n1, s1, b1 = run(1, args.cpu_seconds, 2000, 0)
    nm, sm, bm = run(threads, args.cpu_seconds, 2000 * threads, n1)
    out = dict(value=nm / sm, unit="queries/s", cores=threads, kind="oracle",
               sample=f"select: windows {n1}..{n1 + nm} of the {queries.shape[0]} timed windows against the "
                      f"{rects.shape[0]}-rectangle tree on {threads} threads (static partition of the windows), "
                      f"query phase only; oracle STR build ({build_s:.1f} s, fanout 16) not included",
               cpu_model=model, nproc=nproc,
               one_thread={"value": n1 / s1, "unit": "queries/s", "cores": 1,
                           "sample": f"first {n1} windows of the same workload"},
               checked_queries=n1 + nm, mismatching_chunks=b1 + bm)
    if join is not None:
        a, b, gpu_pairs = join
        ta, tb = o.build_str(a, 32), o.build_str(b, 32)
        t1 = time.perf_counter()
        p1 = o.join(ta, tb)
        j1 = time.perf_counter() - t1
        t1 = time.perf_counter()
        pm = o.join_mt(ta, tb, threads)
        jm = time.perf_counter() - t1
        out["join"] = {"pairs": int(p1.shape[0]), "one_thread_pairs_per_s": p1.shape[0] / j1,
                       "all_cores_pairs_per_s": pm.shape[0] / jm, "cores": threads,
                       "gpu_pairs_equal_oracle": bool(np.array_equal(p1, gpu_pairs) and np.array_equal(pm, p1)),
                       "sample": f"the whole {a.shape[0]} x {b.shape[0]} join (fanout 32 oracle trees)"}
    return out


def join_leg(rt, torch, args):
    """C3 join (2M uniform x 2M clustered at full size).  Trees are built on
    the device with every node sorted by low x; the headline variant is the
    library default on such trees (O3 outer slicing + O5 many-to-many inner
    shrinking + the LB lower bound on the inner scan).  Times are for the
    device-output call (pairs left in HBM); the host-output call (pairs
    copied over PCIe) is reported beside it, and every variant of section 4
    is timed on the same trees and compared with the default's pairs."""
    import rtgen
    a, b = rtgen.c3_join(args.join_n)
    F = args.join_fanout
    ta = rt.build_str(a, F, "soa", sort_lx=True)
    tb = rt.build_str(b, F, "soa", sort_lx=True)
    n = rt.spatial_join_device(ta, tb, 0, 0)
    buf = torch.empty(2 * max(n, 1), dtype=torch.int32, device="cuda")
    ref = None

    def time_dev(flags):
        nonlocal ref
        rt.spatial_join_device(ta, tb, buf.data_ptr(), n, flags)   # warm
        ts = []
        for _ in range(args.join_reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            got = rt.spatial_join_device(ta, tb, buf.data_ptr(), n, flags)
            ts.append(time.perf_counter() - t0)
            assert got == n
        if ref is None:
            ref = buf.clone()
        same = bool(torch.equal(buf, ref))
        return float(np.median(ts)) * 1e3, same

    ms, _ = time_dev(None)
    # one-off join: new trees every call (no graph replay, no reused level sizes)
    once = []
    for k in range(3):
        tb2 = rt.build_str(b, F, "soa", sort_lx=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rt.spatial_join_device(ta, tb2, buf.data_ptr(), n)
        once.append(time.perf_counter() - t0)
        tb2.free()
    hts = []
    for _ in range(args.join_reps):
        t0 = time.perf_counter()
        p = rt.spatial_join(ta, tb)
        hts.append(time.perf_counter() - t0)
    assert p.shape[0] == n
    variants = {}
    all_same = True
    for name, fl in [("tile", rt.JOIN_TILE), ("cand", 0), ("O3", rt.JOIN_O3), ("O3+O4", rt.JOIN_O3 | rt.JOIN_O4),
                     ("O3+O5", rt.JOIN_O3 | rt.JOIN_O5), ("O5", rt.JOIN_O5),
                     ("O3+O5+LB", rt.JOIN_O3 | rt.JOIN_O5 | rt.JOIN_LB)]:
        _, tests = rt.spatial_join(ta, tb, fl, with_tests=True)
        vms, same = time_dev(fl)
        all_same &= same
        variants[name] = dict(ms=round(vms, 4), predicate_tests=tests, pairs_equal_default=same)
    ia, ib = ta.info(), tb.info()
    # byte / operation model of the plain synchronized traversal (section 4):
    # every visited node pair loads both nodes (20 B per entry + 8 B header
    # each), every emitted pair is 8 B; 7 lane operations per entry predicate
    npairs_v, epairs, ents = rt.join_visit_stats(ta, tb)
    vbytes = 20 * ents + 16 * npairs_v + 8 * n
    model = {"node_pairs": npairs_v, "entry_predicates": epairs, "entries_loaded": ents,
             "visit_bytes": vbytes, "effective_GBps": vbytes / (ms / 1e3) / 1e9,
             "effective_frac": vbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
             "algorithmic_lane_ops": 7 * epairs,
             "algorithmic_valu_frac": 7 * epairs / (ms / 1e3) / VALU_LANE_OPS_PER_S,
             "note": "plain-traversal model; the default O3+O5+LB expansion evaluates "
                     f"{variants['O3+O5+LB']['predicate_tests']} of these predicates"}
    return dict(workload=f"join_uniform{args.join_n}_x_clustered{args.join_n}_f{F}_soa_sorted_lx", pairs=int(n),
                model=model,
                ms=ms, pairs_per_s=n / (ms / 1e3), one_off_ms=float(np.median(once)) * 1e3,
                host_output_ms=float(np.median(hts)) * 1e3, variants_ms=variants,
                variants_pairs_equal=all_same, tree_bytes=[int(ia.device_bytes), int(ib.device_bytes)],
                note="device-output call, synchronous; repeated calls replay a captured graph, one_off_ms "
                     "builds a new inner tree before every call"), p, (a, b)


def build_leg(rt, torch, args, rects):
    """Device STR bulk load of the resident rectangles (not part of the
    query step): rectangles already in HBM, and from host memory."""
    d = torch.from_numpy(rects).cuda()
    s = torch.cuda.current_stream()
    out = {}
    for sort_lx in (False, True):
        ts = []
        for _ in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t = rt.build_str_device(d.data_ptr(), rects.shape[0], args.fanout, args.layout, s.cuda_stream,
                                    sort_lx=sort_lx)
            ts.append(time.perf_counter() - t0)
            t.free()
        out["device_ms" + ("_sorted_lx" if sort_lx else "")] = float(np.median(ts[1:])) * 1e3
    t0 = time.perf_counter()
    t = rt.build_str(rects, args.fanout, args.layout)
    out["host_input_ms"] = (time.perf_counter() - t0) * 1e3
    t.free()
    del d
    out["rects"] = int(rects.shape[0])
    out["fanout"] = args.fanout
    out["layout"] = args.layout
    return out


def batch_leg(rt, torch, args):
    """256 independent instances in one persistent launch replayed from a
    HIP graph.  Fanout and layout per size class of the trees, chosen by
    timing each class's batch with every candidate (BatchTuner); beside it
    the library's own per-tree choice (fanout 0, RT_LAYOUT_AUTO).  Baselines:
    the same trees with plain per-tree launches, and plain per-tree launches
    on untuned trees (fanout 32, SoA)."""
    import rtgen
    t0 = time.time()
    inst = rtgen.c4_batch(ntrees=args.batch_trees, scale=args.batch_scale)
    gen_s = time.time() - t0
    nq = sum(x.queries.shape[0] for x in inst)

    def timed(b, fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        tot, flags = b.status()
        assert flags == 0
        return float(np.median(ts)), tot

    # per-size-class fanout and layout, timed in batch context
    from paper_2309_16913_amd.autotune import BatchTuner
    t0 = time.time()
    bt = BatchTuner()
    choice = bt.tune(inst)
    tune_s = time.time() - t0
    t0 = time.time()
    trees = bt.build(inst, choice)
    build_s = time.time() - t0
    cfg = {}
    for t in trees:
        i = t.info()
        k = f"{i.fanout}/{['aos', 'soa', 'auto', 'd2'][i.layout]}"
        cfg[k] = cfg.get(k, 0) + 1
    b = rt.Batch(trees, [x.queries for x in inst])
    out = {}
    for name, fn in (("batched_graph", b.run), ("plain_per_tree", b.run_plain)):
        if args.batch_tuned_only and name != "batched_graph":
            continue
        ms, tot = timed(b, fn, args.batch_reps)
        out[name] = dict(ms=ms * 1e3, queries_per_s=nq / ms, ids=tot)
        if name == "batched_graph":
            chunks, over = b.replay_info()
            out[name]["replay"] = {"record_chunks": chunks, "overflowed": over, "replayed": bool(chunks and not over)}
    if not args.batch_tuned_only:
        # the same graph with the walking fill (second traversal), for reference
        b.set_replay(False)
        ms, tot = timed(b, b.run, args.batch_reps)
        out["batched_graph_walking_fill"] = dict(ms=ms * 1e3, queries_per_s=nq / ms, ids=tot)
        b.set_replay(True)
    if args.batch_tuned_only:
        b.free()
        for t in trees:
            t.free()
        out["size_class_choice"] = {str(k): {kk: v[kk] for kk in ("fanout", "layout", "trees")}
                                    for k, v in choice.items()}
        return out
    # byte model over all trees (same traversal with counters)
    vn = ve = vc = 0
    tree_bytes = 0
    for t, x in zip(trees, inst):
        a_, b_, c_ = rt.visit_stats(t, x.queries)
        vn, ve, vc = vn + a_, ve + b_, vc + c_
        tree_bytes += int(t.info().device_bytes)
    ids = out["batched_graph"]["ids"]
    visit_fill = 16 * nq + 20 * ve + 8 * vn + 4 * ids + 4 * vc + 8 * (nq + 1)
    comp_fill = 16 * nq + tree_bytes + 8 * (nq + 1) + 4 * ids
    rep = out["batched_graph"].get("replay", {})
    if rep.get("replayed"):   # the graph's fill replays the count pass's records
        rb = 16 * 256 * rep["record_chunks"]
        visit_fill = rb + 8 * (nq + 1) + 8 * ids
        comp_fill = rb + 8 * (nq + 1) + 4 * ids + min(tree_bytes, 4 * ids)
    b.free()
    # the library's own per-tree choice (fanout 0, RT_LAYOUT_AUTO: probe
    # windows drawn from each tree's data, not the batch's windows)
    lt = [rt.build_str(x.rects, 0, "auto") for x in inst]
    bl = rt.Batch(lt, [x.queries for x in inst])
    ms, tot = timed(bl, bl.run, args.batch_reps)
    assert tot == out["batched_graph"]["ids"]
    out["batched_graph_library_choice"] = dict(ms=ms * 1e3, queries_per_s=nq / ms, ids=tot)
    bl.free()
    for t in lt:
        t.free()
    g = out["batched_graph"]["ms"]
    out["speedup_vs_plain"] = out["plain_per_tree"]["ms"] / g
    out.update(workload=f"batch_{len(inst)}_trees_{sum(x.rects.shape[0] for x in inst)}_rects_{nq}_windows",
               configs=cfg, size_class_choice={str(k): {kk: v[kk] for kk in ("fanout", "layout", "trees")}
                                               for k, v in choice.items()},
               tune_s=tune_s, gen_s=gen_s, build_s=build_s, tree_bytes=tree_bytes,
               visited={"nodes": vn, "entries": ve, "ids_from_contained_subtrees": vc},
               bytes_model={"visit_fill": visit_fill, "compulsory_fill": comp_fill},
               effective_GBps=visit_fill / (g / 1e3) / 1e9)
    tr = read_traffic(f"batch_c4_{args.batch_trees}")
    if "batch" in tr:
        out["fill_kernel_traffic"] = {"bytes": tr["batch"], "kernel_ms": tr["batch_ms"], "file": tr["file"],
                                      "hbm_frac": tr["batch"] / (tr["batch_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS}
    for t in trees:
        t.free()
    if not args.batch_untuned:
        return out
    # plain launches on untuned trees (the baseline without autotuning)
    ut = [rt.build_str(x.rects, 32, "soa") for x in inst]
    bu = rt.Batch(ut, [x.queries for x in inst])
    ms, tot = timed(bu, bu.run_plain, args.batch_reps)
    assert tot == ids
    out["plain_per_tree_untuned_f32_soa"] = dict(ms=ms * 1e3, queries_per_s=nq / ms, ids=tot)
    ms, tot = timed(bu, bu.run, args.batch_reps)
    out["batched_graph_untuned_f32_soa"] = dict(ms=ms * 1e3, queries_per_s=nq / ms, ids=tot)
    bu.free()
    for t in ut:
        t.free()
    out["speedup_vs_plain_untuned"] = out["plain_per_tree_untuned_f32_soa"]["ms"] / g
    return out


def serve_leg(rt, torch, args, tb, tj):
    from paper_2309_16913_amd.serve import Server
    import rtgen
    info = tb.info()
    out = {"workload": f"serve_clustered{args.serve_n}_f32_soa_plus_uniform{args.serve_join_n}_joins",
           "tree_bytes": info.device_bytes, "tree_height": info.height,
           "requests_per_rate": args.serve_requests, "warmup_requests": args.serve_warmup,
           "open_loop": [], "note": "latency = result in pinned host memory - scheduled arrival"}
    srv = Server(tb, tj, nslots=args.serve_slots, max_windows=args.serve_max_windows, pool_ids=args.serve_pool)
    warm = rtgen.c5_requests(args.serve_warmup, rate=1e6, seed_base=5900, probe_n=10_000)
    srv.run(warm)
    for rate in args.serve_rates:
        reqs = rtgen.c5_requests(args.serve_requests, rate=rate, seed_base=5000 + int(np.log10(rate) * 10),
                                 probe_n=10_000)
        log(f"[bench] serve open loop {rate:g}/s")
        r = srv.run(reqs)
        r["offered_rate"] = rate
        out["open_loop"].append(r)
        del reqs
    # closed loop: every request is waiting at t = 0 (saturation throughput)
    reqs = rtgen.c5_requests(args.serve_requests, rate=1e12, seed_base=5000, probe_n=10_000)
    log("[bench] serve closed loop")
    r = srv.run(reqs)
    sel = np.concatenate([q.payload for q in reqs if q.kind == "select"])
    vn, ve, vc = rt.visit_stats(tb, sel)
    bytes_ = 16 * sel.shape[0] + 20 * ve + 8 * vn + 4 * vc
    for q in reqs:
        if q.kind == "join":
            a, b_, c_ = rt.visit_stats(tj, q.payload)
            bytes_ += 16 * q.payload.shape[0] + 20 * b_ + 8 * a + 4 * c_
    bytes_ += 4 * r["ids"] + 8 * r["batches"]
    r["algorithmic_bytes"] = bytes_
    r["effective_GBps"] = bytes_ / r["wall_s"] / 1e9
    r["pcie_GBps"] = 4 * r["ids"] / r["wall_s"] / 1e9
    out["closed_loop"] = r
    del reqs, sel, srv
    torch.cuda.empty_cache()
    # unbatched baseline: one request per launch, one stream
    base = Server(tb, tj, nslots=1, max_windows=16384, pool_ids=1 << 27, one_per_batch=True)
    reqs = rtgen.c5_requests(min(args.serve_requests, 4000), rate=1e12, seed_base=5000, probe_n=10_000)
    log("[bench] serve unbatched baseline")
    rb = base.run(reqs)
    out["unbatched_closed_loop"] = rb
    out["speedup_vs_unbatched"] = (r["throughput_req_per_s"] / rb["throughput_req_per_s"]
                                   if rb["throughput_req_per_s"] else None)
    return out


def serve_device_leg(rt, torch, ev, args, tb):
    """Closed loop without the host: the served window mix (selectivity
    log-uniform in [1e-7, 1e-2]) against the resident 50M-rectangle tree as
    one device select, results left in HBM (the tree is four times the
    Infinity Cache, so its nodes come from DRAM)."""
    import rtgen
    q = rtgen.windows_loguniform(args.serve_device_windows, 1e-7, 1e-2, 5006)
    nq = q.shape[0]
    dq = torch.from_numpy(q).cuda()
    s = torch.cuda.current_stream()
    off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    wb0 = rt.select_workspace_bytes(nq, 0)
    w0 = torch.empty(wb0, dtype=torch.uint8, device="cuda")
    rt.range_select_device_count(tb, dq.data_ptr(), nq, off.data_ptr(), w0.data_ptr(), wb0, s.cuda_stream)
    cap = int(off[nq].item())
    del w0
    ids = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    wb = (rt.select_replay_workspace_bytes if args.replay else rt.select_workspace_bytes)(nq, cap)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    st = torch.zeros(2, dtype=torch.int64, device="cuda")
    evs = [ev.create(5) for _ in range(args.serve_device_reps)]
    rt.range_select_device_timed(tb, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), cap, work.data_ptr(), wb,
                                 st.data_ptr(), s.cuda_stream, None)
    for e in evs:
        rt.range_select_device_timed(tb, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), cap, work.data_ptr(),
                                     wb, st.data_ptr(), s.cuda_stream, e)
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [cap, 0]
    rec_chunks, rec_over = rt.select_replay_info(work.data_ptr())
    ph = {k: float(np.mean([ev.ms(e[a], e[b]) for e in evs]))
          for k, (a, b) in {"count": (0, 1), "scan": (1, 2), "fill": (2, 3), "sort": (3, 4)}.items()}
    step = float(np.mean([ev.ms(e[0], e[4]) for e in evs]))
    vn, ve, vc = rt.visit_stats(tb, q)
    info = tb.info()
    visit_fill = 16 * nq + 20 * ve + 8 * vn + 4 * cap + 4 * vc + 8 * (nq + 1)
    comp_fill = 16 * nq + int(info.device_bytes) + 8 * (nq + 1) + 4 * cap
    if args.replay and rec_chunks and not rec_over:   # the fill replays the count pass's records
        rb = 16 * 256 * rec_chunks
        visit_fill = rb + 8 * (nq + 1) + 8 * cap
        comp_fill = rb + 8 * (nq + 1) + 4 * cap + min(int(info.device_bytes), 4 * cap)
    tr = read_traffic(f"select_serve50m_w{nq}")
    out = {"workload": f"select_clustered{info.n_objects}_f{info.fanout}_soa_windows{nq}_device",
           "windows": nq, "ids": cap, "ms_per_select": step, "phases_ms": ph,
           "replay": {"record_chunks": rec_chunks, "overflowed": rec_over,
                      "replayed": bool(args.replay and rec_chunks and not rec_over)},
           "queries_per_s": nq / (step / 1e3), "ids_per_s": cap / (step / 1e3),
           "visited": {"nodes": vn, "entries": ve, "ids_from_contained_subtrees": vc},
           "roofline_fill": roofline_entry("select_kernel (fill pass)", ph["fill"], comp_fill, visit_fill,
                                           tr.get("fill"))}
    if "count" in tr:
        out["count_traffic_frac"] = tr["count"] / (ph["count"] / 1e3) / 1e9 / HBM_PEAK_GBS
    if "sort" in tr:
        out["sort_traffic_frac"] = tr["sort"] / (ph["sort"] / 1e3) / 1e9 / HBM_PEAK_GBS
    del ids, work
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--nq", type=int, default=1_000_000)
    ap.add_argument("--fanout", type=int, default=32)
    ap.add_argument("--layout", default="soa")
    ap.add_argument("--legs", default="select,build,join,batch,serve,serve_device,cpu")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first of all, copy this many MiB device-to-device three times (a plain copy of known "
                         "size, used to scale rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="time --fanout/--layout directly instead of the autotuner's choice")
    ap.add_argument("--no-lookahead", dest="lookahead", action="store_false")
    ap.add_argument("--no-replay", dest="replay", action="store_false",
                    help="workspace without room for the count pass's records (the fill walks the tree again)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--join-n", type=int, default=2_000_000)
    ap.add_argument("--join-reps", type=int, default=5)
    ap.add_argument("--join-fanout", type=int, default=32)
    ap.add_argument("--batch-trees", type=int, default=256)
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--no-batch-untuned", dest="batch_untuned", action="store_false",
                    help="skip the untuned (fanout 32, SoA) baselines of the batch leg")
    ap.add_argument("--serve-n", type=int, default=50_000_000)
    ap.add_argument("--serve-join-n", type=int, default=5_000_000)
    ap.add_argument("--serve-requests", type=int, default=200_000)
    ap.add_argument("--serve-warmup", type=int, default=10_000)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-pool", type=int, default=1 << 29)
    ap.add_argument("--serve-max-windows", type=int, default=65536)
    ap.add_argument("--serve-rates", type=float, nargs="*", default=SERVE_RATES)
    ap.add_argument("--serve-device-windows", type=int, default=50_000)
    ap.add_argument("--serve-device-reps", type=int, default=3)
    # counter summaries (host only)
    ap.add_argument("--pmc-summary", action="store_true")
    ap.add_argument("--pmc-table", action="store_true")
    ap.add_argument("--stats-table", action="store_true")
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--kernel-regex", default="")
    ap.add_argument("--fetch-dir")
    ap.add_argument("--write-dir")
    ap.add_argument("--tag")
    ap.add_argument("--title", default="")
    ap.add_argument("--bench-args", default="")
    ap.add_argument("--steps-in-run", type=int, default=1)
    ap.add_argument("--last", type=int, default=0, help="average only the last N launches of each phase")
    ap.add_argument("--batch-tuned-only", action="store_true",
                    help="batch leg: after tuning, time only the tuned batch (for counter runs)")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args)
        return
    if args.pmc_table:
        pmc_table(args)
        return
    if args.stats_table:
        stats_table(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    import paper_2309_16913_amd as rt
    import rtgen
    ev = HipEvents()
    legs = set(x for x in args.legs.split(",") if x)

    if args.calib_copy_mib:
        nb = args.calib_copy_mib << 20
        a = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: 3 x {nb} bytes")
        del a, b
    result = {"metric": METRIC, "value": None, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": {}, "legs": {}}
    rects = queries = None
    s = None
    if "select" in legs or "cpu" in legs or "build" in legs:
        log(f"[bench] generating {args.n} rectangles and {args.nq} windows")
        rects = rtgen.c2_rects(args.n)
        queries = rtgen.c2_queries(args.nq)
    if "select" in legs:
        tune = None
        kmin = 0
        if args.autotune:
            from paper_2309_16913_amd.autotune import Autotuner
            log("[bench] autotuning fanout x layout x mapping on the full workload")
            tuner = Autotuner(cache_path=None, fanouts=(16, 32, 64), layouts=("aos", "soa", "d2"), kmins=(0, 16),
                              sample=args.nq, reps=2, replay=args.replay)
            tune = tuner.tune(rects, queries, "mixed")
            args.fanout, args.layout, kmin = tune["fanout"], tune["layout"], tune["kmin"]
        log(f"[bench] select leg (fanout {args.fanout}, {args.layout}, split kmin {kmin})")
        s = select_leg(rt, torch, ev, args, rects, queries, kmin)
        ms_step = s["wall"] / args.steps * 1e3
        tr = read_traffic(f"select_c2_f{args.fanout}_{args.layout}")
        dom = max(("count", "fill"), key=lambda k: s["avg"][k])
        result.update(
            value=args.nq / (s["wall"] / args.steps), ms_per_step=ms_step,
            config={"workload": f"select_mixed{args.n}_windows{args.nq}_f{args.fanout}_{args.layout}",
                    "n_rects": args.n, "n_queries": args.nq, "fanout": args.fanout, "layout": args.layout,
                    "split_kmin": kmin, "selectivity": "loguniform[1e-6,1e-3]", "ids_out": s["cap"]},
            variants_ms=tune["timings_ms"] if tune else None,
            roofline=roofline_entry(f"select_kernel ({dom} pass)", s["avg"][dom], s["comp"][dom], s["visit"][dom],
                                    tr.get(dom)),
            phases_ms=s["avg"],
            phases_roofline={ph: roofline_entry(ph, s["avg"][ph], s["comp"][ph], s["visit"][ph], tr.get(ph))
                             for ph in ("count", "fill", "sort")},
            traffic_profile=tr.get("file"),
            lookahead_ms=s["lookahead"],
            replay=s["replay"],
            tree={"height": s["info"].height, "nodes": s["info"].n_nodes, "device_bytes": s["info"].device_bytes,
                  "build_s": s["build_s"]},
            visited={"nodes": s["vn"], "entries": s["ve"], "ids_from_contained_subtrees": s["vc"]})
        if tr.get(dom + "_ms") == tr.get(dom + "_ms"):   # not NaN
            result["roofline"]["profile_kernel_ms"] = tr.get(dom + "_ms")
    gpu_off = gpu_ids = None
    if s is not None:
        if "cpu" in legs:
            gpu_off = s["off"].cpu().numpy()
            gpu_ids = s["ids"].cpu().numpy()
        del s
        torch.cuda.empty_cache()
    if "build" in legs:
        log("[bench] build leg")
        result["legs"]["build"] = build_leg(rt, torch, args, rects)
        torch.cuda.empty_cache()
    join_check = None
    if "join" in legs:
        log("[bench] join leg")
        jl, pairs, rel = join_leg(rt, torch, args)
        result["legs"]["join"] = jl
        join_check = (rel[0], rel[1], pairs)
        torch.cuda.empty_cache()
    if "batch" in legs:
        log("[bench] batch leg")
        result["legs"]["batch"] = batch_leg(rt, torch, args)
        torch.cuda.empty_cache()
    if "serve" in legs or "serve_device" in legs:
        t0 = time.time()
        big, jt = rtgen.c5_trees(args.serve_n, args.serve_join_n if "serve" in legs else 1)
        gen_s = time.time() - t0
        t0 = time.time()
        tb = rt.build_str(big, 32, "soa")
        tj = rt.build_str(jt, 32, "soa")
        build_s = time.time() - t0
        del big, jt
        if "serve_device" in legs:
            log("[bench] serve device-side closed loop")
            tb.set_split(16)
            result["legs"]["serve_device"] = serve_device_leg(rt, torch, ev, args, tb)
        if "serve" in legs:
            log("[bench] serve leg")
            sv = serve_leg(rt, torch, args, tb, tj)
            sv.update(gen_s=gen_s, build_s=build_s)
            result["legs"]["serve"] = sv
            result["p99_ms"] = {str(int(x["offered_rate"])): x["select_p99_ms"] for x in sv["open_loop"]
                                if x.get("select_p99_ms") is not None}
        tb.free()
        tj.free()
        torch.cuda.empty_cache()
    if "cpu" in legs and gpu_off is not None:
        log("[bench] cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(args, rects, queries, gpu_off, gpu_ids, join_check)
        if join_check is not None:
            result["legs"]["join"]["checked_against_oracle"] = result["cpu_baseline"]["join"]["gpu_pairs_equal_oracle"]
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
