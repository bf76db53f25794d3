#!/usr/bin/env python3
"""Benchmark: batched R-tree range select (and join / batched / served legs)
on one MI355X.

Default workload (the "step"): one complete range select -- count pass,
scan, fill pass, segmented sort -- of 1,000,000 query windows (selectivity
log-uniform in [1e-6, 1e-3]) against a 10,000,000-rectangle tree (half
uniform, half in 64 Gaussian clusters, sides U[0, 1e-4]), fanout 32, SoA
node layout, with queries, tree and output buffers resident in device memory
before timing starts.  Prints one JSON line.

Extra legs (same JSON line, under "legs"): spatial join of two 2M-rectangle
relations, the 256-instance batched select (persistent + graph vs plain
per-tree launches), and the scalar CPU oracle timed on a bounded sample of the
same select workload ("cpu_baseline").
"""

from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "range queries/s and join pairs/s on 1 GPU (bit-exact), % HBM peak; p99 latency"


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

    def create(self, n):
        out = []
        for _ in range(n):
            e = C.c_void_p()
            assert self.h.hipEventCreate(C.byref(e)) == 0
            out.append(e.value)
        return out

    def ms(self, a, b):
        f = C.c_float()
        assert self.h.hipEventSynchronize(C.c_void_p(b)) == 0
        assert self.h.hipEventElapsedTime(C.byref(f), C.c_void_p(a), C.c_void_p(b)) == 0
        return float(f.value)


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2309_16913_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_tag, src_hash):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.txt")
    if not os.path.exists(p):
        return None
    vals = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != src_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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
    del work0
    ids = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    wb = rt.select_workspace_bytes(nq, cap)
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
    # the lookahead variant (loads one node ahead after each leaf), timed the
    # same way on the same buffers, then switched off again
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
    node_bytes = 20 * ve + 8 * vn
    bytes_count = 16 * nq + node_bytes
    # fill: the same walk, the ids written, and the id arrays of the leaves of
    # subtrees that lie inside their window (copied without comparisons)
    bytes_fill = bytes_count + 4 * cap + 4 * vc + 8 * (nq + 1)
    return dict(tree=tree, info=info, build_s=build_s, cap=cap, wall=wall, avg=avg, vn=vn, ve=ve, vc=vc,
                bytes_count=bytes_count, bytes_fill=bytes_fill, off=off, ids=ids, lookahead=lookahead)


def cpu_baseline(args, rects, queries, gpu_off, gpu_ids):
    import oracle
    o = oracle.get()
    t0 = time.time()
    ot = o.build_str(rects, args.fanout)
    build_s = time.time() - t0
    done, spent, chunk = 0, 0.0, 2000
    mismatches = 0
    while spent < args.cpu_seconds and done < queries.shape[0]:
        q = queries[done:done + chunk]
        t0 = time.perf_counter()
        woff, wids = o.select(ot, q)
        spent += time.perf_counter() - t0
        # bit-exact check of the GPU result on this sample
        g0, g1 = int(gpu_off[done]), int(gpu_off[done + q.shape[0]])
        goff = gpu_off[done:done + q.shape[0] + 1] - g0
        if not (np.array_equal(goff, woff.astype(np.int64)) and
                np.array_equal(gpu_ids[g0:g1].view(np.uint32), wids)):
            mismatches += 1
        done += q.shape[0]
    return dict(value=done / spent, unit="queries/s", cores=1, kind="oracle",
                sample=f"first {done} of the {queries.shape[0]} windows against the "
                       f"{rects.shape[0]}-rectangle tree (fanout {args.fanout}), query phase only, "
                       f"single thread; oracle STR build {build_s:.1f} s not included",
                checked_queries=done, mismatching_chunks=mismatches)


def join_leg(rt, torch, args):
    """C3 join (2M uniform x 2M clustered at full size).  Trees are built on
    the device with every node sorted by low x; the headline variant is the
    library default on such trees (O3 outer slicing + O5 many-to-many inner
    shrinking + the LB lower bound on the inner scan).  Times are for the device-output call (pairs left in HBM);
    the host-output call (pairs copied over PCIe) is reported beside it, and
    every variant of section 4 is timed on the same trees."""
    import rtgen
    a, b = rtgen.c3_join(args.join_n)
    F = args.join_fanout
    ta = rt.build_str(a, F, "soa", sort_lx=True)
    tb = rt.build_str(b, F, "soa", sort_lx=True)
    n = rt.spatial_join_device(ta, tb, 0, 0)
    buf = torch.empty(2 * max(n, 1), dtype=torch.int32, device="cuda")

    def time_dev(flags):
        rt.spatial_join_device(ta, tb, buf.data_ptr(), n, flags)   # warm
        ts = []
        for _ in range(args.join_reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            got = rt.spatial_join_device(ta, tb, buf.data_ptr(), n, flags)
            ts.append(time.perf_counter() - t0)
            assert got == n
        return float(np.median(ts)) * 1e3

    ms = time_dev(None)
    hts = []
    for _ in range(args.join_reps):
        t0 = time.perf_counter()
        p = rt.spatial_join(ta, tb)
        hts.append(time.perf_counter() - t0)
    assert p.shape[0] == n
    variants = {}
    for name, fl in [("tile", rt.JOIN_TILE), ("cand", 0), ("O3", rt.JOIN_O3), ("O3+O4", rt.JOIN_O3 | rt.JOIN_O4),
                     ("O3+O5", rt.JOIN_O3 | rt.JOIN_O5), ("O5", rt.JOIN_O5),
                     ("O3+O5+LB", rt.JOIN_O3 | rt.JOIN_O5 | rt.JOIN_LB)]:
        _, tests = rt.spatial_join(ta, tb, fl, with_tests=True)
        variants[name] = dict(ms=round(time_dev(fl), 4), predicate_tests=tests)
    return dict(workload=f"join_uniform{args.join_n}_x_clustered{args.join_n}_f{F}_soa_sorted_lx", pairs=int(n),
                ms=ms, pairs_per_s=n / (ms / 1e3), host_output_ms=float(np.median(hts)) * 1e3,
                variants_ms=variants,
                note="device-output call, synchronous; includes the final key-count read on the host and the sort")


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
    return out


def batch_leg(rt, torch, args):
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

    # autotune fanout x layout in batch context on a subset of the instances
    # (the persistent kernel serves every tree with its own configuration,
    # but one configuration for the whole batch keeps its waves uniform)
    sub = inst[:: max(1, len(inst) // args.batch_tune_subset)]
    tune = {}
    for F in (16, 32, 64):
        for lay in ("aos", "soa"):
            ts = [rt.build_str(x.rects, F, lay) for x in sub]
            b = rt.Batch(ts, [x.queries for x in sub])
            tune[f"{F}/{lay}"] = timed(b, b.run, 2)[0] * 1e3
            b.free()
            for t in ts:
                t.free()
    best = min(tune, key=tune.get)
    F, lay = best.split("/")
    t0 = time.time()
    trees = [rt.build_str(x.rects, int(F), lay) for x in inst]
    build_s = time.time() - t0
    b = rt.Batch(trees, [x.queries for x in inst])
    out = {}
    for name, fn in (("batched_graph", b.run), ("plain_per_tree", b.run_plain)):
        ms, tot = timed(b, fn, args.batch_reps)
        out[name] = dict(ms=ms * 1e3, queries_per_s=nq / ms, ids=tot)
    out["speedup"] = out["plain_per_tree"]["ms"] / out["batched_graph"]["ms"]
    out.update(workload=f"batch_{len(inst)}_trees_{sum(x.rects.shape[0] for x in inst)}_rects_{nq}_windows",
               fanout=int(F), layout=lay, tune_subset_ms=tune, gen_s=gen_s, build_s=build_s)
    return out


def serve_leg(rt, torch, args):
    import rtgen
    from paper_2309_16913_amd.serve import Server
    t0 = time.time()
    big, jt = rtgen.c5_trees(args.serve_n, args.serve_join_n)
    gen_s = time.time() - t0
    t0 = time.time()
    tb = rt.build_str(big, 32, "soa")
    tj = rt.build_str(jt, 32, "soa")
    build_s = time.time() - t0
    del big, jt
    info = tb.info()
    out = {"workload": f"serve_clustered{args.serve_n}_f32_soa_plus_uniform{args.serve_join_n}_joins",
           "gen_s": gen_s, "build_s": build_s, "tree_bytes": info.device_bytes, "tree_height": info.height,
           "open_loop": [], "note": "latency = result in pinned host memory - scheduled arrival"}
    srv = Server(tb, tj, nslots=3, max_windows=16384, pool_ids=1 << 27)
    warm = rtgen.c5_requests(2000, rate=1e6, seed_base=5900, probe_n=10_000)
    srv.run(warm)
    for rate in args.serve_rates:
        reqs = rtgen.c5_requests(args.serve_requests, rate=rate, seed_base=5000, probe_n=10_000)
        log(f"[bench] serve open loop {rate:g}/s")
        r = srv.run(reqs)
        r["offered_rate"] = rate
        out["open_loop"].append(r)
    # closed loop: every request is waiting at t = 0 (saturation throughput)
    reqs = rtgen.c5_requests(args.serve_requests, rate=1e12, seed_base=5000, probe_n=10_000)
    log("[bench] serve closed loop")
    r = srv.run(reqs)
    sel = np.concatenate([q.payload for q in reqs if q.kind == "select"])
    probes = [q.payload for q in reqs if q.kind == "join"]
    vn, ve, vc = rt.visit_stats(tb, sel)
    bytes_ = 16 * sel.shape[0] + 20 * ve + 8 * vn + 4 * vc
    for p_ in probes:
        a, b_, c_ = rt.visit_stats(tj, p_)
        bytes_ += 16 * p_.shape[0] + 20 * b_ + 8 * a + 4 * c_
    bytes_ += 4 * r["ids"] + 8 * r["batches"]
    r["algorithmic_bytes"] = bytes_
    r["algorithmic_GBps"] = bytes_ / r["wall_s"] / 1e9
    r["hbm_frac"] = r["algorithmic_GBps"] / HBM_PEAK_GBS
    out["closed_loop"] = r
    # unbatched baseline: one request per launch, one stream
    base = Server(tb, tj, nslots=1, max_windows=16384, pool_ids=1 << 27, one_per_batch=True)
    reqs = rtgen.c5_requests(min(args.serve_requests, 4000), rate=1e12, seed_base=5000, probe_n=10_000)
    log("[bench] serve unbatched baseline")
    rb = base.run(reqs)
    out["unbatched_closed_loop"] = rb
    out["speedup_vs_unbatched"] = (r["throughput_req_per_s"] / rb["throughput_req_per_s"]
                                   if rb["throughput_req_per_s"] else None)
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
    ap.add_argument("--legs", default="build,join,batch,serve,cpu")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the select leg, copy this many MiB device-to-device three times (a plain copy "
                         "kernel of known size, used to scale rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="time --fanout/--layout directly instead of the autotuner's choice")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--join-n", type=int, default=2_000_000)
    ap.add_argument("--join-reps", type=int, default=5)
    ap.add_argument("--join-fanout", type=int, default=32)
    ap.add_argument("--batch-trees", type=int, default=256)
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--batch-tune-subset", type=int, default=64)
    ap.add_argument("--serve-n", type=int, default=50_000_000)
    ap.add_argument("--serve-join-n", type=int, default=5_000_000)
    ap.add_argument("--serve-requests", type=int, default=20_000)
    ap.add_argument("--serve-rates", type=float, nargs="*", default=[1e4, 1e5, 1e6])
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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
    log(f"[bench] generating {args.n} rectangles and {args.nq} windows")
    rects = rtgen.c2_rects(args.n)
    queries = rtgen.c2_queries(args.nq)
    tune = None
    kmin = 0
    if args.autotune:
        from paper_2309_16913_amd.autotune import Autotuner
        log("[bench] autotuning fanout x layout x mapping on the full workload")
        tuner = Autotuner(cache_path=None, fanouts=(16, 32, 64), layouts=("aos", "soa"), kmins=(0, 16),
                          sample=args.nq, reps=2)
        tune = tuner.tune(rects, queries, "mixed")
        args.fanout, args.layout, kmin = tune["fanout"], tune["layout"], tune["kmin"]
    log(f"[bench] select leg (fanout {args.fanout}, {args.layout}, split kmin {kmin})")
    s = select_leg(rt, torch, ev, args, rects, queries, kmin)
    ms_step = s["wall"] / args.steps * 1e3
    qps = args.nq / (s["wall"] / args.steps)
    dom = "fill" if s["avg"]["fill"] >= s["avg"]["count"] else "count"
    dom_bytes = s["bytes_fill"] if dom == "fill" else s["bytes_count"]
    achieved = dom_bytes / (s["avg"][dom] / 1e3) / 1e9
    src = source_hash("select.hip", "rt_internal.h")
    traffic = read_traffic(f"select_{dom}_c2_f{args.fanout}_{args.layout}", src)
    result = {
        "metric": METRIC, "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"select_mixed{args.n}_windows{args.nq}_f{args.fanout}_{args.layout}",
                   "n_rects": args.n, "n_queries": args.nq, "fanout": args.fanout, "layout": args.layout,
                   "split_kmin": kmin, "selectivity": "loguniform[1e-6,1e-3]", "ids_out": s["cap"]},
        "variants_ms": tune["timings_ms"] if tune else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"select_kernel ({dom} pass)", "algorithmic_bytes_per_launch": dom_bytes},
        "phases_ms": s["avg"],
        "lookahead_ms": s["lookahead"],
        "tree": {"height": s["info"].height, "nodes": s["info"].n_nodes,
                 "device_bytes": s["info"].device_bytes, "build_s": s["build_s"]},
        "visited": {"nodes": s["vn"], "entries": s["ve"], "ids_from_contained_subtrees": s["vc"]},
        "legs": {},
    }
    if "cpu" in legs:
        log("[bench] cpu baseline (oracle)")
        goff = s["off"].cpu().numpy()
        gids = s["ids"].cpu().numpy()
        result["cpu_baseline"] = cpu_baseline(args, rects, queries, goff, gids)
    del s
    torch.cuda.empty_cache()
    if "build" in legs:
        log("[bench] build leg")
        result["legs"]["build"] = build_leg(rt, torch, args, rects)
        torch.cuda.empty_cache()
    if "join" in legs:
        log("[bench] join leg")
        result["legs"]["join"] = join_leg(rt, torch, args)
        torch.cuda.empty_cache()
    if "batch" in legs:
        log("[bench] batch leg")
        result["legs"]["batch"] = batch_leg(rt, torch, args)
        torch.cuda.empty_cache()
    if "serve" in legs:
        log("[bench] serve leg")
        sv = serve_leg(rt, torch, args)
        result["legs"]["serve"] = sv
        ol = [x for x in sv["open_loop"] if x.get("select_p99_ms") is not None]
        if ol:
            result["p99_ms"] = {str(int(x["offered_rate"])): x["select_p99_ms"] for x in ol}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
