#!/usr/bin/env python3
"""Benchmark of batched isochrone queries on the 18M-vertex synthetic road graph.

One step = one sweep over a batch of `--lanes` queries (source, tau) in the
cell-restricted mode: host upward searches, core sweep with cell flags,
active-cell selection, per-cell sweeps with isochrone-edge extraction, radix
sort and decode of the edges.  The timed region is one iso_query_batch_device
call over `--steps` batches (consecutive sweeps overlap on two streams): the
graph is resident in HBM and the edges stay there, in torch-allocated device
buffers.  The same work through iso_query_batch, which copies the edges to host
memory over PCIe, is reported beside it (host_api_qps).  Also reported:
single-query latency p50/p99 (both sweep modes), the plain-sweep batched
throughput, latency percentiles of the serving loop under Poisson arrivals at
several offered rates, the live roofline of the dominant kernel phase (HIP
events on the sweep streams over the timed region, algorithmic bytes from the
graph structure), and the CPU oracle timed on this host.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload road18m]
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "isochrone queries/s + p50/p99 ms on 18M-vertex graph; sweep HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def load_workload(name, cache_dir):
    import paper_1512_09090_amd as iso
    import synth

    cfg = synth.CONFIGS[name]
    t0 = time.time()
    g = synth.config_graph(name)
    log(f"graph {name}: n={g.n} m={g.m} ({time.time() - t0:.1f}s)")
    os.makedirs(cache_dir, exist_ok=True)
    prep = os.path.join(cache_dir, f"{name}-c{cfg['cells']}-v1.prep")
    t0 = time.time()
    G = iso.Graph.from_synth(g, num_cells=cfg["cells"], device=0, prep_path=prep, verbose=True)
    log(f"loaded on device ({time.time() - t0:.1f}s): {G.info()}")
    return g, G


def run_batches(G, src, tau, lanes, steps, mode, start=0):
    n = len(src)
    times = []
    for i in range(steps):
        b = (start + i * lanes) % n
        idx = (np.arange(lanes) + b) % n
        t0 = time.perf_counter()
        G.query_batch(src[idx], tau[idx], mode)
        times.append(time.perf_counter() - t0)
    return times


class DeviceBatches:
    """Runs iso_query_batch_device over a query list into torch buffers kept between calls
    (grown when a call reports ISO_ESPACE)."""

    def __init__(self, iso, G, per_query_hint):
        import torch
        self.iso, self.G, self.torch = iso, G, torch
        self.hint = per_query_hint
        self.pairs = self.offsets = None

    def reserve(self, k):
        torch = self.torch
        if self.offsets is None or self.offsets.numel() < k + 1:
            self.offsets = torch.empty(k + 1, dtype=torch.int32, device="cuda:0")
        if self.pairs is None or self.pairs.shape[0] < self.hint * k:
            self.pairs = None
            self.pairs = torch.empty((int(self.hint * k), 2), dtype=torch.int32, device="cuda:0")

    def run(self, src, tau, mode):
        torch = self.torch
        k = len(src)
        self.reserve(k)
        try:
            return self.G.query_batch_device(src, tau, mode, self.pairs, self.offsets[:k + 1])
        except self.iso.IsoError as e:
            if e.code != self.iso.ISO_ESPACE:
                raise
            log(f"device result buffer: {self.pairs.shape[0]} pairs, need {e.total}; growing")
            self.hint = max(self.hint, 1.25 * e.total / max(1, k))
            self.pairs = None
            torch.cuda.empty_cache()
            self.pairs = torch.empty((int(self.hint * k), 2), dtype=torch.int32, device="cuda:0")
            return self.G.query_batch_device(src, tau, mode, self.pairs, self.offsets[:k + 1])


def serving(G, n, rates, duration, lanes, inflight, warm=1.0):
    """Poisson arrivals at each offered rate through the continuous-batching server
    (iso_server_*): submit at the trace's arrival times, collect every result, report the
    completed rate and the per-request latency (submit to result ready) p50/p99."""
    import queue

    import paper_1512_09090_amd as iso
    import synth

    out = []
    for rate in rates:
        t, src, tau = synth.serving_trace(n, rate, duration + warm, seed=15)
        srv = iso.Server(G, max_lanes=lanes, max_inflight=inflight, mode=iso.MODE_CELLS)
        q = queue.Queue()
        lat, batch, done_at = [], [], [0.0]

        def collect():
            while True:
                item = q.get()
                if item is None:
                    return
                tk, counted = item
                _, st = srv.wait(tk)
                if counted:
                    lat.append(st["t_total_ms"])
                    batch.append(st["batch_lanes"])
                done_at[0] = time.perf_counter()

        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        backlog = 0
        try:
            for i in range(len(t)):
                dt = t0 + t[i] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                q.put((srv.submit(int(src[i]), int(tau[i])), t[i] >= warm))
            t_sub = time.perf_counter() - t0
            backlog = srv.stats()["queue_depth"]   # requests still waiting for a sweep when the trace ends
        finally:
            q.put(None)
            th.join()
            stats = srv.stats()
            srv.close()
        span = max(done_at[0] - (t0 + warm), 1e-9)
        r = {"offered_hz": rate, "submitted_hz": round((len(t) - int(np.sum(t < warm))) / max(t_sub - warm, 1e-9), 1),
             "requests": len(lat), "completed_qps": round(len(lat) / span, 1),
             "p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
             "mean_batch": round(float(np.mean(batch)), 2), "sweeps": stats["sweeps"],
             "backlog_at_end": int(backlog)}
        log(f"serving {r}")
        out.append(r)
    return out


def copy_probe(mib):
    """A device-to-device copy of `mib` MiB, three times (torch's same-device copy is the HIP
    runtime's copy kernel): it reads and writes a known number of bytes, which calibrates the
    HBM byte counters of a profiler run."""
    import torch

    a = torch.ones((int(mib) << 20) // 4, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    log(f"copy probe: 3 x {mib} MiB device-to-device")


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "road18m_hbm_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1512_09090_amd", "csrc", "sweep.hip")


def kernel_source_sha():
    """sha256 of the device code: the kernel source up to its host-side section."""
    import hashlib

    text = open(KERNEL_SOURCE, "rb").read()
    cut = text.find(b"// ----------------------------------------------------------------- host side")
    return hashlib.sha256(text if cut < 0 else text[:cut]).hexdigest()


def measured_traffic(phase):
    """HBM bytes per launch of a phase from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE passes, scaled by a copy of known size), or None when the summary is missing or
    was taken on another version of the kernel source."""
    import hashlib

    try:
        text = open(TRAFFIC_SUMMARY).read()
        sha = kernel_source_sha()
    except OSError:
        return None
    vals = dict(line.split(":", 1) for line in text.splitlines()
                if line.startswith(("device_code_sha256:", f"{phase}_")))
    if vals.get("device_code_sha256", "").strip() != sha:
        return None
    v = vals.get(f"{phase}_bytes_per_launch")
    return int(v) if v else None


def host_cores():
    """CPUs this process may run on: the affinity mask, capped by a cgroup CPU quota."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        quota, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if quota != "max" and int(period) > 0:
            n = min(n, max(1, -(-int(quota) // int(period))))
    except (OSError, ValueError):
        pass
    return max(1, n)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The two kernels that take most of a step's device time, with HIP events around their launches
# on the sweep's stream: the cell sweep (one launch per sweep; events around that launch alone)
# and the core levels below the top table (one launch per level; events around the level
# launches).  Bytes: the survey's algorithmic count (the graph stream at 8 bytes per entry plus
# offsets, and per query every label written once and read back once, also those kept in LDS),
# and the bytes that must come from or go to HBM (for the cell sweep: each swept cell's data
# once, the referenced core labels once per query; the core levels keep every label in HBM, so
# both counts agree there).
KERNELS = {"cell_sweep": ("k_cell_chunks", "cell_ms", "cell_launches", "cell_bytes_survey", "cell_bytes"),
           "core_levels": ("k_core_level64", "level_ms", "level_launches", "level_bytes", "level_bytes")}


def roofline_of(prof, prof_iso, steps, names=None):
    def entry(p, key):
        name, t, n, b_survey, b_hbm = KERNELS[key]
        name = (names or {}).get(key, name)
        ms, launches = p[t], max(1, p[n])
        if ms <= 0:
            return None
        per = ms / launches
        ach, ach_hbm = p[b_survey] / launches / 1e9 / (per / 1e3), p[b_hbm] / launches / 1e9 / (per / 1e3)
        return {"kernel": name, "launches": p[n], "ms_total": round(ms, 3), "avg_launch_ms": round(per, 4),
                "algorithmic_bytes_per_launch": int(p[b_survey] / launches), "achieved": round(ach, 1),
                "frac": round(ach / HBM_PEAK_GBS, 4), "hbm_bytes_per_launch": int(p[b_hbm] / launches),
                "achieved_hbm": round(ach_hbm, 1), "frac_hbm": round(ach_hbm / HBM_PEAK_GBS, 4)}

    kernels = {k: entry(prof, k) for k in KERNELS}
    kernels = {k: v for k, v in kernels.items() if v}
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
    d = kernels[dom]
    traffic = measured_traffic(dom)
    roof = {"bound": "hbm", "achieved": d["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d["frac"],
            "traffic": traffic, "kernel": d["kernel"], "avg_launch_ms": d["avg_launch_ms"],
            "algorithmic_bytes_per_launch": d["algorithmic_bytes_per_launch"],
            "achieved_hbm_resident": d["achieved_hbm"], "frac_hbm_resident": d["frac_hbm"],
            "hbm_resident_bytes_per_launch": d["hbm_bytes_per_launch"],
            "kernels": kernels,
            "kernel_ms_per_step": {k: round(v["ms_total"] / steps, 4) for k, v in kernels.items()},
            "note": "dominant kernel by summed HIP-event time over the timed region; consecutive sweeps "
                    "overlap on two streams, so a launch's duration includes device time shared with the "
                    "other sweep's kernels; achieved = the survey's algorithmic bytes (labels kept in LDS "
                    "included), achieved_hbm_resident = the bytes that must cross HBM"}
    if traffic:   # counter bytes per launch over the same launch time
        roof["traffic_gbs"] = round(traffic / 1e9 / (d["avg_launch_ms"] / 1e3), 1)
    iso_d = entry(prof_iso, dom) if prof_iso else None
    if iso_d:
        roof["isolated"] = dict(iso_d, note="same kernel, one sweep per call (host API run), no other sweep on "
                                            "the GPU")
        iso_k = {k: entry(prof_iso, k) for k in KERNELS}
        roof["isolated_kernels"] = {k: v for k, v in iso_k.items() if v}
    return roof


def cpu_baseline(g, src, tau, seconds, threads):
    """The oracle on this host: throughput with one query per thread on `threads` threads (the
    plain tau-bounded Dijkstra with the edge rule, and the paper's isoDijkstra); every query runs
    on one thread, so the per-query times of the throughput run are single-thread latencies
    (taken while the other threads run queries of their own).  About `seconds` of wall time."""
    import oracle

    t0 = time.time()
    orc = oracle.Oracle.from_graph(g)
    workers = [oracle.OracleWorker(orc) for _ in range(threads)]
    log(f"cpu baseline: oracle graph built ({time.time() - t0:.1f}s), {threads} threads, ~{seconds}s budget")

    def throughput(method, budget, nthreads, start):
        nxt, done, lock = [start], [], threading.Lock()
        deadline = time.perf_counter() + budget

        def work(wk):
            while True:
                with lock:
                    if time.perf_counter() > deadline:
                        return
                    j = nxt[0] % len(src)
                    nxt[0] += 1
                a = time.perf_counter()
                getattr(wk, method)(int(src[j]), int(tau[j]))
                with lock:
                    done.append(1000.0 * (time.perf_counter() - a))

        t1 = time.perf_counter()
        ths = [threading.Thread(target=work, args=(w,)) for w in workers[:nthreads]]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        return len(done) / (time.perf_counter() - t1), done

    iso_budget = 0.25 * seconds
    qps, lat = throughput("isochrone", seconds - iso_budget, threads, 0)
    iso_qps, _ = throughput("iso_dijkstra", iso_budget, threads, 0)
    return {"value": qps, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"the benchmark's query list (tau uniform 10-240 min) from its start, one query per thread "
                      f"on {threads} threads, about {seconds:.0f}s in total",
            "host": {"nproc": os.cpu_count(), "usable_cores": host_cores(), "cpu_model": cpu_model()},
            "single_thread_latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "queries": len(lat),
                                         "note": "each query on one thread, measured in the all-core run"},
            "iso_dijkstra_qps": iso_qps}


def lanes_sweep(G, src, tau, ks=(8, 16, 32, 64), count=256):
    """Cells-mode throughput of iso_query_batch over `count` queries with k queries per sweep,
    and the same pairs as sequential single plain-mode queries."""
    import paper_1512_09090_amd as iso

    keep = G.get_tuning()
    out = {}
    for k in ks:
        G.set_tuning(**dict(keep, lanes_per_launch=k))
        G.query_batch(src[:k], tau[:k], iso.MODE_CELLS)
        t0 = time.perf_counter()
        G.query_batch(src[:count], tau[:count], iso.MODE_CELLS)
        out[str(k)] = round(count / (time.perf_counter() - t0), 1)
    G.set_tuning(**keep)
    t0 = time.perf_counter()
    for j in range(count):
        G.query(int(src[j]), int(tau[j]), iso.MODE_PLAIN)
    out["sequential_single_plain"] = round(count / (time.perf_counter() - t0), 1)
    return out


def attainable_bandwidth(mib=1024, reps=5):
    """GB/s of device-to-device copies (read + write bytes), the attainable HBM bandwidth."""
    import torch

    nbytes = int(mib) << 20
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del a, b
    return 2.0 * reps * nbytes / el / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="road18m")
    ap.add_argument("--lanes", type=int, default=64)
    ap.add_argument("--latency-queries", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="choose lanes per launch, block size and cell LDS budget on a query sample first")
    ap.add_argument("--tuning", default="", help="JSON file written by the autotuner to apply")
    ap.add_argument("--save-tuning", default="", help="write the autotuner's result to this JSON file")
    ap.add_argument("--knobs", default="",
                    help="explicit tuning, e.g. lanes_per_launch=32,cell_lds_kb=24,cell_stage=0 (others default)")
    ap.add_argument("--serve-rates", default="100,500,1000,2000,5000,10000,20000,40000",
                    help="offered Poisson rates (queries/s) for the serving section; empty to skip")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-warmup", type=float, default=1.0)
    ap.add_argument("--no-sweep", action="store_true", help="skip the queries-per-sweep comparison")
    ap.add_argument("--cd-minutes", default="5,15,45",
                    help="limits (minutes) of the isoPHAST-CD comparison; empty to skip")
    ap.add_argument("--cd-queries", type=int, default=40)
    ap.add_argument("--profile-only", nargs="?", const="cells", default=None, choices=["cells", "plain"],
                    help="run only the warm-up and the timed batches, in cells mode or (plain) the plain sweep "
                         "(for profiler runs)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first copy this many MiB device-to-device (calibrates profiler byte counters)")
    ap.add_argument("--cache-dir", default=os.environ.get("ISO_CACHE", "/tmp/iso_cache"))
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "queries are independent, so more GPUs would each hold a replica of the graph - not measured here",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import paper_1512_09090_amd as iso
    import synth

    g, G = load_workload(args.workload, args.cache_dir)
    if args.copy_probe_mb:
        copy_probe(args.copy_probe_mb)
    info = G.info()
    # the seeded query list of the workload, long enough that the warm-up and the timed batches
    # hold different queries
    src, tau = synth.config_queries(args.workload, max(1000, (max(1, args.warmup) + args.steps) * max(64, args.lanes)))
    lanes = args.lanes
    G.set_tuning(lanes_per_launch=lanes)
    tuning_note = "defaults"
    if args.knobs:
        best = {k: int(v) for k, v in (kv.split("=") for kv in args.knobs.split(",") if kv)}
        G.set_tuning(**best)
        lanes = G.get_tuning()["lanes_per_launch"]
        tuning_note = f"--knobs {args.knobs}"
        log(f"tuning: {G.get_tuning()} ({tuning_note})")
    elif args.autotune or args.tuning:
        from paper_1512_09090_amd import autotune

        if args.tuning:
            best = autotune.apply(G, args.tuning)
            tuning_note = f"from {args.tuning}"
        else:
            ts, tt = autotune.sample(256, src, tau, seed=1)
            res = autotune.tune(G, ts, tt, log=log)
            best = res["best"]
            if args.save_tuning:
                autotune.save(res, args.save_tuning)
            tuning_note = "autotuned on 256 queries"
        lanes = best["lanes_per_launch"]
        log(f"tuning: {best} ({tuning_note})")

    import torch

    def window(start, count):
        idx = (np.arange(count) + start) % len(src)
        return src[idx], tau[idx]

    # warmup: W batches (also grows the library's device buffers and sizes the result buffer)
    dev = DeviceBatches(iso, G, per_query_hint=40_000)
    log(f"warmup {args.warmup} steps of {lanes} queries")
    ws, wt = window(0, max(1, args.warmup) * lanes)
    timed_mode = iso.MODE_PLAIN if args.profile_only == "plain" else iso.MODE_CELLS
    dev.run(ws, wt, timed_mode)
    dev.hint = max(dev.hint, 2.0 * int(dev.offsets[len(ws)].item()) / len(ws))
    ts_, tt_ = window(args.warmup * lanes, args.steps * lanes)
    dev.reserve(len(ts_))   # the timed call's result buffers, allocated before the timed region
    # timed region: one call over `steps` batches of `lanes` queries, cells mode, edges in HBM
    G.profile_enable(True)
    log(f"timed {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    edges_total = dev.run(ts_, tt_, timed_mode)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    prof = G.profile_read()
    G.profile_enable(False)
    qps = args.steps * lanes / total
    batch_stats = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in G.last_stats().items()}
    log(f"cells batched (device output): {qps:.1f} queries/s, {1000 * total / args.steps:.2f} ms/step, "
        f"{edges_total} edges; profile {prof}")
    log(f"timed call: {batch_stats}")

    if args.profile_only:   # the timed batches only (for profiler runs)
        names = {"cell_sweep": "k_plain_level64"} if (args.profile_only == "plain" and lanes == 64 and
                                                        G.get_tuning()["plain_sweep"] == 0) else None
        print(json.dumps({"metric": METRIC, "value": round(qps, 2), "unit": "queries/s", "steps": args.steps,
                          "profile_only": args.profile_only, "profile": prof,
                          "kernels": roofline_of(prof, None, args.steps, names)["kernels"]}), flush=True)
        return

    # the same through the host API (edges copied to host memory over PCIe): one call per batch,
    # and one call over the same queries (overlapping sweeps)
    # (one sweep per call: also the phase times of a sweep that shares the GPU with no other)
    run_batches(G, src, tau, lanes, 1, iso.MODE_CELLS)
    G.profile_enable(True)
    t0 = time.perf_counter()
    times = run_batches(G, src, tau, lanes, args.steps, iso.MODE_CELLS, start=args.warmup * lanes)
    qps_host = args.steps * lanes / (time.perf_counter() - t0)
    prof_iso = G.profile_read()
    G.profile_enable(False)
    G.query_batch(ts_, tt_, iso.MODE_CELLS)   # warms the pinned result pool for a call of this size
    t0 = time.perf_counter()
    G.query_batch(ts_, tt_, iso.MODE_CELLS)
    qps_host_pipe = args.steps * lanes / (time.perf_counter() - t0)
    log(f"host API: {qps_host:.1f} queries/s one batch per call, {qps_host_pipe:.1f} in one call")

    # plain sweep, device output, a quarter of the batches
    np_steps = max(2, args.steps // 4)
    ps_, pt_ = window(args.warmup * lanes, np_steps * lanes)
    dev.run(ps_[:lanes], pt_[:lanes], iso.MODE_PLAIN)
    G.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev.run(ps_, pt_, iso.MODE_PLAIN)
    torch.cuda.synchronize()
    qps_plain = np_steps * lanes / (time.perf_counter() - t0)
    prof_plain = G.profile_read()
    G.profile_enable(False)
    # the plain sweep (every cell for every query): the same two kernels with their own bytes
    # (at 64 queries per sweep the plain mode sweeps the cells as a stream of levels)
    plain_names = {"cell_sweep": "k_plain_level64"} if lanes == 64 and G.get_tuning()["plain_sweep"] == 0 else None
    plain_phases = roofline_of(prof_plain, None, np_steps, plain_names)["kernels"]
    log(f"plain batched (device output): {qps_plain:.1f} queries/s; kernels {plain_phases}")

    # the other output of Section 3: vertices in range, as one bitmap row per query over the
    # original ids, left in HBM (one call per batch of `lanes` queries)
    W = (info["n"] + 63) // 64
    vbits = torch.empty((lanes, W), dtype=torch.int64, device="cuda:0")
    vs_, vt_ = window(args.warmup * lanes, max(2, args.steps // 4) * lanes)
    G.query_batch_vertices_device(vs_[:lanes], vt_[:lanes], iso.MODE_CELLS, vbits)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(0, len(vs_), lanes):
        G.query_batch_vertices_device(vs_[b:b + lanes], vt_[b:b + lanes], iso.MODE_CELLS, vbits)
    torch.cuda.synchronize()
    qps_vert = len(vs_) / (time.perf_counter() - t0)
    in_range = int(np.bitwise_count(vbits.cpu().numpy().view(np.uint64)).sum())
    log(f"vertices in range (device bitmaps): {qps_vert:.1f} queries/s; last batch {in_range} (vertex, query) pairs")

    # isochrone polygons (Section 7) need a planar embedding, which the kNN stand-in lacks: a
    # 300 x 300 jittered grid (the 64 x 64 test grid's generator; grids are slow to contract, so
    # it stays small), 96 cells, limits of about 25-180 edges; the embedding is built on the
    # first call
    gp = synth.grid_graph(300, 300, seed=7)
    t0 = time.perf_counter()
    GP = iso.Graph(gp.n, gp.tail, gp.head, gp.w, xy=gp.xy, num_cells=96, device=0)
    prep_s = time.perf_counter() - t0
    prng = np.random.default_rng(18)
    psrc = prng.integers(0, gp.n, size=max(2, args.steps // 4) * lanes).astype(np.uint32)
    ptau = prng.integers(5_000, 40_000, size=psrc.size).astype(np.uint32)
    t0 = time.perf_counter()
    GP.polygon(int(psrc[0]), int(ptau[0]), iso.MODE_CELLS)
    rot_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    darts = cycles = 0
    for b in range(0, psrc.size, lanes):
        dflat, _, _, coff = GP.polygon_batch_raw(psrc[b:b + lanes], ptau[b:b + lanes], iso.MODE_CELLS)
        darts += len(dflat)
        cycles += int(coff[-1])
    el = time.perf_counter() - t0
    pstats = GP.last_stats()
    polygons = {"value": round(psrc.size / el, 2), "unit": "queries/s",
                "ms_per_batch": round(1000 * el * lanes / psrc.size, 3), "queries_per_call": lanes,
                "darts_per_query": round(darts / psrc.size, 1), "cycles_per_query": round(cycles / psrc.size, 1),
                "graph": f"jittered grid 300 x 300 ({gp.n} vertices, {gp.m} arcs), 96 cells, tau uniform "
                         "5 000-40 000 (about 25-180 edges)",
                "prep_s": round(prep_s, 2), "embedding_build_s": round(rot_s, 3),
                "last_call_ms": {"vertex_sweep": round(pstats["t_device_ms"] + pstats["t_upward_ms"], 3),
                                 "polygon_kernels_and_copy": round(pstats["t_sort_ms"], 3)},
                "note": "iso_query_polygon_batch: darts in cycle order and cycle starts copied to host memory; "
                        "paper's Section 7 context: tens of ms per polygon on one core (continental graph)"}
    GP.close()
    log(f"polygons: {polygons}")

    # one-to-many (RPHAST, the paper's Table 1 workload): a ball of 2^14 targets, sources drawn
    # from the ball, distances left in HBM (one call per batch of `lanes` sources)
    _, ball = synth.target_ball(g, 1 << 14, seed=16)
    tg = G.select_targets(ball)
    tinfo = tg.info()
    rng = np.random.default_rng(17)
    tsrc = ball[rng.integers(0, ball.size, size=max(2, args.steps // 4) * lanes)]
    tdist = torch.empty((lanes, ball.size), dtype=torch.int32, device="cuda:0")
    tg.query_device(tsrc[:lanes], tdist)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(0, tsrc.size, lanes):
        tg.query_device(tsrc[b:b + lanes], tdist)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    one_to_many = {"targets": int(ball.size), "select_ms": round(tinfo["select_ms"], 3),
                   "restricted_vertices": tinfo["vertices"], "restricted_arcs": tinfo["arcs"],
                   "level_groups": tinfo["groups"], "sources_per_call": lanes,
                   "value": round(tsrc.size / el, 2), "unit": "sources/s",
                   "ms_per_call": round(1000 * el / (tsrc.size // lanes), 4),
                   "note": "iso_targets_query_device: d(s, t) for every target of a 2^14 ball (breadth-first "
                           "from a random centre), sources from the ball; paper's Table 1 context (one core): "
                           "selection 1.29 ms, 0.16 ms per source"}
    tg.close()
    log(f"one-to-many: {one_to_many}")

    # single-query latency (one query per call)
    lat = {}
    single_qps = {}
    for name, mode in (("cells", iso.MODE_CELLS), ("plain", iso.MODE_PLAIN)):
        G.query(int(src[0]), int(tau[0]), mode)
        ts = []
        t0 = time.perf_counter()
        for j in range(args.latency_queries):
            a = time.perf_counter()
            G.query(int(src[j]), int(tau[j]), mode)
            ts.append(1000.0 * (time.perf_counter() - a))
        single_qps[name] = args.latency_queries / (time.perf_counter() - t0)
        lat[name] = {"p50": percentile(ts, 50), "p99": percentile(ts, 99), "mean": float(np.mean(ts))}
        st = G.last_stats()
        lat[name]["last_query"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
        log(f"single {name}: {lat[name]}")

    # isoPHAST-CD (core isoDijkstra on the host) against the core sweep at fixed limits: single
    # queries and batches of `lanes`, the same sources for both modes
    core_search = {}
    if args.cd_minutes:
        cd_src = synth.batch_queries(info["n"], max(args.cd_queries, lanes), seed=515)[0]
        cd_dev = DeviceBatches(iso, G, 64.0)
        for minutes in [int(x) for x in args.cd_minutes.split(",") if x]:
            t_lim = np.full(len(cd_src), minutes * 60_000, dtype=np.uint32)
            row = {}
            for name, mode in (("cd", iso.MODE_CD), ("cells", iso.MODE_CELLS)):
                G.query(int(cd_src[0]), int(t_lim[0]), mode)
                ts = []
                for j in range(args.cd_queries):
                    a = time.perf_counter()
                    G.query(int(cd_src[j]), int(t_lim[j]), mode)
                    ts.append(1000.0 * (time.perf_counter() - a))
                    if sum(ts) > 8000.0:   # bounded wall time per limit and mode
                        break
                cd_dev.run(cd_src[:lanes], t_lim[:lanes], mode)
                torch.cuda.synchronize()
                a = time.perf_counter()
                for _ in range(3):
                    cd_dev.run(cd_src[:lanes], t_lim[:lanes], mode)
                torch.cuda.synchronize()
                row[name] = {"queries": len(ts), "single_p50_ms": round(percentile(ts, 50), 3),
                             "single_p99_ms": round(percentile(ts, 99), 3),
                             "batch_qps": round(3 * lanes / (time.perf_counter() - a), 1)}
            core_search[f"{minutes}min"] = row
            log(f"isoPHAST-CD vs CP at {minutes} min: {row}")

    roofline = roofline_of(prof, prof_iso, args.steps)

    serve = None
    if args.serve_rates:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        serve = {"mode": "cells", "max_lanes": lanes, "max_inflight": 2,
                 "trace": f"Poisson arrivals, {args.serve_seconds:g}s per rate after {args.serve_warmup:g}s "
                          "warm-up, uniform sources, tau log-uniform 5-300 min; latency = submit to result ready",
                 "rates": serving(G, info["n"], rates, args.serve_seconds, lanes, 2, args.serve_warmup)}

    sweep = None if args.no_sweep else lanes_sweep(G, src, tau)
    if sweep:
        log(f"queries per sweep: {sweep}")
    bw = attainable_bandwidth()
    if bw:
        log(f"attainable bandwidth (device copy): {bw:.0f} GB/s")
        roofline["attainable_gbs"] = round(bw, 1)
        roofline["frac_of_attainable"] = round(roofline["achieved"] / bw, 4)

    cpu = None
    if not args.no_cpu:
        threads = args.cpu_threads or host_cores()
        cpu = cpu_baseline(g, src, tau, args.cpu_seconds, threads)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": METRIC, "value": round(qps, 2), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1000 * total / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {info['n']}-vertex road-like kNN graph, {info['m']} arcs, "
                               f"{info['num_cells']} cells; batches of {lanes} queries, cell-restricted sweep, edges kept in HBM, "
                               "tau uniform 10-240 min",
                   "n": info["n"], "m": info["m"], "cells": info["num_cells"], "core": info["n_core"],
                   "core_levels": info["core_levels"], "down_arcs": info["down_arcs"], "lanes": lanes,
                   "mode": "cells", "tuning": dict(G.get_tuning(), source=tuning_note)},
        "latency_ms": lat,
        "single_query_qps": {k: round(v, 2) for k, v in single_qps.items()},
        "batched_plain_qps": round(qps_plain, 2),
        "polygons": polygons,
        "plain_sweep_roofline": dict(plain_phases, unit="GB/s", peak=HBM_PEAK_GBS,
                                     note="plain mode (every cell swept for every query), two overlapping "
                                          "streams, HIP events around the kernels' launches"),
        "host_api_qps": {"one_batch_per_call": round(qps_host, 2), "one_call": round(qps_host_pipe, 2),
                         "note": "iso_query_batch, edges copied to host memory (PCIe included)",
                         "call_ms_p50": round(1000 * percentile(times, 50), 3),
                         "call_ms_p99": round(1000 * percentile(times, 99), 3)},
        "vertex_output_qps": {"value": round(qps_vert, 2), "queries_per_call": lanes,
                              "bitmap_bytes_per_call": lanes * W * 8, "in_range_pairs_last_call": in_range,
                              "note": "iso_query_batch_vertices_device: the vertices in range of each query "
                                      "as a bitmap over the original ids, left in HBM"},
        "one_to_many": one_to_many,
        "core_search_mode": dict(core_search, note="isoPHAST-CD (isoDijkstra over the core on the host, stopped at "
                                 "tau) against the core sweep (isoPHAST-CP), fixed tau, same sources; single queries "
                                 "through iso_query, batches through iso_query_batch_device"),
        "queries_per_sweep_qps": sweep,
        "timed_call": dict(batch_stats, edges_in_hbm=int(edges_total)),
        "serving": serve,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
