"""Benchmark: exact convex hulls of 20M-point sets on one MI355X.

A step is one full pass of the hot path (extreme points, quadrilateral
discard and region distribution, region sort, SPA, chain concatenation and
the Melkman finish) over each of the three 20M-point inputs: uniform square,
uniform disk, and Gaussian (sigma 2^20 around 2^22, clamped), integer-valued
float32 in [0, 2^23).  Inputs are generated on the host and copied to HBM
before timing starts.  ``value`` is input points per second over the timed
steps (Mpts/s), with the fastest of four ways to call the library, all
timed: three blocking ``hull2d`` calls per step; three ``hull2d_async``
calls queued on one stream with one synchronisation; one ``hull2d_async``
call per input on three streams; that three-stream step captured in a HIP
graph and replayed.  Their results are checked equal; ``calls`` holds all
four.

Prints one JSON line.  Extra fields: per-distribution rates and counts, the
per-stage times from HIP events recorded on the library's stream, the
roofline of the dominant kernel, and the CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
DISTS = (("square", 2), ("disk", 3), ("gaussian", 4))
N_POINTS = 20_000_000
BATCH_SETS, BATCH_LO, BATCH_HI, BATCH_SEED = 4096, 1_000, 1_000_000, 7
SERVE_LO, SERVE_HI, SERVE_POOL, SERVE_SEED = 10_000, 20_000_000, 48, 8
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1508_05488_amd", "csrc", "chainhull.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N_POINTS, help="points per input (default 20M)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-sets measurement")
    ap.add_argument("--batch-sets", type=int, default=BATCH_SETS)
    ap.add_argument("--batch-calls", type=int, default=30)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-other", action="store_true", help="skip the 100K and adversarial single-hull configurations")
    ap.add_argument("--serve-rate", type=float, default=10_000.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-requests", type=int, default=4000)
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain per-set comparison of the batched measurement")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def src_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(name: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (``profiles/<name>.md``), if its counters were taken on the current
    kernel source.  The summary holds ``key: value`` lines, among them
    ``source_sha256_16`` and ``bytes_per_launch``."""
    path = os.path.join(PROFILE_DIR, f"{name}.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            k, sep, v = line.strip().lstrip("-* ").partition(":")
            if sep:
                rec[k.strip().strip("`")] = v.strip().strip("`")
    if rec.get("source_sha256_16") != src_hash():
        return None
    try:
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def sha16(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measure_other_configs(ch, wl, torch, dev):
    """The other single-hull configurations: 100K uniform points (latency:
    median of 21 blocking calls) and 20M adversarial points (10 % on a
    circle; median of 3 blocking calls, end to end, its finish on the host)."""
    out = {}
    for name, dist, n, seed, reps in (("square_100k", "square", 100_000, 1, 21),
                                      ("adversarial_20m", "adversarial", 20_000_000, 5, 3)):
        pts = wl.generate(dist, n, seed)
        d = torch.from_numpy(pts).to(dev)
        for _ in range(2):
            ch.hull2d(d)
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            a = time.perf_counter()
            h = ch.hull2d(d)
            torch.cuda.synchronize()
            t.append(time.perf_counter() - a)
        ch.set_timing(True)
        ch.hull2d(d)
        torch.cuda.synchronize()
        ch.set_timing(False)
        st = ch.last_stats()
        ms = float(np.median(t)) * 1e3
        out[name] = {"n": n, "seed": seed, "input_sha256_16": sha16(pts), "ms_median": round(ms, 4),
                     "mpts_per_s": round(n / ms / 1e3, 1), "hull": int(h.numel()), "polygon": st["polygon"],
                     "device_finish": st["device_finish"],
                     "stages_ms": {k: round(v, 4) for k, v in st["ms"].items() if not k.startswith("unused")}}
        del d
    torch.cuda.empty_cache()
    return out


def measure_batched(ch, wl, torch, dev, args):
    """Independent sets in one call: 4096 sets with sizes log-uniform in
    [1e3, 1e6], each uniform square, uniform disk or Gaussian.  Times
    blocking hull2d_batched calls (inputs resident in HBM) for hulls/s and
    the p50/p99 call latency, the batched kernel alone with HIP events, and
    the same sets through the plain path, one hull2d call per set."""
    num = args.batch_sets
    pts, offs, dists = wl.batched_sets(num, BATCH_LO, BATCH_HI, BATCH_SEED)
    n_total = int(offs[-1])
    d_pts = torch.from_numpy(pts).to(dev)
    out = torch.empty(max(n_total, 1), dtype=torch.int32, device=dev)
    cnt = torch.zeros(max(num, 1), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    lib = ch.lib()

    def call():
        rc = lib.hull2d_batched(d_pts.data_ptr(), offs.ctypes.data, num, out.data_ptr(), cnt.data_ptr(),
                                stream.cuda_stream)
        if rc != ch.CH_OK:
            raise ch.ChainHullError(rc, "hull2d_batched")

    for _ in range(3):
        call()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.batch_calls):
        a = time.perf_counter()
        call()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
    elapsed = time.perf_counter() - t0
    bstats = ch.last_batch_stats()
    ch.set_timing(True)
    kms = []
    for _ in range(5):
        call()
        kms.append(ch.last_batch_stats()["ms_kernel"])
    ch.set_timing(False)
    torch.cuda.synchronize()
    lat_ms = np.array(lat) * 1e3
    k_ms = float(np.median(kms))
    k_bytes = 8.0 * n_total  # one read of every point
    plain = None
    if not args.no_plain:
        # the plain path on the same sets: one blocking hull2d call per set
        o1 = torch.empty(max(n_total, 1), dtype=torch.int32, device=dev)
        c1 = torch.zeros(1, dtype=torch.int32, device=dev)
        plain_lat = []
        for rep in range(2):
            torch.cuda.synchronize()
            plain_lat = []
            for k in range(num):
                lo, hi = int(offs[k]), int(offs[k + 1])
                a = time.perf_counter()
                rc = lib.hull2d(d_pts.data_ptr() + 8 * lo, hi - lo, o1.data_ptr() + 4 * lo, c1.data_ptr(),
                                stream.cuda_stream)
                if rc != ch.CH_OK:
                    raise ch.ChainHullError(rc, "hull2d")
                plain_lat.append(time.perf_counter() - a)
            torch.cuda.synchronize()
        plain_s = float(np.sum(plain_lat))
        # the batched results equal the plain ones (the plain calls wrote every
        # set's hull at its own offset; counts from the batched call)
        c_host = cnt[:num].cpu().numpy()
        o_b, o_p = out.cpu().numpy(), o1.cpu().numpy()
        same = all(np.array_equal(o_b[offs[k]:offs[k] + c_host[k]], o_p[offs[k]:offs[k] + c_host[k]])
                   for k in range(num))
        plain = {"hulls_per_s": round(num / plain_s, 1), "mpts_per_s": round(n_total / plain_s / 1e6, 1),
                 "latency_ms_p50": round(float(np.percentile(np.array(plain_lat) * 1e3, 50)), 4),
                 "latency_ms_p99": round(float(np.percentile(np.array(plain_lat) * 1e3, 99)), 4),
                 "note": "one blocking hull2d call per set, same sets, same GPU",
                 "speedup_of_batched": round((num * args.batch_calls / elapsed) / (num / plain_s), 2),
                 "results_equal": bool(same)}
        del o1
    del d_pts, out
    torch.cuda.empty_cache()
    return {
        "workload": f"{num} independent sets, sizes log-uniform in [{BATCH_LO}, {BATCH_HI}], "
                    "each uniform square, uniform disk or Gaussian (seed 7); one hull2d_batched call",
        "points": n_total,
        "hulls_per_s": round(num * args.batch_calls / elapsed, 1),
        "mpts_per_s": round(n_total * args.batch_calls / elapsed / 1e6, 1),
        "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 4),
        "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 4),
        "calls": args.batch_calls,
        "kernel_ms": round(k_ms, 4),
        "kernel_roofline": {"bound": "hbm", "kernel": "k_batch_hull", "achieved": round(k_bytes / (k_ms * 1e-3) / 1e9, 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(k_bytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "algorithmic_bytes_per_launch": k_bytes,
                            "traffic": load_traffic("k_batch_hull_4096sets") if num == BATCH_SETS else None},
        "sets_on_single_hull_path": bstats["redo_sets"],
        "plain_path": plain,
    }


def measure_serving(ch, wl, torch, dev, args):
    """Hull requests arriving as a Poisson stream at a fixed rate, sizes
    log-uniform in [1e4, 2e7], each uniform square, disk or Gaussian (a pool
    of 48 seeded requests resident in HBM, submitted in turn), served by the
    continuous-batching server with a 288 GB budget.  Latency is from
    submission to completion.  The same arrival stream is then served by
    the plain path, one blocking hull2d call at a time in arrival order."""
    import threading
    rng = np.random.default_rng(SERVE_SEED)
    names = ("square", "disk", "gaussian")
    sizes = np.floor(np.exp(rng.uniform(np.log(SERVE_LO), np.log(SERVE_HI), size=SERVE_POOL))).astype(np.int64)
    pool = [torch.from_numpy(wl.generate(names[k % 3], int(n), SERVE_SEED * 1000 + k)).to(dev)
            for k, n in enumerate(sizes)]
    nreq = args.serve_requests
    order = np.arange(nreq) % SERVE_POOL
    gaps = rng.exponential(1.0 / args.serve_rate, size=nreq)
    pts_total = int(sum(int(sizes[k]) for k in order))

    def run_server():
        lat = []
        with ch.Server(workers=args.serve_workers, mem_budget=288 << 30) as srv:
            for p in pool[:8]:  # warm the workers' workspaces
                srv.wait(srv.submit(p))
            tickets = []
            done = threading.Event()

            def waiter():
                k = 0
                while k < nreq:
                    if k < len(tickets):
                        lat.append(srv.wait(tickets[k])[1])
                        k += 1
                    else:
                        time.sleep(0)
                done.set()

            th = threading.Thread(target=waiter)
            th.start()
            t0 = time.perf_counter()
            due = t0
            for k in range(nreq):
                due += gaps[k]
                while time.perf_counter() < due:
                    pass
                tickets.append(srv.submit(pool[order[k]]))
            th.join()
            elapsed = time.perf_counter() - t0
            st = srv.stats()
        return np.array(lat), elapsed, st

    lat, elapsed, st = run_server()
    # closed-loop capacity: the same requests all submitted at once
    with ch.Server(workers=args.serve_workers, mem_budget=288 << 30) as srv:
        for p in pool[:8]:
            srv.wait(srv.submit(p))
        t0 = time.perf_counter()
        tk = [srv.submit(pool[order[k]]) for k in range(min(nreq, 4 * SERVE_POOL))]
        for t in tk:
            srv.wait(t)
        cap = len(tk) / (time.perf_counter() - t0)
    # the plain path on the same arrivals: one hull2d at a time
    out = torch.empty(int(sizes.max()), dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    lib = ch.lib()
    torch.cuda.synchronize()
    plat = []
    t0 = time.perf_counter()
    arrive = t0
    for k in range(nreq):
        arrive += gaps[k]
        while time.perf_counter() < arrive:
            pass
        p = pool[order[k]]
        rc = lib.hull2d(p.data_ptr(), p.shape[0], out.data_ptr(), cnt.data_ptr(), stream.cuda_stream)
        if rc != ch.CH_OK:
            raise ch.ChainHullError(rc, "hull2d")
        stream.synchronize()
        plat.append(time.perf_counter() - arrive)
    pel = time.perf_counter() - t0
    plat = np.array(plat) * 1e3
    del pool, out
    torch.cuda.empty_cache()
    return {
        "workload": f"Poisson arrivals at {args.serve_rate:.0f} requests/s, sizes log-uniform in [{SERVE_LO}, "
                    f"{SERVE_HI}], uniform square, disk or Gaussian (a pool of {SERVE_POOL} seeded requests in HBM, "
                    f"submitted in turn); {args.serve_workers} worker streams; 288 GB admission budget",
        "requests": nreq,
        "points": pts_total,
        "hulls_per_s": round(nreq / elapsed, 1),
        "mpts_per_s": round(pts_total / elapsed / 1e6, 1),
        "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
        "latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
        "capacity_hulls_per_s": round(cap, 1),
        "server_stats": st,
        "plain_path": {"hulls_per_s": round(nreq / pel, 1),
                       "latency_ms_p50": round(float(np.percentile(plat, 50)), 4),
                       "latency_ms_p99": round(float(np.percentile(plat, 99)), 4),
                       "note": "same arrivals, one blocking hull2d call at a time in arrival order"},
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1508_05488_amd as ch
    from paper_1508_05488_amd import workloads as wl

    if not os.path.exists(ch.LIB_PATH):
        from paper_1508_05488_amd import build as lib_build
        lib_build.build()
    dev = torch.device("cuda:0")
    n = args.n
    host = {d: wl.generate(d, n, seed) for d, seed in DISTS}
    inputs = {d: torch.from_numpy(host[d]).to(dev) for d, _ in DISTS}
    outs = {d: (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(1, dtype=torch.int32, device=dev))
            for d, _ in DISTS}
    stream = torch.cuda.current_stream()

    def step(collect=None):
        for d, _ in DISTS:
            rc = ch.hull2d_into(inputs[d], outs[d][0], outs[d][1], stream)
            if rc != ch.CH_OK:
                raise ch.ChainHullError(rc, f"hull2d {d}")
            if collect is not None:
                collect[d].append(ch.last_stats())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region 1: the path as a caller runs it (no timing events)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    total_pts = n * len(DISTS) * args.steps
    value_blocking = total_pts / elapsed / 1e6

    # timed region 1b: the same hulls queued with hull2d_async (every step on
    # the device, no host round trip between the inputs), one
    # synchronisation per step when the counts are read; an input left to
    # the host finish (CH_BATCH_REDO) is recomputed with hull2d inside the
    # region
    acnt = torch.empty(len(DISTS), dtype=torch.int32, device=dev)
    aout = {d: torch.empty(n, dtype=torch.int32, device=dev) for d, _ in DISTS}
    redo = [0]

    def step_async():
        for k, (d, _) in enumerate(DISTS):
            rc = ch.hull2d_async(inputs[d], aout[d], acnt[k:k + 1], stream)
            if rc != ch.CH_OK:
                raise ch.ChainHullError(rc, f"hull2d_async {d}")
        counts = acnt.cpu()  # synchronises the stream
        for k, (d, _) in enumerate(DISTS):
            c = int(counts[k])
            if c == ch.CH_BATCH_REDO:
                redo[0] += 1
                rc = ch.hull2d_into(inputs[d], aout[d], acnt[k:k + 1], stream)
                if rc != ch.CH_OK:
                    raise ch.ChainHullError(rc, f"hull2d {d}")
            elif c < 0:
                raise ch.ChainHullError(c, f"hull2d_async {d}")

    for _ in range(args.warmup):
        step_async()
    torch.cuda.synchronize()
    t0a = time.perf_counter()
    for _ in range(args.steps):
        step_async()
    torch.cuda.synchronize()
    t1a = time.perf_counter()
    elapsed_async = t1a - t0a
    # the queued results are the blocking ones
    for k, (d, _) in enumerate(DISTS):
        c = int(outs[d][1].item())
        if int(acnt[k].item()) != c or not torch.equal(aout[d][:c], outs[d][0][:c]):
            raise RuntimeError(f"hull2d_async and hull2d differ on {d}")
    value_async = total_pts / elapsed_async / 1e6

    # timed region 1c: the three inputs on three streams (one library
    # workspace each), so that one hull's short latency-bound kernels overlap
    # another's pass over its points; one synchronisation per step
    streams = [torch.cuda.Stream() for _ in DISTS]
    mcnt = torch.empty(len(DISTS), dtype=torch.int32, device=dev)
    mout = {d: torch.empty(n, dtype=torch.int32, device=dev) for d, _ in DISTS}
    cur = torch.cuda.current_stream()

    def step_streams():
        for k, (d, _) in enumerate(DISTS):
            streams[k].wait_stream(cur)  # the inputs and the count buffer are ready
            rc = ch.hull2d_async(inputs[d], mout[d], mcnt[k:k + 1], streams[k])
            if rc != ch.CH_OK:
                raise ch.ChainHullError(rc, f"hull2d_async {d}")
        for st in streams:
            cur.wait_stream(st)
        counts = mcnt.cpu()  # synchronises the current stream, which waited on all three
        for k, (d, _) in enumerate(DISTS):
            c = int(counts[k])
            if c == ch.CH_BATCH_REDO:
                redo[0] += 1
                rc = ch.hull2d_into(inputs[d], mout[d], mcnt[k:k + 1], cur)
                if rc != ch.CH_OK:
                    raise ch.ChainHullError(rc, f"hull2d {d}")
            elif c < 0:
                raise ch.ChainHullError(c, f"hull2d_async {d}")

    for _ in range(args.warmup):
        step_streams()
    torch.cuda.synchronize()
    t0m = time.perf_counter()
    for _ in range(args.steps):
        step_streams()
    torch.cuda.synchronize()
    t1m = time.perf_counter()
    elapsed_streams = t1m - t0m
    for k, (d, _) in enumerate(DISTS):
        c = int(outs[d][1].item())
        if int(mcnt[k].item()) != c or not torch.equal(mout[d][:c], outs[d][0][:c]):
            raise RuntimeError(f"hull2d_async on three streams and hull2d differ on {d}")
    value_streams = total_pts / elapsed_streams / 1e6

    # timed region 1d: the three-stream step captured once in a HIP graph
    # (the workspaces exist after the steps above, so the capture allocates
    # nothing) and replayed, one launch and one synchronisation per step; the
    # graph ends with a copy of the counts into pinned host memory
    hcnt = torch.empty(len(DISTS), dtype=torch.int32, pin_memory=True)
    gcap = torch.cuda.Stream()
    gcap.wait_stream(cur)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gcap):
        gs = torch.cuda.current_stream()
        for k, (d, _) in enumerate(DISTS):
            streams[k].wait_stream(gs)
            rc = ch.hull2d_async(inputs[d], mout[d], mcnt[k:k + 1], streams[k])
            if rc != ch.CH_OK:
                raise ch.ChainHullError(rc, f"hull2d_async {d} (capture)")
        for st in streams:
            gs.wait_stream(st)
        hcnt.copy_(mcnt, non_blocking=True)

    def step_graph():
        graph.replay()
        cur.synchronize()
        counts = hcnt.numpy()
        for k, (d, _) in enumerate(DISTS):
            c = int(counts[k])
            if c == ch.CH_BATCH_REDO:
                redo[0] += 1
                rc = ch.hull2d_into(inputs[d], mout[d], mcnt[k:k + 1], cur)
                if rc != ch.CH_OK:
                    raise ch.ChainHullError(rc, f"hull2d {d}")
            elif c < 0:
                raise ch.ChainHullError(c, f"hull2d_async {d}")

    for _ in range(args.warmup):
        step_graph()
    torch.cuda.synchronize()
    t0g = time.perf_counter()
    for _ in range(args.steps):
        step_graph()
    torch.cuda.synchronize()
    t1g = time.perf_counter()
    elapsed_graph = t1g - t0g
    for k, (d, _) in enumerate(DISTS):
        c = int(outs[d][1].item())
        if int(mcnt[k].item()) != c or not torch.equal(mout[d][:c], outs[d][0][:c]):
            raise RuntimeError(f"the graph of three hull2d_async streams and hull2d differ on {d}")
    value_graph = total_pts / elapsed_graph / 1e6
    del graph
    torch.cuda.synchronize()
    for st in streams:
        ch.release_stream(st)
    del mout

    ways = {"hull2d": (value_blocking, elapsed), "hull2d_async": (value_async, elapsed_async),
            "hull2d_async_3_streams": (value_streams, elapsed_streams),
            "hull2d_async_3_streams_graph": (value_graph, elapsed_graph)}
    api = max(ways, key=lambda k: ways[k][0])
    value = ways[api][0]
    ms_per_step = 1e3 * ways[api][1] / args.steps

    # timed region 2: the same steps with HIP events recorded by the library
    # on the call's stream around every stage
    ch.set_timing(True)
    stats = {d: [] for d, _ in DISTS}
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step(stats)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ch.set_timing(False)

    stage_ms = {}
    for key in ch.STAGES:
        stage_ms[key] = float(np.mean([s["ms"][key] for d, _ in DISTS for s in stats[d]]))
    per_dist = {}
    for d, _ in DISTS:
        s = stats[d][-1]
        per_dist[d] = {
            "hull": s["hull"], "s1": int(sum(s["s1"])), "open": s["open"], "candidates": s["candidates"],
            "s2": int(sum(s["s2"])),
        }
        for key in ("sample", "stream", "cand", "sort", "spa", "finish_dev", "gather", "finish"):
            per_dist[d][key + "_ms"] = float(np.mean([x["ms"][key] for x in stats[d]]))

    # counts of the discard rounds (the stats mode of the library counts the
    # round-1 survivors; outside the timed regions)
    for d, _ in DISTS:
        _, pst = ch.polygon(inputs[d])
        per_dist[d].update({"s1": int(sum(pst["s1"])), "s2": int(sum(pst["s2"]))})
    torch.cuda.synchronize()

    # roofline of the dominant kernel, the one pass over the points: it reads
    # 8 bytes per point and writes 12 bytes per listed (open) point; its
    # duration is the event pair that brackets its launch alone
    open_mean = float(np.mean([s["open"] for d, _ in DISTS for s in stats[d]]))
    dom = "k_stream"
    dom_ms, dom_bytes = stage_ms["stream"], 8.0 * n + 12.0 * open_mean
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    traffic = load_traffic("k_stream_traffic_20m")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": dom_bytes, "avg_launch_ms": dom_ms}

    # whole-preprocessing accounting with B_alg = 16n + 24*s1 + 12*s2
    b_alg = [16.0 * n + 24.0 * per_dist[d]["s1"] + 12.0 * per_dist[d]["s2"] for d, _ in DISTS]
    t_pre = sum(stage_ms[k] for k in ("sample", "stream", "cand", "sort", "spa"))
    pre_frac = float(np.mean(b_alg)) / (t_pre * 1e-3) / (HBM_PEAK_GBS * 1e9) if t_pre > 0 else 0.0

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import hull as oracle
        tc = 0.0
        for d, _ in DISTS:
            a = time.perf_counter()
            oracle.hull(host[d])
            tc += time.perf_counter() - a
        cpu = {"value": round(n * len(DISTS) / tc / 1e6, 3), "unit": "Mpts/s", "cores": 1, "kind": "oracle",
               "sample": f"one single-threaded oracle run on each of the three {n}-point inputs ({tc:.1f} s); "
                         f"host CPU {cpu_model()}, {os.cpu_count()} logical CPUs"}

    other = None if args.no_other else measure_other_configs(ch, wl, torch, dev)

    batched = None
    if not args.no_batched:
        del inputs, outs
        torch.cuda.empty_cache()
        batched = measure_batched(ch, wl, torch, dev, args)

    serving = None
    if not args.no_serving:
        serving = measure_serving(ch, wl, torch, dev, args)

    if args.copy_probe_mb:
        src = torch.empty(args.copy_probe_mb << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    line = {
        "metric": "Mpts/s on 20M-pt exact hull",
        "value": round(value, 2),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+u32 exact",
        "data": "synthetic",
        "config": {"workload": f"exact 2D hull, {n} integer-valued f32 points in [0,2^23), "
                               "three inputs per step: uniform square, uniform disk, Gaussian sigma 2^20",
                   "n_points": n, "inputs_per_step": len(DISTS), "seeds": [s for _, s in DISTS],
                   "input_sha256_16": {d: sha16(host[d]) for d, _ in DISTS},
                   "api": api},
        "calls": {"hull2d_async": {"value": round(value_async, 2), "ms_per_step": round(1e3 * elapsed_async / args.steps, 4),
                                   "redo": redo[0],
                                   "note": "three calls queued per step, one synchronisation when the counts are read"},
                  "hull2d": {"value": round(value_blocking, 2), "ms_per_step": round(1e3 * elapsed / args.steps, 4),
                             "note": "three blocking calls per step"},
                  "hull2d_async_3_streams": {"value": round(value_streams, 2),
                                             "ms_per_step": round(1e3 * elapsed_streams / args.steps, 4),
                                             "note": "one hull2d_async call per input, each on its own stream "
                                                     "(and library workspace), one synchronisation per step"},
                  "hull2d_async_3_streams_graph": {"value": round(value_graph, 2),
                                                   "ms_per_step": round(1e3 * elapsed_graph / args.steps, 4),
                                                   "note": "the three-stream step captured once in a HIP graph and "
                                                           "replayed: one launch and one synchronisation per step"}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stages_ms": {k: round(v, 4) for k in ("sample", "stream", "cand", "sort", "spa", "finish_dev", "gather", "finish")
                      for v in [stage_ms[k]]},
        "ms_per_step_with_events": round(1e3 * (t3 - t2) / args.steps, 4),
        "preprocess_b_alg_frac": round(pre_frac, 4),
        "per_distribution": per_dist,
        "other_configs": other,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
