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

``per_config`` times every single-hull configuration on its own, cold: a
1 GiB write precedes each repetition so that no input is served from the
256 MB last-level cache.  For each it gives the preprocessing time t_pre
(one HIP event pair around steps 1-6 on the library's stream), the
end-to-end time of one ``hull2d_async`` call (host clock, until the count
is read), the B_alg roofline fraction of t_pre and the per-stage split.

Prints one JSON line.  Further fields: the roofline of the dominant kernel,
the CPU oracle timed on the host, the batched workload against the plain
path, and the serving loop at several arrival rates against the plain path.
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
FLUSH_BYTES = 1 << 30
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1508_05488_amd", "csrc", "chainhull.hip")
# single-hull configurations timed one by one: name -> (distribution, n, seed, cold repetitions)
PER_CONFIG = (
    ("square_100k", "square", 100_000, 1, 21),
    ("square_20m", "square", 20_000_000, 2, 20),
    ("disk_20m", "disk", 20_000_000, 3, 20),
    ("gaussian_20m", "gaussian", 20_000_000, 4, 20),
    ("adversarial_20m", "adversarial", 20_000_000, 5, 20),
    ("adversarial_100m", "adversarial", 100_000_000, 6, 20),
)
# the paper's own figures, quoted as context only (other hardware)
PAPER_CONTEXT = {
    "claim": "5x-6x speedup over Qhull at 20M points (abstract, introduction, conclusion)",
    "hardware": "GTX 660M (Table 2) and GT 640 (Table 4), Kepler, 384 CUDA cores each, CUDA 5.5, "
                "with Intel i7-3610QM / i5-3470 hosts",
    "caveat": "the 20M random-square rows of Tables 2 and 4 give 4.01x and 4.07x; the 5x-6x come from the "
              "projected mesh sets (Tables 3 and 5)",
    "paper_20m_square_gpu_mpts_per_s": {"gtx660m": 34.4, "gt640": 36.9},
    "paper_20m_square_total_ms": {"gtx660m": 587.4, "gt640": 544.4},
}


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
    ap.add_argument("--no-per-config", action="store_true", help="skip the per-configuration single-hull table")
    ap.add_argument("--configs", default="", help="comma-separated subset of the per-configuration names")
    ap.add_argument("--serve-rates", default="0.25,0.5,0.75,1.0,1.2",
                    help="arrival rates as fractions of the server's measured capacity")
    ap.add_argument("--serve-requests", type=int, default=1500)
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain per-set comparison of the batched measurement")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--profile-config", default="",
                    help="only run one per-configuration input (a PER_CONFIG name) --warmup + --steps times "
                         "through hull2d_async, for profiler traces of that input alone")
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


def b_alg(n, s1, s2) -> float:
    """Algorithmic bytes of steps 1-6: two passes over the points, each
    round-1 survivor record written and read once, each SPA survivor written."""
    return 16.0 * n + 24.0 * s1 + 12.0 * s2


def moved_bytes(n, st) -> float:
    """Bytes the path's kernels must move at least, from the call's counts:
    the points once; the open points written by the pass and read back; the
    sort records written, re-read and read by the per-bucket pass; the chain
    points written and read."""
    return 8.0 * n + 24.0 * st["open"] + 36.0 * st["candidates"] + 24.0 * float(sum(st["s2"]))


class Flusher:
    """Writes 1 GiB of device memory: the 256 MB last-level cache then holds
    none of an input, so the next repetition reads it from HBM."""

    def __init__(self, torch, dev):
        self.buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
        self.k = 0

    def __call__(self):
        self.k += 1
        self.buf.fill_(float(self.k))


def measure_per_config(ch, wl, torch, dev, args, flush, names):
    """Each single-hull configuration alone, cold (see the module docstring)."""
    out = {}
    stream = torch.cuda.current_stream()
    for name, dist, n, seed, reps in PER_CONFIG:
        if names and name not in names:
            continue
        print(f"bench: per-config {name}", file=sys.stderr, flush=True)
        pts = wl.generate(dist, n, seed)
        d = torch.from_numpy(pts).to(dev)
        o_b = torch.empty(n, dtype=torch.int32, device=dev)
        c_b = torch.zeros(1, dtype=torch.int32, device=dev)
        o_a = torch.empty(n, dtype=torch.int32, device=dev)
        c_a = torch.zeros(1, dtype=torch.int32, device=dev)
        for _ in range(3):
            ch.hull2d_into(d, o_b, c_b, stream)
            ch.hull2d_async(d, o_a, c_a, stream)
        torch.cuda.synchronize()
        # t_pre: one event pair around steps 1-6 (and one around the finish)
        ch.set_timing(2)
        t_pre, t_fin = [], []
        for _ in range(reps):
            flush()
            rc = ch.hull2d_into(d, o_b, c_b, stream)
            if rc != ch.CH_OK:
                raise ch.ChainHullError(rc, f"hull2d {name}")
            st = ch.last_stats()
            t_pre.append(st["ms_pre"])
            t_fin.append(st["ms_finish"])
        ch.set_timing(0)
        torch.cuda.synchronize()
        # t_e2e: one hull2d_async call, until its count is on the host
        t_e2e, redo = [], 0
        for _ in range(reps):
            flush()
            c_a.fill_(-7)
            torch.cuda.synchronize()
            a = time.perf_counter()
            rc = ch.hull2d_async(d, o_a, c_a, stream)
            if rc != ch.CH_OK:
                raise ch.ChainHullError(rc, f"hull2d_async {name}")
            c = int(c_a.item())
            if c == ch.CH_BATCH_REDO:
                redo += 1
                rc = ch.hull2d_into(d, o_a, c_a, stream)
                if rc != ch.CH_OK:
                    raise ch.ChainHullError(rc, f"hull2d {name}")
                c = int(c_a.item())
            t_e2e.append(time.perf_counter() - a)
        cb = int(c_b.item())
        same = int(c_a.item()) == cb and torch.equal(o_a[:cb], o_b[:cb])
        # the stage split (every stage bracketed by events), cold
        flush()
        ch.set_timing(1)
        ch.hull2d_into(d, o_b, c_b, stream)
        st1 = ch.last_stats()
        ch.set_timing(0)
        # exact round-1 and SPA counts (outside the timed calls)
        _, pst = ch.polygon(d)
        torch.cuda.synchronize()
        tp = float(np.median(t_pre))
        te = float(np.median(t_e2e)) * 1e3
        s1, s2 = int(sum(pst["s1"])), int(sum(pst["s2"]))
        ba = b_alg(n, s1, s2)
        mv = moved_bytes(n, st1)
        out[name] = {
            "n": n, "seed": seed, "input_sha256_16": sha16(pts), "reps": reps,
            "t_pre_us": round(tp * 1e3, 2), "t_pre_us_p10_p90": [round(float(np.percentile(t_pre, q)) * 1e3, 2)
                                                                for q in (10, 90)],
            "t_finish_us": round(float(np.median(t_fin)) * 1e3, 2),
            "t_e2e_us": round(te * 1e3, 2),
            "mpts_per_s_e2e": round(n / te / 1e3, 1),
            "mpts_per_s_pre": round(n / tp / 1e3, 1),
            "b_alg_bytes": ba, "b_alg_frac": round(ba / (tp * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "moved_bytes": mv, "moved_frac": round(mv / (tp * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "hull": cb, "polygon": st1["polygon"], "open": st1["open"], "candidates": st1["candidates"],
            "s1": s1, "s2": s2, "device_finish": st1["device_finish"], "async_redo": redo,
            "async_equals_blocking": bool(same),
            "stages_us": {k: round(v * 1e3, 2) for k, v in st1["ms"].items()},
        }
        del d, o_a, o_b
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
    """Hull requests arriving as a Poisson stream, sizes log-uniform in
    [1e4, 2e7], each uniform square, disk or Gaussian, served by the
    continuous-batching server with a 288 GB budget.  The requests cycle
    through a pool of 48 seeded inputs resident in HBM (about 1 GB, four
    times the last-level cache, so a request's points are not cached from
    its previous turn).  First the server's closed-loop capacity (all
    requests submitted at once); then, at each arrival rate of a sweep
    (fractions of that capacity), the server and the plain path (one
    blocking hull2d at a time, in arrival order) on the same arrival
    times.  Latency is from arrival to completion."""
    import threading
    rng = np.random.default_rng(SERVE_SEED)
    names = ("square", "disk", "gaussian")
    sizes = np.floor(np.exp(rng.uniform(np.log(SERVE_LO), np.log(SERVE_HI), size=SERVE_POOL))).astype(np.int64)
    pool = [torch.from_numpy(wl.generate(names[k % 3], int(n), SERVE_SEED * 1000 + k)).to(dev)
            for k, n in enumerate(sizes)]
    pool_bytes = int(8 * sizes.sum())
    nreq = args.serve_requests
    order = np.arange(nreq) % SERVE_POOL
    unit_gaps = rng.exponential(1.0, size=nreq)
    pts_total = int(sum(int(sizes[k]) for k in order))

    # closed-loop capacity: the same requests all submitted at once
    with ch.Server(workers=args.serve_workers, mem_budget=288 << 30) as srv:
        for p in pool[:8]:
            srv.wait(srv.submit(p))
        t0 = time.perf_counter()
        tk = [srv.submit(pool[order[k]]) for k in range(min(nreq, 8 * SERVE_POOL))]
        for t in tk:
            srv.wait(t)
        cap = len(tk) / (time.perf_counter() - t0)

    def run_server(rate):
        gaps = unit_gaps / rate
        lat = []
        with ch.Server(workers=args.serve_workers, mem_budget=288 << 30) as srv:
            for p in pool[:8]:  # warm the workers' workspaces
                srv.wait(srv.submit(p))
            tickets = []

            def waiter():
                k = 0
                while k < nreq:
                    if k < len(tickets):
                        lat.append(srv.wait(tickets[k])[1])
                        k += 1
                    else:
                        time.sleep(0)

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

    out = torch.empty(int(sizes.max()), dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    lib = ch.lib()

    def run_plain(rate):
        gaps = unit_gaps / rate
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
        return np.array(plat) * 1e3, time.perf_counter() - t0

    sweep = []
    for frac in [float(x) for x in args.serve_rates.split(",") if x]:
        rate = frac * cap
        print(f"bench: serving at {rate:.0f} requests/s", file=sys.stderr, flush=True)
        lat, elapsed, st = run_server(rate)
        plat, pel = run_plain(rate)
        sweep.append({
            "rate_fraction_of_capacity": frac, "arrival_rate": round(rate, 1),
            "server": {"hulls_per_s": round(nreq / elapsed, 1), "mpts_per_s": round(pts_total / elapsed / 1e6, 1),
                       "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
                       "latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
                       "batches": st["batches"], "batched_requests": st["batched_requests"],
                       "single_requests": st["single_requests"], "max_inflight": st["max_inflight"]},
            "plain_path": {"hulls_per_s": round(nreq / pel, 1),
                           "latency_ms_p50": round(float(np.percentile(plat, 50)), 4),
                           "latency_ms_p99": round(float(np.percentile(plat, 99)), 4)},
        })
    del pool, out
    torch.cuda.empty_cache()
    return {
        "workload": f"Poisson arrivals, sizes log-uniform in [{SERVE_LO}, {SERVE_HI}], uniform square, disk or "
                    f"Gaussian (a pool of {SERVE_POOL} seeded requests in HBM, {pool_bytes / 1e9:.2f} GB, cycled); "
                    f"{args.serve_workers} worker streams; 288 GB admission budget; {nreq} requests per rate",
        "requests_per_rate": nreq,
        "points_per_rate": pts_total,
        "capacity_hulls_per_s": round(cap, 1),
        "sweep": sweep,
        "note": "plain path: one blocking hull2d call at a time in arrival order, same arrival times",
    }


def profile_config(ch, wl, torch, dev, args):
    """One per-configuration input alone, for a profiler: --warmup + --steps
    hull2d_async calls, one synchronisation at the end; prints one JSON line
    naming it."""
    cfg = {c[0]: c for c in PER_CONFIG}.get(args.profile_config)
    if cfg is None:
        raise SystemExit(f"unknown configuration {args.profile_config!r}; one of {[c[0] for c in PER_CONFIG]}")
    name, dist, n, seed, _ = cfg
    d = torch.from_numpy(wl.generate(dist, n, seed)).to(dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    for _ in range(args.warmup + args.steps):
        rc = ch.hull2d_async(d, out, cnt)
        if rc != ch.CH_OK:
            raise ch.ChainHullError(rc, f"hull2d_async {name}")
    torch.cuda.synchronize()
    print(json.dumps({"profile_config": name, "n": n, "calls": args.warmup + args.steps, "hull": int(cnt.item())}))


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
    if args.profile_config:
        profile_config(ch, wl, torch, dev, args)
        return
    n = args.n
    host = {d: wl.generate(d, n, seed) for d, seed in DISTS}
    inputs = {d: torch.from_numpy(host[d]).to(dev) for d, _ in DISTS}
    outs = {d: (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(1, dtype=torch.int32, device=dev))
            for d, _ in DISTS}
    stream = torch.cuda.current_stream()
    print("bench: headline steps", file=sys.stderr, flush=True)

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
    acnt.fill_(-7)
    for d, _ in DISTS:
        aout[d].fill_(-7)
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

    def clear_multi():
        mcnt.fill_(-7)
        for d, _ in DISTS:
            mout[d].fill_(-7)
        torch.cuda.synchronize()

    def check_multi(what):
        for k, (d, _) in enumerate(DISTS):
            c = int(outs[d][1].item())
            if int(mcnt[k].item()) != c or not torch.equal(mout[d][:c], outs[d][0][:c]):
                raise RuntimeError(f"{what} and hull2d differ on {d}")

    for _ in range(args.warmup):
        step_streams()
    clear_multi()
    t0m = time.perf_counter()
    for _ in range(args.steps):
        step_streams()
    torch.cuda.synchronize()
    t1m = time.perf_counter()
    elapsed_streams = t1m - t0m
    check_multi("hull2d_async on three streams")
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
    # the replays below must write every result again: clear them first
    clear_multi()
    t0g = time.perf_counter()
    for _ in range(args.steps):
        step_graph()
    torch.cuda.synchronize()
    t1g = time.perf_counter()
    elapsed_graph = t1g - t0g
    check_multi("the graph of three hull2d_async streams")
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

    # the autotuner's launch shapes (a file under tuning/ for this GPU, applied
    # when the library loaded) against the built-in defaults, on the queued
    # path: the same steps again with the defaults
    try:
        key = ch.device_key()
    except Exception as e:  # (reported, not fatal)
        key = repr(e)
    tuning = {"source": os.path.relpath(ch.tuning_source(), ROOT) if ch.tuning_source() else None,
              "device_key": key, "note": ch.tuning_note(),
              "shapes_20m": ch.get_tuning(n), "default_shapes": ch.get_tuning(-1)}
    if ch.tuning_source():
        ch.clear_tuning()
        for _ in range(args.warmup):
            step_async()
        torch.cuda.synchronize()
        t0d = time.perf_counter()
        for _ in range(args.steps):
            step_async()
        torch.cuda.synchronize()
        t1d = time.perf_counter()
        ch.load_tuning(ch.tuning_source())
        tuning["hull2d_async_tuned_mpts_per_s"] = round(value_async, 2)
        tuning["hull2d_async_default_mpts_per_s"] = round(total_pts / (t1d - t0d) / 1e6, 2)

    # timed region 2: the same steps with HIP events recorded by the library
    # on the call's stream around every stage
    ch.set_timing(True)
    stats = {d: [] for d, _ in DISTS}
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step(stats)
    torch.cuda.synchronize()
    ch.set_timing(False)
    stage_ms = {}
    for key in ch.STAGES:
        stage_ms[key] = float(np.mean([s["ms"][key] for d, _ in DISTS for s in stats[d]]))

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

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        from oracle import hull as oracle
        per = []
        for d, _ in DISTS:
            t = []
            for _ in range(3):
                a = time.perf_counter()
                oracle.hull(host[d])
                t.append(time.perf_counter() - a)
            per.append(float(np.median(t)))
        tc = float(sum(per))
        cpu = {"value": round(n * len(DISTS) / tc / 1e6, 3), "unit": "Mpts/s", "cores": 1, "kind": "oracle",
               "sample": f"the single-threaded C oracle on each of the three {n}-point inputs, median of 3 runs "
                         f"each ({tc:.1f} s for the three medians); host CPU {cpu_model()}, "
                         f"{os.cpu_count()} logical CPUs"}
    del inputs, outs, aout
    torch.cuda.empty_cache()

    flush = Flusher(torch, dev)
    per_config = None
    if not args.no_per_config:
        names = [x for x in args.configs.split(",") if x]
        per_config = measure_per_config(ch, wl, torch, dev, args, flush, names)
    del flush
    torch.cuda.empty_cache()

    batched = None
    if not args.no_batched:
        print("bench: batched", file=sys.stderr, flush=True)
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
                                   "note": "three calls queued on one stream per step, one synchronisation when "
                                           "the counts are read"},
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
        "tuning": tuning,
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "per_config": per_config,
        "paper_context": PAPER_CONTEXT,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
