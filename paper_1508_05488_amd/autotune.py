"""Autotuner of the library's launch shapes (ch_tuning in include/chainhull.h).

The paper fixes its block size by the GPU generation and notes that the best
amount of work per thread depends on the input size, the survivors and the
GPU, and needs experiments (Sections 2.2.2, 4.3).  This module runs those
experiments on the current GPU: for each size class it times every candidate
shape of the single-hull path (k_stream grid and loads in flight, open
points per k_cand workgroup, k_chain and k_finish_wide grids) on seeded
inputs of each distribution, checks that every candidate gives exactly the
default shape's hulls (a shape never changes a result), and keeps the
fastest (with the small-input path off, so that the single-hull kernels
themselves are timed); then the batched kernel's loads in flight and launch
order on a batch of sets; then two thresholds from one sweep of sizes: the
small-input path's (the largest size up to which the batched kernel's one
workgroup, with the single-hull kernels gated behind it, is not slower than
the single-hull kernels) and the serving one (the largest request for which
one workgroup of the batched kernel is at most ``SERVE_RATIO`` times slower
than the whole device).  The result is a JSON file under ``tuning/``, keyed
by the GPU, that the binding applies when the library loads.

    python -m paper_1508_05488_amd.autotune [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1508_05488_amd as ch  # noqa: E402
from paper_1508_05488_amd import workloads as wl  # noqa: E402

# size classes: (largest n of the class, n timed)
CLASSES = ((300_000, 100_000), (4_000_000, 2_000_000), (2**31 - 1, 20_000_000))
DISTS = ("square", "disk", "gaussian", "adversarial")
SERVE_RATIO = 1.5
FLUSH_BYTES = 1 << 30


def candidates(quick: bool = False):
    """Every single-hull shape the autotuner tries (the defaults among them)."""
    grids = (256, 512, 1024)
    unrolls = (2, 4)
    per_row = (1024, 2048, 4096, 8192)
    chain = (256, 1024)
    wide = (512, 1024, 2048)
    if quick:
        grids, unrolls, per_row, chain, wide = (512, 1024), (4,), (2048, 4096), (1024,), (1024,)
    return [{"stream_grid": g, "stream_unroll": u, "cand_per_row": r, "chain_grid": c, "wide_grid": w}
            for g, u, r, c, w in itertools.product(grids, unrolls, per_row, chain, wide)]


def shape(base: dict, **kw) -> dict:
    t = dict(base)
    t.update(kw)
    return t


class Timer:
    """Median wall time of a stream-ordered call, inputs evicted from the
    last-level cache before each repetition when they would fit in it."""

    def __init__(self, torch, dev):
        self.torch = torch
        self.buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
        self.k = 0

    def flush(self):
        self.k += 1
        self.buf.fill_(float(self.k))

    def time(self, fn, reps: int, flush: bool) -> float:
        torch = self.torch
        s = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        fn()  # warm-up (workspace, code)
        for a, b in ev:
            if flush:
                self.flush()
            a.record(s)
            fn()
            b.record(s)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))


# A candidate replaces the default shapes only when it is this much faster
# over the four inputs (run-to-run timing noise is about 1 %).
KEEP_DEFAULT_MARGIN = 0.02


def tune_single(torch, dev, timer, quick: bool, log) -> list:
    classes = []
    default = ch.get_tuning(-1)
    for n_max, n in CLASSES:
        inputs = {d: torch.from_numpy(wl.generate(d, n, 500 + k)).to(dev) for k, d in enumerate(DISTS)}
        out = torch.empty(n, dtype=torch.int32, device=dev)
        cnt = torch.empty(1, dtype=torch.int32, device=dev)
        # the default shape's hulls: every candidate must reproduce them
        ch.clear_tuning()
        ch.set_tuning(2**40, shape(default, fused_max=0, list_max=0))
        ref = {}
        for d, x in inputs.items():
            assert ch.hull2d_async(x, out, cnt) == ch.CH_OK
            torch.cuda.synchronize()
            c = int(cnt.item())
            assert c > 0, (d, c)
            ref[d] = (c, out[:c].clone())
        reps = 5 if n >= 10_000_000 else 9
        flush = n * 8 < 512 << 20
        rows = []
        for cand in candidates(quick):
            t = shape(default, **cand, fused_max=0, list_max=0)  # (the single-hull kernels themselves)
            ch.clear_tuning()
            ch.set_tuning(n_max, t)
            ms, ok = {}, True
            for d, x in inputs.items():
                def call(x=x):
                    ch.hull2d_async(x, out, cnt)
                ms[d] = timer.time(call, reps, flush)
                c = int(cnt.item())
                same = c == ref[d][0] and bool(torch.equal(out[:c], ref[d][1]))
                ok = ok and same
            rows.append({"tuning": cand, "ms": ms, "total_ms": sum(ms.values()), "equal": ok})
            log(f"autotune n={n}: {cand} {sum(ms.values()):.4f} ms{'' if ok else ' MISMATCH'}")
        good = [r for r in rows if r["equal"]]
        bad = [r["tuning"] for r in rows if not r["equal"]]
        best = min(good, key=lambda r: r["total_ms"])
        dflt = next(r for r in rows if all(r["tuning"][k] == default[k] for k in r["tuning"]))
        if dflt["equal"] and best["total_ms"] > (1.0 - KEEP_DEFAULT_MARGIN) * dflt["total_ms"]:
            best = dflt  # (a gain within the timing noise keeps the defaults)
        classes.append({"n_max": n_max, "n_timed": n, "tuning": shape(default, **best["tuning"]),
                        "ms": best["ms"], "total_ms": best["total_ms"], "default_total_ms": dflt["total_ms"],
                        "candidates": len(rows), "mismatches": bad})
        del inputs
        torch.cuda.empty_cache()
    ch.clear_tuning()
    return classes


def tune_batched(torch, dev, timer, log, sets: int = 1024) -> dict:
    pts, offs, _ = wl.batched_sets(sets, 1_000, 1_000_000, seed=7)
    d = torch.from_numpy(pts).to(dev)
    base = ch.get_tuning(-1)
    res, ref = [], None
    for u, o in itertools.product((1, 2), (0, 1)):
        ch.clear_tuning()
        ch.set_tuning(2**62, shape(base, batch_unroll=u, batch_order=o))
        hulls, cnt = ch.hull2d_batched(d, offs)
        got = [h.cpu().numpy() for h in hulls]
        same = ref is None or all(np.array_equal(a, b) for a, b in zip(got, ref))
        ref = got if ref is None else ref
        t = timer.time(lambda: ch.hull2d_batched(d, offs), 5, False)
        res.append({"batch_unroll": u, "batch_order": o, "ms": t, "equal": same})
        log(f"autotune batched: unroll {u} order {o}: {t:.3f} ms{'' if same else ' MISMATCH'}")
    ch.clear_tuning()
    best = min((r for r in res if r["equal"]), key=lambda r: r["ms"])
    return {"sets": sets, "points": int(offs[-1]), "batch_unroll": best["batch_unroll"],
            "batch_order": best["batch_order"], "ms": best["ms"],
            "default_ms": next(r["ms"] for r in res if r["batch_unroll"] == base["batch_unroll"]
                               and r["batch_order"] == base["batch_order"]),
            "mismatches": [r for r in res if not r["equal"]]}


def tune_serving(torch, dev, timer, log) -> dict:
    """Per size n on the uniform disk: the single-hull kernels alone
    (fused_max 0), the small-input path (the batched kernel's one workgroup
    with the single-hull kernels gated behind it) and the batched kernel
    alone on the one set.  fused_max: the largest n for which the
    small-input path is not slower than the single-hull kernels;
    serve_batch_max: the largest n for which the batched kernel is at most
    SERVE_RATIO times slower than them."""
    sizes = [int(2 ** k) for k in np.arange(12, 22.5, 0.5)]
    rows, best_serve, best_fused = [], 4096, 0
    base = ch.get_tuning(-1)
    try:
        for m in sizes:
            pts = wl.generate("disk", m, 700 + m % 997)
            d = torch.from_numpy(pts).to(dev)
            out = torch.empty(m, dtype=torch.int32, device=dev)
            cnt = torch.empty(1, dtype=torch.int32, device=dev)
            offs_d = torch.tensor([0, m], dtype=torch.int64, device=dev)
            cnts = torch.empty(1, dtype=torch.int32, device=dev)
            ch.clear_tuning()
            ch.set_tuning(2**40, shape(base, fused_max=0))
            t_one = timer.time(lambda: ch.hull2d_async(d, out, cnt), 7, False)
            ch.clear_tuning()
            ch.set_tuning(2**40, shape(base, fused_max=1 << 22))
            t_fus = timer.time(lambda: ch.hull2d_async(d, out, cnt), 7, False)
            ch.clear_tuning()
            t_bat = timer.time(lambda: ch.hull2d_batched_async(d, offs_d, None, out, cnts), 7, False)
            rows.append({"n": m, "single_ms": t_one, "fused_ms": t_fus, "batched_ms": t_bat})
            log(f"autotune serving: n={m} single {t_one:.4f} ms fused {t_fus:.4f} ms batched {t_bat:.4f} ms")
            if t_bat <= SERVE_RATIO * t_one:
                best_serve = m
            if t_fus <= t_one and (len(rows) == 1 or best_fused == rows[-2]["n"]):
                best_fused = m  # (the sizes up to m all gain)
    finally:
        ch.clear_tuning()
    return {"serve_batch_max": int(min(best_serve, 1 << 22)), "fused_max": int(min(best_fused, 1 << 22)),
            "ratio": SERVE_RATIO, "sizes": rows}


def run(out_path: str | None = None, quick: bool = False, log=print) -> dict:
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the autotuner needs a GPU")
    dev = torch.device("cuda:0")
    ch.lib()
    timer = Timer(torch, dev)
    t0 = time.time()
    classes = tune_single(torch, dev, timer, quick, log)
    bat = tune_batched(torch, dev, timer, log)
    srv = tune_serving(torch, dev, timer, log)
    for c in classes:
        c["tuning"]["batch_unroll"] = bat["batch_unroll"]
        c["tuning"]["batch_order"] = bat["batch_order"]
        c["tuning"]["serve_batch_max"] = srv["serve_batch_max"]
        c["tuning"]["fused_max"] = srv["fused_max"]
    doc = {"device": ch.device_key(), "generated_unix": int(time.time()), "seconds": round(time.time() - t0, 1),
           "classes": classes, "batched": bat, "serving": srv}
    path = out_path or ch.tuning_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    log(f"autotune: wrote {path}")
    return doc


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=None, help="output JSON (default: tuning/<device>.json in the package)")
    ap.add_argument("--quick", action="store_true", help="a smaller candidate set")
    a = ap.parse_args()
    run(a.out, a.quick, log=lambda m: print(m, file=sys.stderr, flush=True))


if __name__ == "__main__":
    main()
