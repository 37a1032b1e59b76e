"""Per-phase time of the batched kernel (k_batch_hull).

A second build of the library, compiled with ``CH_PHASE_TIMING``, makes
every workgroup of the batched kernel read the 100 MHz real-time counter at
its phase boundaries (the list or the stream, the quadrilateral, the exact
regions and slot filter, the sort, SPA, the polygon, the pre-hull rounds and
finish) and add the differences to device counters; ``chainhull_phase_ticks``
reads and clears them.  The product library is not instrumented.

    python -m paper_1508_05488_amd.phase_timing --build        # here (hipcc)
    python -m paper_1508_05488_amd.phase_timing                # on the GPU

The run times the batched path on the benchmark's 4096-set workload (one
call) and the list mode (the batched kernel on k_stream's open lists) on
20M-point uniform square and Gaussian inputs and a 100K-point square, and
prints the mean time per set and phase.
"""
from __future__ import annotations

import argparse
import ctypes
import os
import subprocess

from . import build as _build

PHASES = ("list/stream", "quad", "regions+filter", "sort", "spa", "polygon", "finish")
LIB = os.path.join(_build.LIBDIR, "libchainhull_phases.so")


def build_instrumented(verbose: bool = False) -> str:
    os.makedirs(_build.LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [_build.hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-DCH_PHASE_TIMING",
           "-Wall", "-Wno-unused-function", "-I", _build.INCLUDE, "-I", _build.CSRC, "-o", tmp]
    cmd += [os.path.join(_build.CSRC, s) for s in _build.SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _report(label: str, ticks, base: int, sets_slot: int) -> None:
    sets = int(ticks[sets_slot])
    if sets == 0:
        print(f"{label}: no set finished on the device")
        return
    us = [ticks[base + k] * 0.01 / sets for k in range(len(PHASES))]
    parts = "  ".join(f"{p} {u:.2f}" for p, u in zip(PHASES, us))
    print(f"{label}: {sets} sets, us per set: {parts}  | total {sum(us):.2f}")


def run() -> None:
    import torch

    from . import workloads as wl
    import paper_1508_05488_amd as ch

    if not os.path.exists(LIB):
        raise SystemExit(f"{LIB} is missing: build it with --build first")
    ch.LIB_PATH = LIB
    lib = ch.lib()
    lib.chainhull_phase_ticks.argtypes = [ctypes.POINTER(ctypes.c_ulonglong)]
    ticks = (ctypes.c_ulonglong * 18)()

    def take():
        rc = lib.chainhull_phase_ticks(ticks)
        if rc != 0:
            raise ch.ChainHullError(rc, "chainhull_phase_ticks")
        return list(ticks)

    dev = "cuda"
    # the batched path: the benchmark's 4096 sets, one warm call, then one timed
    pts, offs, _ = wl.batched_sets(4096, 1_000, 1_000_000, 7)
    d = torch.from_numpy(pts).to(dev)
    ch.hull2d_batched(d, offs)
    torch.cuda.synchronize()
    take()
    ch.hull2d_batched(d, offs)
    torch.cuda.synchronize()
    _report("batched, 4096 sets (1e3..1e6 points)", take(), 0, 16)
    del d
    # the list mode
    for dist, n, seed in (("square", 20_000_000, 2), ("gaussian", 20_000_000, 4), ("square", 100_000, 1)):
        d = torch.from_numpy(wl.generate(dist, n, seed)).to(dev)
        o = torch.empty(n, dtype=torch.int32, device=dev)
        c = torch.zeros(1, dtype=torch.int32, device=dev)
        ch.hull2d_async(d, o, c)
        torch.cuda.synchronize()
        take()
        for _ in range(5):
            ch.hull2d_async(d, o, c)
        torch.cuda.synchronize()
        _report(f"list mode, {dist} {n}", take(), 8, 17)
        del d


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--build", action="store_true", help="build the instrumented library (hipcc) and exit")
    a = ap.parse_args()
    if a.build:
        print(build_instrumented(verbose=True))
    else:
        run()


if __name__ == "__main__":
    main()
