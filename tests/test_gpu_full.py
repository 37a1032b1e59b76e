"""GPU parity at the paper-scale sizes.

20M points per distribution: every hull index against the C oracle, with
blocking hull2d calls, and with the benchmark's fastest configuration (one
hull2d_async call per input on three streams, captured in a HIP graph and
replayed).  100M adversarial points: against the oracle too (about a
minute of CPU), and a 100M-point constructed convex polygon whose hull is
known without an oracle.
"""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1508_05488_amd as ch  # noqa: E402
from oracle import hull as oracle  # noqa: E402
from paper_1508_05488_amd import workloads as wl  # noqa: E402
from hullcheck import polygon_with_extras  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run_gpu(pts, name):
    say(f"  hull2d {name} n={pts.shape[0]}: upload")
    t = torch.from_numpy(pts).cuda()
    say(f"  hull2d {name}: run")
    t0 = time.perf_counter()
    got = ch.hull2d(t).cpu().numpy()
    st = ch.last_stats()
    say(f"  hull2d {name}: {1e3 * (time.perf_counter() - t0):.1f} ms, hull {got.size}, "
        f"s1 {sum(st['s1'])}, candidates {st['candidates']}, s2 {sum(st['s2'])}")
    del t
    return got, st


@pytest.mark.parametrize("name", ["square_20m", "disk_20m", "gaussian_20m", "adversarial_20m"])
def test_paper_scale_against_oracle(name):
    say(f"  generate {name}")
    pts = wl.workload(name)
    got, st = run_gpu(pts, name)
    say(f"  oracle {name}")
    want = oracle.hull(pts)
    assert np.array_equal(got, want)
    assert st["candidates"] >= sum(st["s2"])


@pytest.mark.timeout(400)
def test_adversarial_100m_against_oracle():
    say("  generate adversarial_100m")
    pts = wl.workload("adversarial_100m")
    got, st = run_gpu(pts, "adversarial_100m")
    say("  oracle adversarial_100m (about a minute)")
    want = oracle.hull(pts)
    assert np.array_equal(got, want)


@pytest.mark.timeout(300)
def test_constructed_polygon_100m_known_hull():
    rng = wl.rng_for(81)
    say("  generate constructed polygon, 100M points")
    pts, want = polygon_with_extras(99_000_000, 500_000, 500_000, rng, scale=400_000, base=(7, 11), core=0.99)
    got, _ = run_gpu(pts, "polygon_100m")
    assert np.array_equal(got, want)


@pytest.mark.timeout(300)
def test_paper_scale_three_stream_graph():
    names = ("square_20m", "disk_20m", "gaussian_20m")
    host = [wl.workload(nm) for nm in names]
    say("  oracle on the three 20M inputs")
    want = [oracle.hull(p) for p in host]
    d = [torch.from_numpy(p).cuda() for p in host]
    n = host[0].shape[0]
    outs = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in names]
    cnt = torch.empty(len(names), dtype=torch.int32, device="cuda")
    streams = [torch.cuda.Stream() for _ in names]

    def fork_join(base):
        for k in range(len(names)):
            streams[k].wait_stream(base)
            assert ch.hull2d_async(d[k], outs[k], cnt[k:k + 1], streams[k]) == ch.CH_OK
        for st in streams:
            base.wait_stream(st)

    say("  three streams: warm-up and capture")
    fork_join(torch.cuda.current_stream())
    torch.cuda.synchronize()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cap):
        fork_join(torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:
            o.zero_()
        cnt.fill_(-7)
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        c = cnt.cpu().numpy()
        for k, nm in enumerate(names):
            assert np.array_equal(outs[k][:c[k]].cpu().numpy(), want[k]), (rep, nm)
    del g
    torch.cuda.synchronize()
    for st in streams:
        ch.release_stream(st)
