"""The small-input path (inputs of at most fused_max points): every step in
one workgroup of the batched kernel, and the single-hull kernels queued
behind it gated on its count, so that they run only for an input it leaves
(its LDS capacities exceeded).  Results against the oracle for hull2d,
hull2d_async and hull2d_noalloc at sizes from 1 point to just above the
threshold; an input the batched kernel leaves, through the gated kernels
(blocking, asynchronous, and in graph replays with eager work between
them); the threshold 0 turns the path off.  Each case prints its name before
its GPU calls."""
import contextlib
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1508_05488_amd as ch  # noqa: E402
from oracle import hull as oracle  # noqa: E402
from paper_1508_05488_amd import autotune  # noqa: E402
from paper_1508_05488_amd import workloads as wl  # noqa: E402

FUSED_MAX = 1 << 18


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@contextlib.contextmanager
def fused_max(v):
    base = ch.get_tuning(-1)
    ch.clear_tuning()
    ch.set_tuning(2**40, autotune.shape(base, fused_max=v))
    try:
        yield
    finally:
        ch.clear_tuning()
        ch.load_tuning()


def run_async(fn, d):
    out = torch.full((max(d.shape[0], 1),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    assert fn(d, out, cnt) == ch.CH_OK
    torch.cuda.synchronize()
    c = int(cnt.item())
    return out[:max(c, 0)].cpu().numpy(), c


@pytest.mark.parametrize("dist", ["square", "disk", "gaussian", "adversarial"])
@pytest.mark.parametrize("n", [1, 2, 3, 100, 4097, 65_537, FUSED_MAX, FUSED_MAX + 1])
def test_fused_sizes_against_oracle(dist, n):
    pts = wl.generate(dist, n, seed=901 + n % 13)
    want = oracle.hull(pts)
    d = torch.from_numpy(pts).cuda()
    with fused_max(FUSED_MAX):
        say(f"  hull2d {dist} n={n}")
        got = ch.hull2d(d).cpu().numpy()
        st = ch.last_stats()
        assert np.array_equal(got, want)
        if n > FUSED_MAX:
            assert not st["fused"]
        for name, fn in (("hull2d_async", ch.hull2d_async), ("hull2d_noalloc", ch.hull2d_noalloc)):
            say(f"  {name} {dist} n={n}")
            got, c = run_async(fn, d)
            assert c == want.size and np.array_equal(got, want), (name, c)


def circle_heavy(n, seed):
    # every point on a rounded circle: a hull far beyond the batched
    # kernel's polygon capacity, so that it leaves the set
    rng = wl.rng_for(seed)
    t = rng.uniform(0, 2 * np.pi, n)
    xy = np.clip(np.rint(wl.CENTER + wl.RADIUS * np.stack([np.cos(t), np.sin(t)], 1)), 0, wl.M)
    return np.ascontiguousarray(xy.astype(np.float32))


def test_input_left_by_the_batched_kernel():
    pts = circle_heavy(200_000, 911)
    want = oracle.hull(pts)
    assert want.size > 3584
    d = torch.from_numpy(pts).cuda()
    with fused_max(FUSED_MAX):
        say("  hull2d circle n=200000 (left to the single-hull kernels)")
        got = ch.hull2d(d).cpu().numpy()
        assert not ch.last_stats()["fused"]
        assert np.array_equal(got, want)
        for name, fn in (("hull2d_async", ch.hull2d_async), ("hull2d_noalloc", ch.hull2d_noalloc)):
            say(f"  {name} circle n=200000 (gated kernels run)")
            got, c = run_async(fn, d)
            assert c == want.size and np.array_equal(got, want), (name, c)


def test_fused_flag_and_threshold_zero():
    pts = wl.generate("square", 100_000, 921)
    want = oracle.hull(pts)
    d = torch.from_numpy(pts).cuda()
    with fused_max(FUSED_MAX):
        say("  hull2d square n=100000, small-input path")
        assert np.array_equal(ch.hull2d(d).cpu().numpy(), want)
        st = ch.last_stats()
        assert st["fused"] and st["device_finish"] and st["hull"] == want.size
    with fused_max(0):
        say("  hull2d square n=100000, threshold 0")
        assert np.array_equal(ch.hull2d(d).cpu().numpy(), want)
        st = ch.last_stats()
        assert not st["fused"] and st["open"] > 0


def test_fused_graph_replays_with_a_left_input():
    n = 200_000
    inputs = [wl.generate("square", n, 931), circle_heavy(n, 932), wl.generate("gaussian", n, 933),
              wl.generate("adversarial", n, 934)]
    wants = [oracle.hull(p) for p in inputs]
    with fused_max(FUSED_MAX):
        d = torch.from_numpy(inputs[0]).cuda()
        out = torch.zeros(n, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        say("  hull2d_async small-input path: warm-up and capture")
        with torch.cuda.stream(s):
            assert ch.hull2d_async(d, out, cnt, stream=s) == ch.CH_OK
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            rc = ch.hull2d_async(d, out, cnt, stream=s)
        assert rc == ch.CH_OK
        for rep, (pts, want) in enumerate(list(zip(inputs, wants)) * 2):
            d.copy_(torch.from_numpy(pts))
            out.zero_()
            cnt.fill_(-7)
            _ = ch.hull2d(d)  # eager work between the replays
            torch.cuda.synchronize()
            say(f"  replay {rep}")
            g.replay()
            torch.cuda.synchronize()
            c = int(cnt.item())
            assert c == want.size and np.array_equal(out[:c].cpu().numpy(), want), rep
        del g
        ch.release_stream(s)


@contextlib.contextmanager
def list_max(v):
    base = ch.get_tuning(-1)
    ch.clear_tuning()
    ch.set_tuning(2**40, autotune.shape(base, list_max=v))
    try:
        yield
    finally:
        ch.clear_tuning()
        ch.load_tuning()


@pytest.mark.parametrize("dist,n,seed", [("gaussian", 3_000_000, 941), ("square", 5_000_000, 942),
                                         ("disk", 300_000, 943)])
def test_list_mode_on_large_inputs(dist, n, seed):
    # few open points after the pass over a large input: one workgroup takes
    # every later step from k_stream's lists (or leaves the input to the
    # single-hull kernels when they are too many)
    pts = wl.generate(dist, n, seed)
    want = oracle.hull(pts)
    d = torch.from_numpy(pts).cuda()
    say(f"  hull2d {dist} n={n} (list mode)")
    got = ch.hull2d(d).cpu().numpy()
    st = ch.last_stats()
    assert np.array_equal(got, want)
    assert st["device_finish"] and st["open"] > 0
    got, c = run_async(ch.hull2d_async, d)
    assert c == want.size and np.array_equal(got, want)
    with list_max(0):
        say(f"  hull2d {dist} n={n} (single-hull kernels)")
        assert np.array_equal(ch.hull2d(d).cpu().numpy(), want)
