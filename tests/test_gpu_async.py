"""hull2d_async (every step on the device, nothing synchronised): its
results equal hull2d's and, where the oracle finishes in seconds, the
oracle's; several calls queued back to back on one stream; the count code
for an out-of-domain input; polygons beyond one workgroup (points on a
circle, up to the 20M adversarial input) finished by the wide device
finish; a HIP graph of the call replayed on new inputs.  Each case prints its name
before its GPU calls."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1508_05488_amd as ch  # noqa: E402
from oracle import hull as oracle  # noqa: E402
from paper_1508_05488_amd import workloads as wl  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run_async(d, stream=None):
    out = torch.full((max(d.shape[0], 1),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    assert ch.hull2d_async(d, out, cnt, stream=stream) == ch.CH_OK
    return out, cnt


@pytest.mark.parametrize("dist,n,seed", [("square", 100_000, 301), ("disk", 100_000, 302),
                                         ("gaussian", 100_000, 303), ("square", 2_000_003, 304),
                                         ("disk", 1_000_001, 305), ("gaussian", 3_000_000, 306)])
def test_async_equals_blocking_and_oracle(dist, n, seed):
    pts = wl.generate(dist, n, seed)
    d = torch.from_numpy(pts).cuda()
    say(f"  hull2d_async {dist} n={n}")
    out, cnt = run_async(d)
    torch.cuda.synchronize()
    c = int(cnt.item())
    assert c > 0, c
    ref = ch.hull2d(d).cpu().numpy()
    assert np.array_equal(out[:c].cpu().numpy(), ref)
    if n <= 100_000:
        assert np.array_equal(ref, oracle.hull(pts))


def test_async_small_and_degenerate():
    cases = [np.zeros((0, 2), np.float32), np.array([[3, 4]], np.float32),
             np.array([[3, 4], [3, 4]], np.float32), np.array([[1, 1], [5, 5], [9, 9]], np.float32),
             np.full((1000, 2), 12345, np.float32),
             np.stack([np.arange(700) % 13, np.arange(700) % 13], 1).astype(np.float32),
             wl.generate("square", 3, 311), wl.generate("disk", 257, 312), wl.generate("gaussian", 4097, 313)]
    for k, pts in enumerate(cases):
        say(f"  hull2d_async small case {k} (n={pts.shape[0]})")
        d = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
        out, cnt = run_async(d)
        torch.cuda.synchronize()
        c = int(cnt.item())
        assert c >= 0, (k, c)
        assert np.array_equal(out[:c].cpu().numpy(), oracle.hull(pts)), k


def test_async_queued_back_to_back():
    inputs = [wl.generate(dist, n, 320 + k) for k, (dist, n) in
              enumerate([("square", 1_500_000), ("gaussian", 40_000), ("disk", 2_500_000), ("square", 7),
                         ("gaussian", 2_000_000)])]
    dev = [torch.from_numpy(p).cuda() for p in inputs]
    refs = [ch.hull2d(d).cpu().numpy() for d in dev]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    say("  hull2d_async: five calls queued on one stream")
    with torch.cuda.stream(s):
        res = [run_async(d, stream=s) for d in dev]
    s.synchronize()
    for k, ((out, cnt), ref) in enumerate(zip(res, refs)):
        c = int(cnt.item())
        assert np.array_equal(out[:c].cpu().numpy(), ref), k


def test_async_domain_error_and_wide_finish():
    bad = wl.generate("square", 50_000, 331)
    bad[777, 1] = 0.5
    say("  hull2d_async: out-of-domain coordinate")
    _, cnt = run_async(torch.from_numpy(bad).cuda())
    torch.cuda.synchronize()
    assert int(cnt.item()) == ch.CH_EDOMAIN
    # many points on a circle: a polygon beyond one workgroup, finished by
    # the wide device finish
    for n, seed in ((2_000_000, 332), (700_001, 334)):
        big = wl.generate("adversarial", n, seed)
        d = torch.from_numpy(big).cuda()
        say(f"  hull2d_async: adversarial n={n} (wide finish)")
        out, cnt = run_async(d)
        torch.cuda.synchronize()
        c = int(cnt.item())
        assert c > 0, c
        assert np.array_equal(out[:c].cpu().numpy(), oracle.hull(big))
    # the workspace serves a good call after both
    good = wl.generate("disk", 300_000, 333)
    out, cnt = run_async(torch.from_numpy(good).cuda())
    torch.cuda.synchronize()
    c = int(cnt.item())
    assert np.array_equal(out[:c].cpu().numpy(), oracle.hull(good))


@pytest.mark.timeout(300)
def test_async_adversarial_20m_against_oracle():
    pts = wl.workload("adversarial_20m")
    d = torch.from_numpy(pts).cuda()
    say("  hull2d_async adversarial_20m")
    out, cnt = run_async(d)
    torch.cuda.synchronize()
    c = int(cnt.item())
    assert c > 0, c
    got = out[:c].cpu().numpy()
    say("  oracle adversarial_20m")
    assert np.array_equal(got, oracle.hull(pts))


def test_async_graph_replays():
    n = 1_000_000
    seeds = (341, 342, 343, 344)
    inputs = [wl.generate(("square", "disk", "gaussian", "adversarial")[k], n, s) for k, s in enumerate(seeds)]
    d = torch.from_numpy(inputs[0]).cuda()
    out = torch.zeros(n, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    say("  hull2d_async: warm-up and capture")
    with torch.cuda.stream(s):  # warm-up outside the capture: the workspace exists
        assert ch.hull2d_async(d, out, cnt, stream=s) == ch.CH_OK
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rc = ch.hull2d_async(d, out, cnt, stream=s)
    assert rc == ch.CH_OK
    for rep, pts in enumerate(inputs * 2):
        d.copy_(torch.from_numpy(pts))
        out.zero_()
        cnt.fill_(-7)
        ref = ch.hull2d(d).cpu().numpy()  # eager work between the replays
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        c = int(cnt.item())
        assert np.array_equal(out[:c].cpu().numpy(), ref), rep


def test_async_three_stream_graph_replays():
    # one call per input on its own stream, the fork and join captured in one
    # graph, as the benchmark replays it
    n = 1_000_000
    kinds = ("square", "disk", "gaussian")
    d = [torch.from_numpy(wl.generate(kinds[k], n, 351 + k)).cuda() for k in range(3)]
    outs = [torch.zeros(n, dtype=torch.int32, device="cuda") for _ in range(3)]
    cnt = torch.zeros(3, dtype=torch.int32, device="cuda")
    streams = [torch.cuda.Stream() for _ in range(3)]
    cur = torch.cuda.current_stream()
    say("  hull2d_async on three streams: warm-up and capture")

    def fork_join(base):
        for k in range(3):
            streams[k].wait_stream(base)
            assert ch.hull2d_async(d[k], outs[k], cnt[k:k + 1], streams[k]) == ch.CH_OK
        for st in streams:
            base.wait_stream(st)

    fork_join(cur)  # warm-up: the workspaces exist before the capture
    torch.cuda.synchronize()
    cap = torch.cuda.Stream()
    cap.wait_stream(cur)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cap):
        fork_join(torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(4):
        pts = [wl.generate(kinds[(k + rep) % 3], n, 360 + 3 * rep + k) for k in range(3)]
        for k in range(3):
            d[k].copy_(torch.from_numpy(pts[k]))
            outs[k].zero_()
        cnt.fill_(-7)
        refs = [ch.hull2d(x).cpu().numpy() for x in d]  # eager work between the replays
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        c = cnt.cpu().numpy()
        for k in range(3):
            assert np.array_equal(outs[k][:c[k]].cpu().numpy(), refs[k]), (rep, k)
    del g
    torch.cuda.synchronize()
    for st in streams:
        ch.release_stream(st)


def test_captured_workspace_does_not_move():
    # a graph holds the stream's workspace addresses: from the capture on, a
    # call that would grow the workspace is refused until the stream is
    # released; under capture a call that would allocate is refused
    small = torch.from_numpy(wl.generate("disk", 200_000, 371)).cuda()
    big = torch.from_numpy(wl.generate("disk", 3_000_000, 372)).cuda()
    out = torch.zeros(3_000_000, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    ch.release_stream(s)  # (torch reuses streams: no workspace of an earlier test)
    say("  hull2d_async: under capture, a call on a stream without a workspace is refused")
    g0 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g0, stream=s):
        cnt.fill_(-3)  # (a kernel, so that the graph is not empty)
        rc = ch.hull2d_async(small, out, cnt, stream=s)
    assert rc == ch.CH_EINVAL
    del g0
    say("  hull2d_async: warm-up, capture, then a larger call")
    assert ch.hull2d_async(small, out, cnt, stream=s) == ch.CH_OK
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        assert ch.hull2d_async(small, out, cnt, stream=s) == ch.CH_OK
    assert ch.hull2d_async(big, out, cnt, stream=s) == ch.CH_EINVAL
    cnt.fill_(-7)
    g.replay()
    torch.cuda.synchronize()
    c = int(cnt.item())
    assert np.array_equal(out[:c].cpu().numpy(), ch.hull2d(small).cpu().numpy())
    del g
    torch.cuda.synchronize()
    ch.release_stream(s)
    say("  hull2d_async: after the release the larger call runs")
    assert ch.hull2d_async(big, out, cnt, stream=s) == ch.CH_OK
    s.synchronize()
    c = int(cnt.item())
    assert np.array_equal(out[:c].cpu().numpy(), ch.hull2d(big).cpu().numpy())
    ch.release_stream(s)
