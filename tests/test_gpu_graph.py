"""The batched kernel captured in a HIP graph (hull2d_batched_async):
every replay, with new inputs copied into the captured buffers and eager
work between the replays, equals the oracle per set.  Each case prints its
name before its GPU calls."""
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


def batch(seed, sizes):
    """Sets of the given sizes (same layout for every seed)."""
    parts = [wl.generate(("square", "disk", "gaussian")[k % 3], int(n), seed * 100 + k) for k, n in enumerate(sizes)]
    offs = np.zeros(len(parts) + 1, np.int64)
    offs[1:] = np.cumsum(sizes)
    return np.ascontiguousarray(np.concatenate(parts)), offs, parts


def check(parts, offs, out, cnt, what):
    c = cnt.cpu().numpy()
    o = out.cpu().numpy()
    for s, p in enumerate(parts):
        assert c[s] >= 0, f"{what}: set {s} count {c[s]}"
        assert np.array_equal(o[offs[s]:offs[s] + c[s]], oracle.hull(p)), f"{what}: set {s}"


def test_async_matches_oracle_and_sync():
    rng = np.random.default_rng(121)
    sizes = np.floor(np.exp(rng.uniform(np.log(1e3), np.log(3e5), size=40))).astype(np.int64)
    pts, offs, parts = batch(1, sizes)
    d_pts = torch.from_numpy(pts).cuda()
    d_offs = torch.from_numpy(offs).cuda()
    order = torch.from_numpy(np.argsort(-sizes, kind="stable").astype(np.int32)).cuda()
    out = torch.zeros(pts.shape[0], dtype=torch.int32, device="cuda")
    cnt = torch.zeros(len(parts), dtype=torch.int32, device="cuda")
    say("  hull2d_batched_async eager, 40 sets")
    assert ch.hull2d_batched_async(d_pts, d_offs, order, out, cnt) == ch.CH_OK
    torch.cuda.synchronize()
    check(parts, offs, out, cnt, "eager")
    hulls, counts = ch.hull2d_batched(d_pts, offs)
    assert torch.equal(counts, cnt)
    # no order: the same results
    out2 = torch.zeros_like(out)
    cnt2 = torch.zeros_like(cnt)
    assert ch.hull2d_batched_async(d_pts, d_offs, None, out2, cnt2) == ch.CH_OK
    torch.cuda.synchronize()
    assert torch.equal(cnt2, cnt) and torch.equal(out2, out)


def test_async_reports_bad_offsets():
    pts = torch.from_numpy(wl.generate("square", 3000, 122)).cuda()
    offs = torch.tensor([0, 1000, 500, 3000], dtype=torch.int64, device="cuda")
    out = torch.zeros(3000, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(3, dtype=torch.int32, device="cuda")
    say("  hull2d_batched_async with a decreasing offset")
    assert ch.hull2d_batched_async(pts, offs, None, out, cnt) == ch.CH_OK
    c = cnt.cpu().numpy()
    assert c[1] == ch.CH_EINVAL
    assert c[0] > 0 and c[2] > 0


def test_graph_replays():
    rng = np.random.default_rng(123)
    sizes = np.floor(np.exp(rng.uniform(np.log(1e3), np.log(2e5), size=24))).astype(np.int64)
    pts, offs, parts = batch(2, sizes)
    d_pts = torch.from_numpy(pts).cuda()
    d_offs = torch.from_numpy(offs).cuda()
    order = torch.from_numpy(np.argsort(-sizes, kind="stable").astype(np.int32)).cuda()
    out = torch.zeros(pts.shape[0], dtype=torch.int32, device="cuda")
    cnt = torch.zeros(len(parts), dtype=torch.int32, device="cuda")
    say("  hull2d_batched_async: capture")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside the capture
        assert ch.hull2d_batched_async(d_pts, d_offs, order, out, cnt, stream=s) == ch.CH_OK
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rc = ch.hull2d_batched_async(d_pts, d_offs, order, out, cnt, stream=torch.cuda.current_stream())
    assert rc == ch.CH_OK
    for rep, seed in enumerate((2, 3, 4)):
        new_pts, _, new_parts = batch(seed, sizes)
        d_pts.copy_(torch.from_numpy(new_pts))  # new inputs in the captured buffer
        out.zero_()
        cnt.zero_()
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        check(new_parts, offs, out, cnt, f"replay {rep}")
