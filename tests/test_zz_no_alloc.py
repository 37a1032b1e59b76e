"""hull2d_noalloc (the entry point for callers that cannot allocate device
memory: every intermediate array in the library's fixed per-device buffer)
called through the C ABI: its counts and vertex indices equal
hull2d_async's on the same inputs, exactly, on calls in a row with the
buffer keeping the previous call's contents (a large input, then a
smaller one, then the largest allowed size, then a tiny one); the
oracle agrees where it finishes in seconds; a size beyond the buffer is
refused before any device work.  Each case prints its name before its GPU
calls."""
import ctypes
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


def call(fn, d):
    """One call of a C entry point on the current stream; the count and the
    hull indices after a synchronisation."""
    n = d.shape[0]
    out = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    rc = fn(ctypes.c_void_p(d.data_ptr()), ctypes.c_int64(n), ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(s))
    assert rc == ch.CH_OK, ch.strerror(rc)
    torch.cuda.synchronize()
    c = int(cnt.item())
    return c, out[:max(c, 0)].cpu().numpy()


CASES = [("disk", 1_000_000, 901), ("gaussian", 300_001, 902), ("square", ch.NOALLOC_MAX_POINTS, 903),
         ("adversarial", 30_000, 904), ("square", 5, 905), ("disk", 777, 906)]


def test_noalloc_equals_async_on_calls_in_a_row():
    L = ch.lib()
    for dist, n, seed in CASES:
        pts = wl.generate(dist, n, seed)
        d = torch.from_numpy(pts).cuda()
        say(f"  hull2d_noalloc {dist} n={n} seed={seed}")
        c0, h0 = call(L.hull2d_noalloc, d)
        say(f"  hull2d_async {dist} n={n} seed={seed}")
        c1, h1 = call(L.hull2d_async, d)
        assert c1 > 0 and c0 == c1, (c0, c1)
        assert np.array_equal(h0, h1)
        if n <= 300_001:
            assert np.array_equal(h0, oracle.hull(pts))


def test_noalloc_degenerate_and_refused():
    L = ch.lib()
    cases = [np.zeros((0, 2), np.float32), np.array([[3, 4]], np.float32),
             np.array([[1, 1], [5, 5], [9, 9]], np.float32), np.full((1000, 2), 12345, np.float32)]
    for k, pts in enumerate(cases):
        say(f"  hull2d_noalloc degenerate case {k} (n={pts.shape[0]})")
        d = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
        c, h = call(L.hull2d_noalloc, d)
        assert c == len(oracle.hull(pts)) and np.array_equal(h, oracle.hull(pts))
    # one point more than the buffer holds: refused on the host
    big = torch.zeros((ch.NOALLOC_MAX_POINTS + 1, 2), dtype=torch.float32, device="cuda")
    out = torch.empty(1, dtype=torch.int32, device="cuda")
    say("  hull2d_noalloc refuses n = max + 1")
    rc = L.hull2d_noalloc(ctypes.c_void_p(big.data_ptr()), ctypes.c_int64(big.shape[0]),
                          ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(out.data_ptr()), None)
    assert rc == ch.CH_ECAPACITY
