"""GPU parity of the batched path (one workgroup per set, device finish,
single-hull path for sets beyond its capacities) against the CPU oracle.

Every set's hull indices must match the oracle bit for bit.  Each case
prints its name before its GPU call.
"""
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


def batched_parity(parts, name):
    pts = np.ascontiguousarray(np.concatenate(parts).astype(np.float32)) if parts else np.zeros((0, 2), np.float32)
    offs = np.zeros(len(parts) + 1, np.int64)
    offs[1:] = np.cumsum([p.shape[0] for p in parts])
    say(f"  hull2d_batched {name}: {len(parts)} sets, {offs[-1]} points")
    hulls, counts = ch.hull2d_batched(torch.from_numpy(pts).cuda(), offs)
    for s, p in enumerate(parts):
        want = oracle.hull(p.astype(np.float32))
        got = hulls[s].cpu().numpy()
        assert np.array_equal(got, want), f"{name} set {s} (n={p.shape[0]}): got {got[:8]} ({got.size}) want {want[:8]} ({want.size})"


def test_degenerate_sets():
    parts = [
        np.zeros((0, 2)),
        np.array([[7, 9]]),
        np.array([[9, 9], [1, 2]]),
        np.full((1000, 2), 12345),
        np.stack([np.arange(500) % 97, np.full(500, 3)], 1),
        np.stack([np.full(500, 3), np.arange(500) % 97], 1),
        np.stack([np.arange(500) % 97, np.arange(500) % 97], 1),
        np.array([[0, 0], [wl.M, 0], [wl.M, wl.M], [0, wl.M], [5, 5]]),
        np.array([(x, y) for y in range(40) for x in range(40)]),
        np.zeros((0, 2)),
    ]
    batched_parity(parts, "degenerate")


def test_small_lattices():
    rng = wl.rng_for(91)
    parts = [wl.small_lattice(int(rng.integers(1, 300)), int(rng.choice([2, 3, 5, 33, 1 << 23])), rng)
             for _ in range(400)]
    batched_parity(parts, "lattices")


@pytest.mark.parametrize("hi", [5_000, 200_000, 1_000_000])
def test_mixed_distributions(hi):
    pts, offs, dists = wl.batched_sets(48, 1_000, hi, seed=92 + hi % 97)
    parts = [pts[offs[s]:offs[s + 1]] for s in range(len(dists))]
    batched_parity(parts, f"mixed up to {hi}")


def test_sets_beyond_workgroup_capacity():
    # a circle set has a hull vertex almost everywhere: its chain exceeds the
    # workgroup's polygon room and the set goes to the single-hull path
    circle = wl.generate("adversarial", 300_000, seed=93)
    theta = np.linspace(0, 2 * np.pi, 20_000, endpoint=False)
    ring = np.rint(4_000_000 + 3_000_000 * np.stack([np.cos(theta), np.sin(theta)], 1))
    parts = [wl.generate("square", 10_000, seed=94), circle, ring, wl.generate("disk", 50_000, seed=95)]
    batched_parity(parts, "beyond capacity")


def test_domain_error_in_one_set():
    good = wl.generate("square", 5_000, seed=96)
    bad = wl.generate("disk", 5_000, seed=97)
    bad[17, 1] = 0.5
    parts = [good, bad, good]
    pts = np.ascontiguousarray(np.concatenate(parts))
    offs = np.array([0, 5_000, 10_000, 15_000], np.int64)
    t = torch.from_numpy(pts).cuda()
    out = torch.zeros(15_000, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(3, dtype=torch.int32, device="cuda")
    say("  hull2d_batched domain error")
    rc = ch.lib().hull2d_batched(t.data_ptr(), offs.ctypes.data, 3, out.data_ptr(), cnt.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    assert rc == ch.CH_EDOMAIN
    c = cnt.cpu().numpy()
    assert c[1] == ch.CH_EDOMAIN
    want = oracle.hull(good)
    for s in (0, 2):
        assert np.array_equal(out[offs[s]:offs[s] + c[s]].cpu().numpy(), want)


def test_batched_repeat_is_deterministic():
    pts, offs, dists = wl.batched_sets(64, 1_000, 100_000, seed=98)
    t = torch.from_numpy(pts).cuda()
    say("  hull2d_batched repeat")
    a, ca = ch.hull2d_batched(t, offs)
    b, cb = ch.hull2d_batched(t, offs)
    assert torch.equal(ca, cb)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.timeout(300)
def test_benchmark_workload_sampled_sets():
    # the 4096-set workload the benchmark times (594M points, one call), the
    # hull of a seeded sample of 256 sets against the oracle, every count
    # a hull size (no set handed back)
    pts, offs, dists = wl.batched_sets(4096, 1_000, 1_000_000, seed=7)
    say(f"  hull2d_batched: 4096 sets, {offs[-1]} points")
    hulls, counts = ch.hull2d_batched(torch.from_numpy(pts).cuda(), offs)
    c = counts.cpu().numpy()
    assert np.all(c > 0)
    st = ch.last_batch_stats()
    assert st["redo_sets"] == 0 and st["device_sets"] == 4096, st
    rng = np.random.default_rng(4096)
    for s in sorted(rng.choice(4096, size=256, replace=False)):
        want = oracle.hull(pts[offs[s]:offs[s + 1]])
        assert np.array_equal(hulls[s].cpu().numpy(), want), (s, dists[s], int(offs[s + 1] - offs[s]))
