"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Hull indices must match the oracle bit for bit.  Stage outputs (extreme
points, round-1 survivor counts, SPA survivor counts and the simple polygon)
must match the step-by-step model exactly.  Each case prints its name before
its GPU call.
"""
import contextlib
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1508_05488_amd as ch  # noqa: E402
from oracle import hull as oracle  # noqa: E402
from oracle import steps  # noqa: E402
from paper_1508_05488_amd import autotune  # noqa: E402
from paper_1508_05488_amd import workloads as wl  # noqa: E402
from hullcheck import polygon_with_extras  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@contextlib.contextmanager
def tuned(**kw):
    base = ch.get_tuning(-1)
    ch.clear_tuning()
    ch.set_tuning(2**40, autotune.shape(base, **kw))
    try:
        yield
    finally:
        ch.clear_tuning()
        ch.load_tuning()


def single_hull_kernels_only():
    """Neither the small-input path nor the list mode (fused_max, list_max 0)."""
    return tuned(fused_max=0, list_max=0)


def gpu_hull(pts, name=""):
    # every path of a small input: the default (the batched kernel's one
    # workgroup on the points, or on k_stream's open lists), the list mode
    # alone, and the single-hull kernels throughout
    say(f"  hull2d {name} n={pts.shape[0]}")
    d = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    got = ch.hull2d(d).cpu().numpy()
    say(f"  hull2d {name}: list mode")
    with tuned(fused_max=0):
        alt = ch.hull2d(d).cpu().numpy()
    assert np.array_equal(got, alt), f"{name}: the list mode differs"
    say(f"  hull2d {name}: single-hull kernels")
    with single_hull_kernels_only():
        alt = ch.hull2d(d).cpu().numpy()
    assert np.array_equal(got, alt), f"{name}: the single-hull kernels differ"
    return got


def assert_parity(pts, name=""):
    got = gpu_hull(pts, name)
    want = oracle.hull(pts)
    assert np.array_equal(got, want), f"{name}: got {got[:10]}.. ({got.size}) want {want[:10]}.. ({want.size})"


def test_every_subset_of_3x3_lattice():
    rng = wl.rng_for(61)
    lattice = np.array([(x, y) for x in range(3) for y in range(3)], np.float32)
    for mask in range(1, 1 << 9):
        base = lattice[[i for i in range(9) if mask >> i & 1]]
        extra = base[rng.integers(0, base.shape[0], size=int(rng.integers(0, 4)))]
        pts = np.concatenate([base, extra])
        assert_parity(pts[rng.permutation(pts.shape[0])], f"3x3 mask={mask}")


@pytest.mark.parametrize("k", [2, 3, 5, 9, 33, 1000, 1 << 23])
def test_random_small_sets(k):
    rng = wl.rng_for(62 + k % 83)
    for t in range(150):
        n = int(rng.integers(1, 300))
        assert_parity(wl.small_lattice(n, k, rng), f"lattice k={k} t={t}")


@pytest.mark.parametrize("n", [4095, 4096, 4097, 8191, 8193, 12345, 65537, 100_000, 262_145])
@pytest.mark.parametrize("dist", ["square", "disk", "gaussian", "adversarial"])
def test_tiles_and_ragged_tails(dist, n):
    assert_parity(wl.generate(dist, n, seed=63 + n % 7), f"{dist}")


@pytest.mark.parametrize("dist", ["square", "adversarial"])
def test_misaligned_input(dist):
    # a view starting one point in is 8-byte but not 16-byte aligned
    pts = wl.generate(dist, 50_001, seed=64)
    t = torch.from_numpy(pts).cuda()
    view = t[1:]
    assert view.data_ptr() % 16 == 8
    say(f"  hull2d misaligned {dist}")
    got = ch.hull2d(view).cpu().numpy()
    assert np.array_equal(got, oracle.hull(pts[1:]))


def test_degenerate_inputs():
    cases = {
        "one": np.array([[7, 9]], np.float32),
        "two": np.array([[9, 9], [1, 2]], np.float32),
        "same": np.full((10_000, 2), 12345, np.float32),
        "horizontal": np.stack([np.arange(5000) % 977, np.full(5000, 3)], 1).astype(np.float32),
        "vertical": np.stack([np.full(5000, 3), np.arange(5000) % 977], 1).astype(np.float32),
        "diagonal": np.stack([np.arange(5000) % 977, np.arange(5000) % 977], 1).astype(np.float32),
        "antidiagonal": np.stack([np.arange(5000) % 977, 977 - np.arange(5000) % 977], 1).astype(np.float32),
        "corners_max": np.array([[0, 0], [wl.M, 0], [wl.M, wl.M], [0, wl.M], [5, 5]], np.float32),
        "grid": np.array([(x, y) for y in range(60) for x in range(60)], np.float32),
    }
    for name, pts in cases.items():
        assert_parity(pts, name)


def test_constructed_polygons_known_hull():
    rng = wl.rng_for(65)
    for t in range(10):
        pts, want = polygon_with_extras(int(rng.integers(0, 20_000)), int(rng.integers(0, 500)),
                                        int(rng.integers(0, 500)), rng, scale=int(rng.integers(2, 40000)),
                                        base=(int(rng.integers(0, 1000)), int(rng.integers(0, 1000))))
        got = gpu_hull(pts, f"polygon t={t}")
        assert np.array_equal(got, want)


def test_empty_input():
    say("  hull2d n=0")
    out = ch.hull2d(torch.zeros((0, 2), dtype=torch.float32, device="cuda"))
    assert out.numel() == 0


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf, 0.5, -1.0, 2.0 ** 23, 3e9])
def test_domain_errors(bad):
    pts = wl.generate("square", 10_000, seed=66)
    pts[1234, 0] = bad
    say(f"  hull2d bad value {bad}")
    with pytest.raises(ch.ChainHullError) as e:
        ch.hull2d(torch.from_numpy(pts).cuda())
    assert e.value.status == ch.CH_EDOMAIN
    say(f"  hull2d bad value {bad}: single-hull kernels")
    with single_hull_kernels_only(), pytest.raises(ch.ChainHullError) as e:
        ch.hull2d(torch.from_numpy(pts).cuda())
    assert e.value.status == ch.CH_EDOMAIN
    # the stream stays usable
    assert_parity(wl.generate("square", 1000, seed=67), "after error")


@pytest.mark.parametrize("bad", [np.nan, 0.5, 2.0 ** 23])
def test_domain_error_in_the_list_mode_leaves_a_clean_sample_table(bad):
    # above the small-input path: the pass over the points, then the list
    # mode finds the error; the sample table must be clear for the calls
    # after it (a stale table would drop hull points)
    pts = wl.generate("square", 200_000, seed=69)
    pts[54321, 1] = bad
    say(f"  hull2d 200K bad value {bad}")
    with pytest.raises(ch.ChainHullError) as e:
        ch.hull2d(torch.from_numpy(pts).cuda())
    assert e.value.status == ch.CH_EDOMAIN
    out, cnt = torch.empty(200_000, dtype=torch.int32, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda")
    assert ch.hull2d_async(torch.from_numpy(pts).cuda(), out, cnt) == 0
    torch.cuda.synchronize()
    assert int(cnt.item()) == ch.CH_EDOMAIN
    for dist, seed in (("disk", 70), ("square", 71), ("gaussian", 72)):
        assert_parity(wl.generate(dist, 300_000, seed=seed), f"{dist} 300K after the error")


def test_negative_zero_is_zero():
    pts = wl.generate("square", 5000, seed=68)
    pts[:100] = -0.0
    assert_parity(pts, "negative zero")


def test_invalid_arguments_through_c_abi():
    L = ch.lib()
    t = torch.zeros((10, 2), dtype=torch.float32, device="cuda")
    out = torch.zeros(10, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    say("  hull2d invalid arguments")
    assert L.hull2d(t.data_ptr(), -1, out.data_ptr(), cnt.data_ptr(), s) == ch.CH_EINVAL
    assert L.hull2d(None, 5, out.data_ptr(), cnt.data_ptr(), s) == ch.CH_EINVAL
    assert L.hull2d(t.data_ptr(), 5, out.data_ptr(), None, s) == ch.CH_EINVAL
    assert L.hull2d(t.data_ptr() + 4, 5, out.data_ptr(), cnt.data_ptr(), s) == ch.CH_EINVAL
    assert L.hull2d(t.data_ptr(), 1 << 31, out.data_ptr(), cnt.data_ptr(), s) == ch.CH_EINVAL


def stage_parity(pts, name):
    say(f"  polygon {name} n={pts.shape[0]}")
    poly, st = ch.polygon(torch.from_numpy(pts).cuda())
    ref = steps.cudachain(pts)
    e = ref["ext"]
    assert st["ext_idx"] == [e["minx"], e["miny"], e["maxx"], e["maxy"]], name
    assert st["s1"] == [ref["s1"][r] for r in steps.REGIONS], name
    assert st["s2"] == [ref["s2"][r] for r in steps.REGIONS], name
    assert poly.tolist() == ref["polygon"].tolist(), name
    assert st["candidates"] <= sum(st["s1"])
    assert st["candidates"] >= sum(st["s2"])


@pytest.mark.parametrize("dist", wl.DISTRIBUTIONS)
@pytest.mark.parametrize("n", [1000, 100_000, 1_000_000])
def test_stage_parity(dist, n):
    stage_parity(wl.generate(dist, n, seed=69), f"{dist}")


def test_stage_parity_small_lattices():
    rng = wl.rng_for(70)
    for t in range(200):
        k = int(rng.choice([2, 3, 4, 7, 20, 1 << 23]))
        stage_parity(wl.small_lattice(int(rng.integers(1, 200)), k, rng), f"lattice k={k} t={t}")


def test_repeat_calls_are_deterministic():
    pts = torch.from_numpy(wl.generate("adversarial", 300_000, seed=71)).cuda()
    say("  hull2d repeat x3")
    a = ch.hull2d(pts).cpu().numpy()
    b = ch.hull2d(pts).cpu().numpy()
    c = ch.hull2d(pts).cpu().numpy()
    assert np.array_equal(a, b) and np.array_equal(b, c)


def test_batched_matches_single():
    pts, offs, dists = wl.batched_sets(24, 1, 50_000, seed=72)
    say(f"  hull2d_batched sets={len(dists)} total={offs[-1]}")
    hulls, counts = ch.hull2d_batched(torch.from_numpy(pts).cuda(), offs)
    for s in range(len(dists)):
        want = oracle.hull(pts[offs[s]:offs[s + 1]])
        assert np.array_equal(hulls[s].cpu().numpy(), want), s


def test_timing_stats():
    pts = torch.from_numpy(wl.generate("square", 200_000, seed=73)).cuda()
    ch.set_timing(True)
    try:
        say("  hull2d timing")
        with single_hull_kernels_only():
            ch.hull2d(pts)
            st = ch.last_stats()
    finally:
        ch.set_timing(False)
    assert st["n"] == 200_000 and st["hull"] > 2
    assert all(v >= 0 for v in st["ms"].values())
    assert st["ms"]["stream"] > 0 and st["ms"]["cand"] > 0


@pytest.mark.parametrize("seed", [74, 75])
def test_long_groups_across_tiles(seed):
    """Many points share a region's k1 (box sides, a column inside a region,
    repeated vertices), so equal-key groups span several sort and SPA tiles."""
    rng = wl.rng_for(seed)
    m = 60_000
    side = rng.integers(0, 1 << 23, size=m)
    parts = [
        np.stack([np.zeros(m), side], 1),                       # x = 0
        np.stack([side, np.zeros(m)], 1),                       # y = 0
        np.stack([np.full(m, wl.M), rng.integers(0, 1 << 23, m)], 1),   # x = M
        np.stack([np.full(m, 123), rng.integers(0, 4_000_000, m)], 1),  # a column in R1
        np.tile(np.array([[0, 5_000_000]]), (m, 1)),            # a repeated vertex
        rng.integers(1_000_000, 7_000_000, size=(4 * m, 2)),
    ]
    pts = np.concatenate(parts).astype(np.float32)
    pts = pts[rng.permutation(pts.shape[0])]
    assert_parity(pts, f"long groups seed={seed}")
    stage_parity(pts, f"long groups seed={seed}")


@pytest.mark.parametrize("m", [10, 63, 64, 65, 300, 4096])
def test_bucket_paths(m):
    """m hull vertices of region R1 in one sort bucket (k1 = x in [0, 4096)):
    a bucket of at most 64 records goes to one wave, a larger one to the
    LDS table; a chain longer than a pre-hull segment spans several."""
    rng = wl.rng_for(90 + m)
    i = np.arange(m, dtype=np.int64)
    x = (i * 4095) // max(m - 1, 1)
    y = 3_000_000 + ((m - i) ** 2 * 2_000_000) // (m * m)   # convex, decreasing
    arc = np.stack([x, y], 1)
    box = np.array([[0, 6_000_000], [4_000_000, 0], [8_000_000, 4_000_000], [5_000_000, 8_000_000]])
    inner = rng.integers(2_000_000, 6_000_000, size=(20_000, 2))
    pts = np.concatenate([arc, box, inner]).astype(np.float32)
    pts = pts[rng.permutation(pts.shape[0])]
    assert_parity(pts, f"bucket m={m}")
    stage_parity(pts, f"bucket m={m}")


def test_device_finish_one_and_many_workgroups():
    # a short polygon is finished by one workgroup; the rounded circle leaves
    # more than one workgroup holds, and the wide finish (tangents to the
    # pieces' hulls, many workgroups) takes it
    sq = wl.generate("square", 1_000_000, 81)
    print("  hull2d square 1M (one-workgroup finish)", file=sys.stderr, flush=True)
    got = ch.hull2d(torch.from_numpy(sq).cuda()).cpu().numpy()
    assert ch.last_stats()["device_finish"]
    assert np.array_equal(got, oracle.hull(sq))
    for n, seed in ((2_000_000, 82), (5_000_001, 83)):
        adv = wl.generate("adversarial", n, seed)
        print(f"  hull2d adversarial n={n} (wide finish)", file=sys.stderr, flush=True)
        got = ch.hull2d(torch.from_numpy(adv).cuda()).cpu().numpy()
        st = ch.last_stats()
        assert st["device_finish"] and st["polygon"] > 3584
        assert np.array_equal(got, oracle.hull(adv))


def _edge_inputs():
    # the sampled staircases' first slots (k1 below 2^13 in each frame) and
    # their sub-slots (2^5 wide), and the list mode's filter slots
    rng = wl.rng_for(81)
    M = (1 << 23) - 1
    n = 200_000
    out = {}
    # a thin vertical strip: every point in x-slot 0
    out["strip x<8192"] = np.stack([rng.integers(0, 8192, n), rng.integers(0, M + 1, n)], 1)
    # a square frame: only the four edge strips
    side = rng.integers(0, 4, n)
    a = rng.integers(0, M + 1, n)
    b = rng.integers(0, 8192, n)
    x = np.where(side == 0, b, np.where(side == 1, M - b, a))
    y = np.where(side == 2, b, np.where(side == 3, M - b, a))
    out["frame"] = np.stack([x, y], 1)
    # coordinates on sub-slot and slot boundaries near every edge
    cand = np.array([0, 1, 31, 32, 33, 63, 64, 8159, 8160, 8191, 8192, 8193, 16383, 16384])
    vals = np.concatenate([cand, M - cand, rng.integers(0, M + 1, 64)])
    out["slot boundaries"] = np.stack([rng.choice(vals, n), rng.choice(vals, n)], 1)
    # a uniform square with its edge strips crowded (a quarter of the points)
    sq = rng.integers(0, M + 1, (n, 2))
    k = n // 4
    sq[:k, 0] = rng.integers(0, 64, k)
    out["crowded left edge"] = sq
    return {k: v.astype(np.float32) for k, v in out.items()}


@pytest.mark.parametrize("name", ["strip x<8192", "frame", "slot boundaries", "crowded left edge"])
def test_first_slot_and_sub_slot_edges(name):
    pts = _edge_inputs()[name]
    assert_parity(pts, name)


@pytest.mark.parametrize("n", [20_000, 262_144, 262_145])
def test_own_sample_and_sampling_kernel_bound(n):
    # up to 2^18 points every k_stream workgroup samples the input itself;
    # above, k_sample's table: both sides of the bound, shuffled and sorted
    for dist, seed in (("square", 90), ("disk", 91), ("gaussian", 92)):
        pts = wl.generate(dist, n, seed=seed)
        assert_parity(pts, f"{dist} {n}")
        assert_parity(np.ascontiguousarray(pts[np.argsort(pts[:, 0], kind="stable")]), f"{dist} {n} sorted by x")
