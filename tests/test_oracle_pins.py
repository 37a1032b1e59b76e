"""Pins of the C hull oracle against things other than itself.

Brute force from the edge definition on every subset of small lattices,
closed forms whose answer is known by construction, complete invariants on
large random sets, Qhull (scipy) on sets in general position, and the domain
rules.
"""
import itertools

import numpy as np
import pytest

from oracle import hull as oracle
from paper_1508_05488_amd import workloads as wl
from hullcheck import brute_hull, check_hull, polygon_with_extras


def _with_dups(base: np.ndarray, rng, max_extra: int = 4) -> np.ndarray:
    """Append random duplicates of base points and shuffle."""
    k = int(rng.integers(0, max_extra + 1))
    extra = base[rng.integers(0, base.shape[0], size=k)] if k else np.zeros((0, 2), base.dtype)
    pts = np.concatenate([base, extra])
    return np.ascontiguousarray(pts[rng.permutation(pts.shape[0])])


def test_every_subset_of_3x3_lattice():
    rng = wl.rng_for(11)
    lattice = np.array([(x, y) for x in range(3) for y in range(3)], dtype=np.float32)
    for mask in range(1, 1 << 9):
        base = lattice[[i for i in range(9) if mask >> i & 1]]
        pts = _with_dups(base, rng)
        assert oracle.hull(pts).tolist() == brute_hull(pts), (mask, pts.tolist())


def test_random_subsets_of_4x4_and_5x5_lattices():
    rng = wl.rng_for(12)
    for side, trials in ((4, 1500), (5, 500)):
        lattice = np.array([(x, y) for x in range(side) for y in range(side)], dtype=np.float32)
        for _ in range(trials):
            keep = rng.random(side * side) < rng.uniform(0.1, 0.9)
            if not keep.any():
                continue
            pts = _with_dups(lattice[keep] * rng.integers(1, 4), rng)
            assert oracle.hull(pts).tolist() == brute_hull(pts)


@pytest.mark.parametrize("k", [3, 5, 9, 33, 1 << 23])
def test_random_tiny_sets(k):
    rng = wl.rng_for(13 + k % 97)
    for _ in range(300):
        m = int(rng.integers(1, 25))
        pts = wl.small_lattice(m, k, rng)
        assert oracle.hull(pts).tolist() == brute_hull(pts)


def test_empty_single_and_two():
    assert oracle.hull(np.zeros((0, 2), np.float32)).tolist() == []
    assert oracle.hull(np.array([[5, 7]], np.float32)).tolist() == [0]
    assert oracle.hull(np.array([[5, 7]] * 6, np.float32)).tolist() == [0]
    # two distinct points: lowest-then-leftmost first
    assert oracle.hull(np.array([[9, 9], [1, 2]], np.float32)).tolist() == [1, 0]
    assert oracle.hull(np.array([[1, 2], [9, 2], [1, 2]], np.float32)).tolist() == [0, 1]


def test_full_grid_has_four_corners():
    k = 40
    g = np.array([(x, y) for y in range(k + 1) for x in range(k + 1)], np.float32)
    idx = {(int(x), int(y)): i for i, (x, y) in enumerate(g)}
    want = [idx[(0, 0)], idx[(k, 0)], idx[(k, k)], idx[(0, k)]]
    assert oracle.hull(g).tolist() == want
    rng = wl.rng_for(14)
    perm = rng.permutation(g.shape[0])
    inv = np.argsort(perm)
    assert oracle.hull(g[perm]).tolist() == [int(inv[i]) for i in want]


def test_square_boundary_and_triangle():
    k = 25
    ring = [(x, 0) for x in range(k + 1)] + [(k, y) for y in range(1, k + 1)] + \
           [(x, k) for x in range(k - 1, -1, -1)] + [(0, y) for y in range(k - 1, 0, -1)]
    pts = np.array(ring, np.float32)
    idx = {p: i for i, p in enumerate(ring)}
    assert oracle.hull(pts).tolist() == [idx[(0, 0)], idx[(k, 0)], idx[(k, k)], idx[(0, k)]]
    tri = [(x, y) for x in range(k + 1) for y in range(k + 1) if x + y <= k]
    idx = {p: i for i, p in enumerate(tri)}
    assert oracle.hull(np.array(tri, np.float32)).tolist() == [idx[(0, 0)], idx[(k, 0)], idx[(0, k)]]


@pytest.mark.parametrize("direction", [(1, 0), (0, 1), (1, 1), (3, -2), (-1, 5)])
def test_collinear_sets_give_two_endpoints(direction):
    rng = wl.rng_for(15)
    dx, dy = direction
    t = rng.integers(0, 200, size=300)
    x0, y0 = 5000, 5000
    pts = np.stack([x0 + dx * t, y0 + dy * t], axis=1).astype(np.float32)
    lo, hi = t.min(), t.max()
    i_lo = int(np.flatnonzero(t == lo)[0])
    i_hi = int(np.flatnonzero(t == hi)[0])
    a, b = (i_lo, i_hi)
    ya, yb = pts[a, 1], pts[b, 1]
    if (yb, pts[b, 0]) < (ya, pts[a, 0]):
        a, b = b, a
    assert oracle.hull(pts).tolist() == [a, b]


def test_constructed_convex_polygon_with_extras():
    rng = wl.rng_for(16)
    for scale in (2, 3, 7):
        for _ in range(20):
            pts, want = polygon_with_extras(int(rng.integers(0, 300)), int(rng.integers(0, 50)),
                                            int(rng.integers(0, 30)), rng, scale=scale)
            assert oracle.hull(pts).tolist() == want.tolist()


def test_constructed_polygon_at_scale():
    rng = wl.rng_for(17)
    pts, want = polygon_with_extras(200_000, 5_000, 5_000, rng, scale=50_000, base=(10, 2_000_000))
    assert oracle.hull(pts).tolist() == want.tolist()


@pytest.mark.parametrize("dist", wl.DISTRIBUTIONS)
def test_invariants_on_random_sets(dist):
    pts = wl.generate(dist, 200_000, seed=21)
    check_hull(pts, oracle.hull(pts))


def test_invariants_on_clamped_gaussian_with_many_ties():
    # sigma large enough that many points are clamped onto the box sides
    rng = wl.rng_for(22)
    v = np.clip(np.rint(2 ** 22 + 2 ** 22 * rng.standard_normal((100_000, 2))), 0, wl.M)
    pts = v.astype(np.float32)
    check_hull(pts, oracle.hull(pts))


def test_vertex_sets_match_qhull_in_general_position():
    from scipy.spatial import ConvexHull
    rng = wl.rng_for(23)
    for _ in range(30):
        n = int(rng.integers(5, 3000))
        th = rng.uniform(0, 2 * np.pi, n)
        r = 2 ** 20 * np.sqrt(rng.uniform(0, 1, n))
        pts = np.stack([2 ** 22 + r * np.cos(th), 2 ** 22 + r * np.sin(th)], 1)
        pts = np.unique(np.rint(pts), axis=0)
        pts = pts[rng.permutation(pts.shape[0])].astype(np.float32)
        q = ConvexHull(pts.astype(np.float64))
        assert set(oracle.hull(pts).tolist()) == set(int(v) for v in q.vertices)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf, 0.5, -1.0, 2.0 ** 23, 1e30, 3.25])
def test_domain_rejected(bad):
    pts = np.array([[1, 2], [3, 4], [5, 1]], np.float32)
    pts[1, 1] = bad
    assert oracle.first_invalid(pts) == 1
    with pytest.raises(oracle.OracleDomainError):
        oracle.hull(pts)


def test_negative_zero_accepted():
    pts = np.array([[-0.0, 3], [4, -0.0], [4, 3]], np.float32)
    assert oracle.hull(pts).tolist() == brute_hull(np.abs(pts))


def test_largest_coordinate_accepted():
    m = float(wl.M)
    pts = np.array([[0, 0], [m, 0], [m, m], [0, m], [1, 1]], np.float32)
    assert oracle.hull(pts).tolist() == [0, 1, 2, 3]
