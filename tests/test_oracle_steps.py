"""Pins of the step-by-step CPU model of the method (oracle/steps.py).

Every intermediate is checked against something independent of it: the
paper's Figure 4 narrative (golden fixture), Table 1's orders, brute-force
Pareto dominance for SPA, an exact point-in-triangle test for round 1, a
segment-intersection test for polygon simplicity, and the C hull oracle (which
is pinned on its own) for the final answer.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import hull as oracle
from oracle import steps
from paper_1508_05488_amd import workloads as wl
from hullcheck import brute_hull, check_hull

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_fig4():
    rows = []
    for line in open(os.path.join(GOLDEN, "fig4_r3_spa.txt")):
        line = line.split("#")[0].strip()
        if line:
            lab, x, y, role = line.split()
            rows.append((lab, int(x), int(y), role))
    pts = np.array([(r[1], r[2]) for r in rows], np.float32)
    return rows, pts


def test_fig4_worked_example():
    rows, pts = load_fig4()
    lab = {r[0]: i for i, r in enumerate(rows)}
    res = steps.cudachain(pts)
    ext = res["ext"]
    assert (ext["minx"], ext["miny"], ext["maxx"], ext["maxy"]) == (lab["A"], lab["B"], lab["C"], lab["D"])
    r3 = [lab[f"P{k}"] for k in range(1, 8)]
    assert sorted(np.flatnonzero(res["code"] == 3).tolist()) == sorted(r3)
    assert (res["code"][[lab[c] for c in "ABCD"]] == 0).all()
    kept = [lab[r[0]] for r in sorted(rows, key=lambda r: -r[1]) if r[3] == "keep"]
    assert res["chains"][3].tolist() == kept
    assert res["s1"] == {1: 0, 2: 0, 3: 7, 4: 0} and res["s2"][3] == 4
    assert res["hull"].tolist() == brute_hull(pts)


def test_fig4_loop_rule_matches_narrative():
    rows, _ = load_fig4()
    C = [r for r in rows if r[0] == "C"][0]
    seq = sorted([r for r in rows if r[0].startswith("P")], key=lambda r: -r[1])
    # Figure 2(c) in the R3 frame: k2 = M - y, threshold starts at P_maxx
    keep = steps.spa_keep_loop([steps.M - r[2] for r in seq], steps.M - C[2])
    assert keep == [r[3] == "keep" for r in seq]


def test_frames_reproduce_table1_orders():
    """Table 1: each region's primary sort key and direction, and how x and y
    move along its chain (k1 rising and k2 falling along a kept chain)."""
    table1 = {1: ("x", +1, (+1, -1)), 2: ("y", +1, (+1, +1)),
              3: ("x", -1, (-1, +1)), 4: ("y", -1, (-1, -1))}
    rng = wl.rng_for(31)
    X = rng.integers(0, 1 << 23, 4000)
    Y = rng.integers(0, 1 << 23, 4000)
    for r, (key, direction, (ox, oy)) in table1.items():
        k1, k2 = steps.frame(r, X, Y)
        prim = X if key == "x" else Y
        assert np.array_equal(k1, prim if direction > 0 else steps.M - prim)
        a, b = np.arange(0, 4000, 2), np.arange(1, 4000, 2)
        step = (k1[b] > k1[a]) & (k2[b] < k2[a])
        assert step.sum() > 100
        assert np.all(np.sign(X[b] - X[a])[step] == ox)
        assert np.all(np.sign(Y[b] - Y[a])[step] == oy)


def _tiny_sets(rng, count, k):
    for _ in range(count):
        m = int(rng.integers(1, 30))
        yield wl.small_lattice(m, k, rng)


def test_steps_hull_on_every_3x3_subset():
    rng = wl.rng_for(32)
    lattice = np.array([(x, y) for x in range(3) for y in range(3)], np.float32)
    for mask in range(1, 1 << 9):
        base = lattice[[i for i in range(9) if mask >> i & 1]]
        extra = base[rng.integers(0, base.shape[0], size=int(rng.integers(0, 4)))]
        pts = np.concatenate([base, extra])
        pts = pts[rng.permutation(pts.shape[0])]
        assert steps.cudachain(pts)["hull"].tolist() == oracle.hull(pts).tolist()


@pytest.mark.parametrize("k", [3, 4, 6, 11, 64, 1 << 23])
def test_steps_hull_on_random_small_sets(k):
    rng = wl.rng_for(33 + k % 101)
    for pts in _tiny_sets(rng, 400, k):
        assert steps.cudachain(pts)["hull"].tolist() == oracle.hull(pts).tolist()


@pytest.mark.parametrize("dist", wl.DISTRIBUTIONS)
def test_steps_hull_on_distributions(dist):
    pts = wl.generate(dist, 100_000, seed=34)
    res = steps.cudachain(pts)
    assert res["hull"].tolist() == oracle.hull(pts).tolist()
    assert res["outside"].max() <= 1


def test_extremes_against_tuple_minimum():
    rng = wl.rng_for(35)
    for k in (3, 7, 1000):
        for pts in _tiny_sets(rng, 200, k):
            X, Y = steps.to_int(pts)
            e = steps.extreme_points(X, Y)
            items = [(int(X[i]), int(Y[i]), i) for i in range(X.shape[0])]
            assert e["minx"] == min(items, key=lambda t: (t[0], -t[1], t[2]))[2]
            assert e["miny"] == min(items, key=lambda t: (t[1], t[0], t[2]))[2]
            assert e["maxx"] == min(items, key=lambda t: (-t[0], t[1], t[2]))[2]
            assert e["maxy"] == min(items, key=lambda t: (-t[1], -t[0], t[2]))[2]


def _in_closed_triangle(a, b, c, p):
    """Exact barycentric test with rationals (an independent formula)."""
    det = (b[1] - c[1]) * (a[0] - c[0]) + (c[0] - b[0]) * (a[1] - c[1])
    if det == 0:
        # degenerate triangle: on the segment hull of the three points
        xs = sorted([a, b, c])
        lo, hi = xs[0], xs[-1]
        colin = (hi[0] - lo[0]) * (p[1] - lo[1]) - (hi[1] - lo[1]) * (p[0] - lo[0]) == 0
        return colin and min(lo[0], hi[0]) <= p[0] <= max(lo[0], hi[0]) and \
            min(lo[1], hi[1]) <= p[1] <= max(lo[1], hi[1])
    l1 = Fraction((b[1] - c[1]) * (p[0] - c[0]) + (c[0] - b[0]) * (p[1] - c[1]), det)
    l2 = Fraction((c[1] - a[1]) * (p[0] - c[0]) + (a[0] - c[0]) * (p[1] - c[1]), det)
    return l1 >= 0 and l2 >= 0 and 1 - l1 - l2 >= 0


def test_round1_survivors_are_the_points_outside_the_closed_quad():
    rng = wl.rng_for(36)
    for k in (5, 9, 40, 1 << 23):
        for pts in _tiny_sets(rng, 150, k):
            X, Y = steps.to_int(pts)
            e = steps.extreme_points(X, Y)
            code, outside = steps.regions(X, Y, e)
            A, B, C, D = [(int(X[i]), int(Y[i])) for i in steps.quad_vertices(e)]
            for i in range(X.shape[0]):
                p = (int(X[i]), int(Y[i]))
                inside = _in_closed_triangle(A, B, C, p) or _in_closed_triangle(A, C, D, p)
                assert (code[i] == 0) == inside, (pts.tolist(), i)
            assert outside.max() <= 1


def test_spa_vectorised_rule_equals_the_loop():
    rng = wl.rng_for(37)
    for _ in range(300):
        m = int(rng.integers(0, 60))
        k2 = np.sort(rng.integers(0, 20, m))[::-1] if rng.random() < 0.3 else rng.integers(0, 20, m)
        sigma = int(rng.integers(0, 25))
        assert steps.spa_keep(np.asarray(k2), sigma).tolist() == steps.spa_keep_loop(list(k2), sigma)


def test_spa_survivors_are_the_undominated_points():
    """Kept iff no other point of the region (nor its first point) dominates it."""
    rng = wl.rng_for(38)
    for k in (6, 30, 1 << 23):
        for pts in _tiny_sets(rng, 150, k):
            X, Y = steps.to_int(pts)
            res = steps.cudachain(pts)
            if res["n"] == 0:
                continue
            for r in steps.REGIONS:
                members = np.flatnonzero(res["code"] == r).tolist()
                first, _ = steps.region_endpoints(r, res["ext"])
                k1, k2 = steps.frame(r, X, Y)
                want = []
                for i in members:
                    dom = k1[first] <= k1[i] and k2[first] <= k2[i]
                    for j in members:
                        if j == i:
                            continue
                        if k1[j] <= k1[i] and k2[j] <= k2[i] and (k1[j], k2[j], j) < (k1[i], k2[i], i):
                            dom = True
                            break
                    if not dom:
                        want.append(i)
                assert sorted(res["chains"][r].tolist()) == sorted(want)


def _segments_cross(p1, p2, p3, p4):
    def o(a, b, c):
        v = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
        return (v > 0) - (v < 0)

    def on(a, b, c):
        return min(a[0], b[0]) <= c[0] <= max(a[0], b[0]) and min(a[1], b[1]) <= c[1] <= max(a[1], b[1])

    d1, d2, d3, d4 = o(p3, p4, p1), o(p3, p4, p2), o(p1, p2, p3), o(p1, p2, p4)
    if d1 * d2 < 0 and d3 * d4 < 0:
        return True
    return (d1 == 0 and on(p3, p4, p1)) or (d2 == 0 and on(p3, p4, p2)) or \
        (d3 == 0 and on(p1, p2, p3)) or (d4 == 0 and on(p1, p2, p4))


def test_polygon_is_simple_and_keeps_every_hull_vertex():
    rng = wl.rng_for(39)
    for k in (8, 50, 1 << 23):
        for pts in _tiny_sets(rng, 150, k):
            X, Y = steps.to_int(pts)
            res = steps.cudachain(pts)
            poly = [(int(X[i]), int(Y[i])) for i in res["polygon"]]
            assert len(set(poly)) == len(poly)
            m = len(poly)
            if m >= 4:
                for a in range(m):
                    for b in range(a + 2, m):
                        if a == 0 and b == m - 1:
                            continue
                        assert not _segments_cross(poly[a], poly[(a + 1) % m], poly[b], poly[(b + 1) % m])
            # Section 4.2: no strict vertex is ever discarded
            assert set(oracle.hull(pts).tolist()) <= set(res["polygon"].tolist())


def test_steps_invariants_on_adversarial_circle():
    pts = wl.generate("adversarial", 60_000, seed=40)
    res = steps.cudachain(pts)
    check_hull(pts, res["hull"])
    assert res["hull"].tolist() == oracle.hull(pts).tolist()


# --- the paper's divide-and-conquer SPA (Section 2.2.2, Section 4.3) ---

def test_spa_chunked_pins():
    rng = np.random.default_rng(91)
    for _ in range(200):
        m = int(rng.integers(0, 40))
        k2 = rng.integers(0, 30, size=m)
        sigma = int(rng.integers(0, 35))
        exact = steps.spa_keep(k2, sigma)
        # one subset: the exact rule
        assert np.array_equal(steps.spa_keep_chunked(k2, sigma, max(m, 1)), exact)
        for chunk in (1, 2, 3, 7):
            got = steps.spa_keep_chunked(k2, sigma, chunk)
            # a superset of the exact survivors
            assert np.all(got[exact])
            # each subset by the literal loop, a later one from its first point
            want = []
            for s0 in range(0, m, chunk):
                part = list(k2[s0:s0 + chunk])
                if s0 == 0:
                    want += steps.spa_keep_loop(part, sigma)
                else:
                    want += [True] + steps.spa_keep_loop(part[1:], part[0])
            assert got.tolist() == want
        if m:
            one = steps.spa_keep_chunked(k2, sigma, 1)
            assert one[0] == (k2[0] < sigma) and bool(np.all(one[1:]))


@pytest.mark.parametrize("dist", ["square", "disk", "gaussian"])
def test_chunked_spa_keeps_the_hull_on_tie_free_inputs(dist):
    # without ties in x or y every chain stays monotone in k1, so the polygon
    # is still simple and Melkman still returns the hull
    pts = wl.tie_free(dist, 3000, 92)
    assert np.unique(pts[:, 0]).size == pts.shape[0] and np.unique(pts[:, 1]).size == pts.shape[0]
    want = oracle.hull(pts)
    for chunk in (1, 2, 5, 16, 100):
        r = steps.cudachain(pts, chunk=chunk)
        assert np.array_equal(r["hull"], want), chunk
        exact = steps.cudachain(pts)
        assert sum(r["s2"].values()) >= sum(exact["s2"].values())
