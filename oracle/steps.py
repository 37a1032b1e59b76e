"""TEST INFRASTRUCTURE ONLY: the CudaChain procedure, step by step, on the CPU.

Mei, "CudaChain: A Practical GPU-accelerated 2D Convex Hull Algorithm",
Section 2.1 lists seven steps.  This module takes them in the paper's order
and notation, in plain numpy with exact int64 arithmetic, so that each
intermediate result of the GPU path (extreme points, regions, round-1
survivors, SPA survivors, the simple polygon, the hull) can be compared with
something a reader can check against the paper by eye.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg use it; the product path
never imports it.

Readings taken where the paper is silent, ambiguous or garbled (each is also
listed in the design notes):

* Extreme-point ties (step 1).  The paper takes single-coordinate min/max
  reductions.  Here ``P_minx`` is the point with minimum x, then maximum y;
  ``P_miny`` minimum y then minimum x; ``P_maxx`` maximum x then minimum y;
  ``P_maxy`` maximum y then maximum x; remaining ties go to the smallest index.
  All four are then strict hull vertices (or the endpoints of a collinear set).
* Side of the directed lines (Section 2.1.1).  With the y axis up and the
  quadrilateral walked P_minx -> P_miny -> P_maxx -> P_maxy (counter-clockwise),
  the corner regions lie strictly to the *right* of each directed edge
  (negative cross product).  Points inside or on the quadrilateral are R0.
* Sort order (Table 1, step 4).  Only the primary order is given.  Each region
  is sorted in a frame ``(k1, k2)`` obtained from R1's by a rotation, ascending
  by ``(k1, k2, index)``; ``k1`` reproduces Table 1's primary order.
* SPA strictness (Figure 2, step 5).  A point is kept only if its ``k2`` is
  strictly below the running threshold ``t``, which starts at the region's
  first point (Table 1) and otherwise takes each kept point's ``k2``.  Ties
  are discarded: a tied point lies in a closed triangle of input points and
  is not a strict hull vertex, and exact duplicates keep their first (minimum
  index) copy.
* The paper's per-chunk parallel SPA (Section 2.2.2) is not used: the
  threshold is carried over the whole region, as in the sequential rule.
* Melkman degeneracies (Section 2.1.3).  Consecutive duplicate vertices are
  dropped; two or fewer distinct vertices are the answer; a collinear prefix
  is replaced by the segment between its two far ends; the last vertex, which
  the deque keeps at both ends, is dropped at the end when it lies on the
  segment between its neighbours.
* Output (the paper returns coordinates): vertex indices, counter-clockwise,
  starting at the lowest-then-leftmost vertex, collinear points excluded.
"""
from __future__ import annotations

from collections import deque

import numpy as np

M = (1 << 23) - 1

# Region numbers follow the paper: 1 lower left, 2 lower right, 3 upper
# right, 4 upper left, 0 interior (the paper's d_pos indicator, Section 2.2.1).
REGIONS = (1, 2, 3, 4)


class DomainError(ValueError):
    pass


def to_int(points) -> tuple[np.ndarray, np.ndarray]:
    """Integer coordinates X, Y (int64) of an ``[n, 2]`` float32 array."""
    pts = np.asarray(points, dtype=np.float32)
    if pts.ndim != 2 or pts.shape[1] != 2:
        raise ValueError("points must have shape [n, 2]")
    v = pts.astype(np.float64)
    ok = np.isfinite(v) & (v >= 0) & (v < 2.0 ** 23) & (np.floor(v) == v)
    if not ok.all():
        raise DomainError("point coordinates must be integers in [0, 2**23)")
    return v[:, 0].astype(np.int64), v[:, 1].astype(np.int64)


def cross(ox, oy, ax, ay, bx, by):
    """Twice the signed area of (o, a, b): > 0 when o -> a -> b turns left."""
    return (ax - ox) * (by - oy) - (ay - oy) * (bx - ox)


# --- Step 1: the four extreme points (Section 2.1 step 1, Section 2.2.1) ---

def _argmin_lex(primary: np.ndarray, secondary: np.ndarray) -> int:
    """Smallest index among points minimising (primary, secondary)."""
    first = primary == primary.min()
    second = np.where(first, secondary, np.iinfo(np.int64).max)
    return int(np.flatnonzero(second == second.min())[0])


def extreme_points(X: np.ndarray, Y: np.ndarray) -> dict:
    """Indices of P_minx, P_miny, P_maxx, P_maxy with the tie-breaks above."""
    return {
        "minx": _argmin_lex(X, -Y),
        "miny": _argmin_lex(Y, X),
        "maxx": _argmin_lex(-X, Y),
        "maxy": _argmin_lex(-Y, -X),
    }


def quad_vertices(ext: dict) -> list:
    """The quadrilateral in the order P_minx, P_miny, P_maxx, P_maxy (CCW)."""
    return [ext["minx"], ext["miny"], ext["maxx"], ext["maxy"]]


# --- Step 2: distribution and first discard (Section 2.1.1) ---

def regions(X: np.ndarray, Y: np.ndarray, ext: dict):
    """Region number of every point (1..4), or 0 for interior points.

    Region r holds the points strictly right of the directed line
    E[r-1] -> E[r] with E = (P_minx, P_miny, P_maxx, P_maxy, P_minx), tested
    in the paper's if/else order R1, R2, R3, R4.  Also returns, per point, how
    many of the four lines it is strictly right of (never more than one).
    """
    E = quad_vertices(ext) + [ext["minx"]]
    code = np.zeros(X.shape[0], dtype=np.int64)
    outside = np.zeros(X.shape[0], dtype=np.int64)
    for r in REGIONS:
        a, b = E[r - 1], E[r]
        c = cross(X[a], Y[a], X[b], Y[b], X, Y)
        right = c < 0
        outside += right
        code[(code == 0) & right] = r
    return code, outside


# --- Steps 3-4: per-region frames and sort (Table 1) ---

def frame(r: int, X: np.ndarray, Y: np.ndarray):
    """(k1, k2) of region r.  Table 1's sort order is k1 ascending."""
    if r == 1:            # lower left: x ascending
        return X, Y
    if r == 2:            # lower right: y ascending
        return Y, M - X
    if r == 3:            # upper right: x descending
        return M - X, M - Y
    if r == 4:            # upper left: y descending
        return M - Y, X
    raise ValueError(r)


def region_endpoints(r: int, ext: dict) -> tuple[int, int]:
    """Table 1's first and last point of region r."""
    q = quad_vertices(ext)
    return q[r - 1], q[r % 4]


def sort_region(idx: np.ndarray, k1: np.ndarray, k2: np.ndarray) -> np.ndarray:
    """Positions that sort the region ascending by (k1, k2, index)."""
    return np.lexsort((idx, k2, k1))


# --- Step 5: SPA (Figure 2) ---

def spa_keep(k2_sorted: np.ndarray, sigma: int) -> np.ndarray:
    """Figure 2: keep a point iff its k2 is below the running threshold.

    The threshold starts at the region's first point (``sigma``) and becomes
    each kept point's k2; a discarded point never lowers it, so it equals the
    minimum k2 seen so far (``minimum.accumulate``).
    """
    seen = np.concatenate([np.array([sigma], dtype=np.int64), k2_sorted.astype(np.int64)])
    threshold = np.minimum.accumulate(seen)[:-1]
    return k2_sorted < threshold


def spa_keep_loop(k2_sorted, sigma: int) -> list:
    """The same rule as a literal loop over the sorted points."""
    t = sigma
    keep = []
    for v in k2_sorted:
        if v < t:
            keep.append(True)
            t = v
        else:
            keep.append(False)
    return keep


def spa_keep_chunked(k2_sorted: np.ndarray, sigma: int, chunk: int) -> np.ndarray:
    """The divide-and-conquer variant of SPA that the paper implements
    (Section 2.2.2; its limitation in Section 4.3): the region's sorted
    points are split into consecutive subsets of ``chunk`` points, and each
    subset is checked on its own with the rule of Figure 2, in parallel.

    Reading (the paper does not say how a subset starts): the first subset
    starts from the region's first point (threshold ``sigma``), as the whole
    region would; a later subset knows no earlier point of the chain, so its
    first point is kept and starts its threshold.  With one subset this is
    exactly ``spa_keep``; with smaller subsets it keeps a superset.
    """
    k2 = np.asarray(k2_sorted, dtype=np.int64)
    m = k2.shape[0]
    keep = np.zeros(m, dtype=bool)
    if chunk < 1:
        raise ValueError("chunk must be positive")
    for s0 in range(0, m, chunk):
        part = k2[s0:s0 + chunk]
        start = sigma if s0 == 0 else np.iinfo(np.int64).max
        keep[s0:s0 + chunk] = spa_keep(part, start)
    return keep


# --- Steps 5-6: chains and the simple polygon ---

def simple_polygon(X, Y, ext: dict, code: np.ndarray, chunk: int | None = None):
    """Chains of the four regions joined counter-clockwise.

    Returns ``(poly_idx, chains, s1, s2)``: the polygon
    [P_minx, R1 chain, P_miny, R2 chain, P_maxx, R3 chain, P_maxy, R4 chain]
    as point indices with consecutive coincident vertices dropped (cyclic),
    the per-region kept indices, and per-region round-1 and SPA survivor
    counts.  With ``chunk``, SPA runs in subsets of that many points
    (``spa_keep_chunked``) instead of over the whole region.
    """
    n = X.shape[0]
    all_idx = np.arange(n, dtype=np.int64)
    chains, s1, s2 = {}, {}, {}
    for r in REGIONS:
        sel = all_idx[code == r]
        k1, k2 = frame(r, X[sel], Y[sel])
        order = sort_region(sel, k1, k2)
        first, _ = region_endpoints(r, ext)
        sigma = int(frame(r, X[first:first + 1], Y[first:first + 1])[1][0])
        keep = spa_keep(k2[order], sigma) if chunk is None else spa_keep_chunked(k2[order], sigma, chunk)
        chains[r] = sel[order][keep]
        s1[r] = int(sel.shape[0])
        s2[r] = int(keep.sum())
    raw = []
    for r in REGIONS:
        first, _ = region_endpoints(r, ext)
        raw.append(first)
        raw.extend(int(i) for i in chains[r])
    poly = []
    for i in raw:
        if poly and X[poly[-1]] == X[i] and Y[poly[-1]] == Y[i]:
            continue
        poly.append(i)
    while len(poly) > 1 and X[poly[-1]] == X[poly[0]] and Y[poly[-1]] == Y[poly[0]]:
        poly.pop()
    return poly, chains, s1, s2


# --- Step 7: Melkman's convex hull of a simple polygon (Section 2.1.3) ---

def melkman(poly, X, Y) -> list:
    """Hull of a simple polygon (list of point indices), counter-clockwise.

    The deque holds the hull of the vertices seen so far with the newest
    vertex at both ends; a vertex strictly left of both edges at the ends is
    inside, otherwise the ends are trimmed until it sees them on its left and
    it is added at both ends.  Pops on non-left turns exclude collinear points.
    """
    def turn(a, b, c):
        return int(cross(X[a], Y[a], X[b], Y[b], X[c], Y[c]))

    m = len(poly)
    if m <= 2:
        return list(poly)
    p0, p1 = poly[0], poly[1]
    k = 2
    while k < m and turn(p0, p1, poly[k]) == 0:
        k += 1
    dx, dy = int(X[p1] - X[p0]), int(Y[p1] - Y[p0])

    def along(i):
        return dx * int(X[i] - X[p0]) + dy * int(Y[i] - Y[p0])

    head = poly[:k]
    lo = min(head, key=along)
    hi = max(head, key=along)
    if k == m:
        return [lo, hi]
    pk = poly[k]
    if turn(lo, hi, pk) > 0:
        dq = deque([pk, lo, hi, pk])
    else:
        dq = deque([pk, hi, lo, pk])
    for i in poly[k + 1:]:
        if turn(dq[0], dq[1], i) > 0 and turn(dq[-2], dq[-1], i) > 0:
            continue
        while turn(dq[0], dq[1], i) <= 0:
            dq.popleft()
            if len(dq) < 2:
                raise ValueError("polygon is not simple")
        dq.appendleft(i)
        while turn(dq[-2], dq[-1], i) <= 0:
            dq.pop()
            if len(dq) < 2:
                raise ValueError("polygon is not simple")
        dq.append(i)
    # The newest vertex sits at both ends and was never tested against the
    # polygon's closing edge: drop it when it lies on the segment joining
    # its two deque neighbours (collinear points are excluded).
    if turn(dq[-2], dq[0], dq[1]) <= 0:
        dq.pop()
        dq.popleft()
        return list(dq)
    return list(dq)[:-1]


def rotate_to_lowest(hull, X, Y) -> list:
    """Rotate a cyclic vertex list to start at the smallest (y, x)."""
    if not hull:
        return []
    start = min(range(len(hull)), key=lambda k: (int(Y[hull[k]]), int(X[hull[k]])))
    return list(hull[start:]) + list(hull[:start])


def region_sequences(points) -> dict:
    """Per region r: (k2 of its points in sorted order, the k2 of its first
    point), the input of SPA (steps 1-4)."""
    X, Y = to_int(points)
    ext = extreme_points(X, Y)
    code, _ = regions(X, Y, ext)
    out = {}
    all_idx = np.arange(X.shape[0], dtype=np.int64)
    for r in REGIONS:
        sel = all_idx[code == r]
        k1, k2 = frame(r, X[sel], Y[sel])
        order = sort_region(sel, k1, k2)
        first, _ = region_endpoints(r, ext)
        sigma = int(frame(r, X[first:first + 1], Y[first:first + 1])[1][0])
        out[r] = (k2[order], sigma)
    return out


def cudachain(points, chunk: int | None = None) -> dict:
    """All seven steps.  Returns every intermediate and the hull indices.
    ``chunk``: run SPA in subsets (the paper's divide-and-conquer variant)."""
    X, Y = to_int(points)
    n = X.shape[0]
    if n == 0:
        return {"n": 0, "hull": np.zeros(0, np.int32)}
    ext = extreme_points(X, Y)
    code, outside = regions(X, Y, ext)
    poly, chains, s1, s2 = simple_polygon(X, Y, ext, code, chunk)
    hull = rotate_to_lowest(melkman(poly, X, Y), X, Y)
    return {
        "n": n,
        "ext": ext,
        "code": code,
        "outside": outside,
        "s1": s1,
        "s2": s2,
        "chains": chains,
        "polygon": np.asarray(poly, dtype=np.int64),
        "hull": np.asarray(hull, dtype=np.int32),
    }
