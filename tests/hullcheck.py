"""Independent checks of a hull answer, used to pin the oracle and the GPU path.

Nothing here calls the oracle or the library: brute force on tiny inputs,
exhaustive invariants that characterise the answer completely, and
constructions whose hull is known by design.
"""
from __future__ import annotations

import numpy as np

M = (1 << 23) - 1


def int_coords(points):
    v = np.asarray(points, dtype=np.float32).astype(np.float64)
    return v[:, 0].astype(np.int64), v[:, 1].astype(np.int64)


def _cross(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def _between(a, b, c):
    """c (collinear with a, b, distinct from both) lies strictly inside ab."""
    return min(a[0], b[0]) <= c[0] <= max(a[0], b[0]) and min(a[1], b[1]) <= c[1] <= max(a[1], b[1])


def brute_hull(points) -> list:
    """O(m^3) hull from the edge definition.

    The ordered pair (a, b) of distinct coordinates is a counter-clockwise
    hull edge iff every other distinct coordinate is strictly left of a -> b
    or lies strictly between a and b.  Walk the edges from the lowest, then
    leftmost coordinate.  Duplicates report their minimum index.
    """
    X, Y = int_coords(points)
    first = {}
    for i in range(X.shape[0]):
        first.setdefault((int(X[i]), int(Y[i])), i)
    pts = list(first.keys())
    if not pts:
        return []
    if len(pts) == 1:
        return [first[pts[0]]]
    nxt = {}
    for a in pts:
        for b in pts:
            if a == b:
                continue
            ok = True
            for c in pts:
                if c == a or c == b:
                    continue
                cr = _cross(a, b, c)
                if cr < 0 or (cr == 0 and not _between(a, b, c)):
                    ok = False
                    break
            if ok:
                nxt.setdefault(a, []).append(b)
    start = min(pts, key=lambda p: (p[1], p[0]))
    out = [start]
    cur = start
    while True:
        cands = nxt[cur]
        if len(cands) != 1:
            raise AssertionError(f"ambiguous hull edge at {cur}: {cands}")
        cur = cands[0]
        if cur == start:
            break
        out.append(cur)
        if len(out) > len(pts):
            raise AssertionError("edge walk does not close")
    return [first[p] for p in out]


def check_hull(points, hull, chunk: int = 1 << 20) -> None:
    """Assert that ``hull`` is the exact answer for ``points``.

    A cyclic list of input vertices that is strictly convex and counter-
    clockwise and that contains every input point is the convex hull with
    exactly its strict vertices; the remaining checks fix the start vertex
    and the min-index rule.  Cost O(n * h).
    """
    X, Y = int_coords(points)
    n = X.shape[0]
    H = np.asarray(hull, dtype=np.int64)
    h = H.shape[0]
    if n == 0:
        assert h == 0
        return
    assert h >= 1
    assert H.min() >= 0 and H.max() < n, "index out of range"
    assert np.unique(H).shape[0] == h, "repeated index"
    hx, hy = X[H], Y[H]
    # first vertex: smallest (y, x) over every point
    ymin = Y.min()
    xmin = X[Y == ymin].min()
    assert (hx[0], hy[0]) == (xmin, ymin), "does not start at the lowest-then-leftmost point"
    # min index among duplicates
    key = X * (M + 1) + Y
    hk = key[H]
    order = np.argsort(key, kind="stable")
    sk = key[order]
    pos = np.searchsorted(sk, hk, side="left")
    assert np.array_equal(order[pos], H), "a vertex is not reported by its minimum index"
    assert np.unique(hk).shape[0] == h, "two vertices share a coordinate"
    if h == 1:
        assert np.all(X == hx[0]) and np.all(Y == hy[0])
        return
    if h == 2:
        ax, ay, bx, by = hx[0], hy[0], hx[1], hy[1]
        for s in range(0, n, chunk):
            x, y = X[s:s + chunk], Y[s:s + chunk]
            cr = (bx - ax) * (y - ay) - (by - ay) * (x - ax)
            assert np.all(cr == 0), "points off the two-vertex hull line"
            assert np.all((x >= min(ax, bx)) & (x <= max(ax, bx)) & (y >= min(ay, by)) & (y <= max(ay, by)))
        return
    nx_, ny_ = np.roll(hx, -1), np.roll(hy, -1)
    px_, py_ = np.roll(hx, 1), np.roll(hy, 1)
    turn = (hx - px_) * (ny_ - hy) - (hy - py_) * (nx_ - hx)
    assert np.all(turn > 0), "hull is not strictly convex counter-clockwise"
    ex, ey = nx_ - hx, ny_ - hy
    for s in range(0, n, chunk):
        x, y = X[s:s + chunk], Y[s:s + chunk]
        for k in range(h):
            cr = ex[k] * (y - hy[k]) - ey[k] * (x - hx[k])
            assert cr.min() >= 0, "a point lies outside the hull"


def convex_lattice_polygon(scale: int = 3, base=(1000, 1000)):
    """A strictly convex lattice polygon built from primitive edge vectors.

    Edge vectors are primitive, have distinct directions and are taken in
    angular order together with their negatives, so they close up and every
    vertex is strict.  Each is multiplied by ``scale`` so that every edge
    carries ``scale - 1`` lattice points in its interior.  Returns the
    vertices (counter-clockwise, starting at the lowest-then-leftmost one) and
    the edge step vectors.
    """
    half = [(1, 0), (3, 1), (2, 1), (1, 1), (1, 2), (0, 1), (-1, 3), (-1, 1), (-2, 1)]
    ang = sorted(half, key=lambda v: np.arctan2(v[1], v[0]))
    edges = ang + [(-a, -b) for (a, b) in ang]
    verts = [(0, 0)]
    for (a, b) in edges[:-1]:
        x, y = verts[-1]
        verts.append((x + scale * a, y + scale * b))
    # shift so that the bounding box starts at ``base``
    mx = min(v[0] for v in verts)
    my = min(v[1] for v in verts)
    verts = [(x - mx + base[0], y - my + base[1]) for (x, y) in verts]
    start = min(range(len(verts)), key=lambda k: (verts[k][1], verts[k][0]))
    verts = verts[start:] + verts[:start]
    steps = edges[start:] + edges[:start]
    return verts, steps


def _inner_rectangle(V):
    """An axis-aligned rectangle strictly inside the convex polygon V: all
    four corners are strictly inside, hence (convexity) the whole of it."""
    ex = np.roll(V, -1, axis=0) - V
    c = V.mean(axis=0)
    half = (V.max(axis=0) - V.min(axis=0)) / 2.0
    for a in np.linspace(0.7, 0.05, 14):
        lo = np.floor(c - a * half).astype(np.int64)
        hi = np.ceil(c + a * half).astype(np.int64)
        corners = np.array([[lo[0], lo[1]], [hi[0], lo[1]], [hi[0], hi[1]], [lo[0], hi[1]]])
        cr = ex[:, None, 0] * (corners[None, :, 1] - V[:, None, 1]) - ex[:, None, 1] * (corners[None, :, 0] - V[:, None, 0])
        if (cr > 0).all():
            return lo, hi
    return None


def polygon_with_extras(n_interior: int, n_edge: int, n_dup: int, rng, scale: int = 3,
                        base=(1000, 1000), core: float = 0.0):
    """Points whose exact hull is known: polygon vertices plus extras.

    Returns ``(points f32 [n,2], expected hull indices)``.  Vertices are
    placed at random positions; interior points are strictly inside (a
    fraction ``core`` of them uniform in a rectangle that is strictly inside,
    the rest by rejection over the bounding box), points lie strictly inside
    edges, and duplicates of vertices come after every vertex copy that must
    be reported.
    """
    verts, steps = convex_lattice_polygon(scale, base)
    V = np.array(verts, dtype=np.int64)
    h = V.shape[0]
    ex = np.roll(V, -1, axis=0) - V
    inner = []
    n_core = int(n_interior * core)
    if n_core:
        rect = _inner_rectangle(V)
        assert rect is not None
        lo, hi = rect
        inner.append(np.stack([rng.integers(lo[0], hi[0] + 1, size=n_core),
                               rng.integers(lo[1], hi[1] + 1, size=n_core)], axis=1))
    lo, hi = V.min(axis=0), V.max(axis=0)
    need = n_interior - n_core
    while need > 0:
        batch = min(2 * need + 16, 1 << 23)
        cand = np.stack([rng.integers(lo[0], hi[0] + 1, size=batch),
                         rng.integers(lo[1], hi[1] + 1, size=batch)], axis=1)
        ok = np.ones(cand.shape[0], dtype=bool)
        for k in range(h):
            cr = ex[k, 0] * (cand[:, 1] - V[k, 1]) - ex[k, 1] * (cand[:, 0] - V[k, 0])
            ok &= cr > 0
        got = cand[ok][:need]
        inner.append(got)
        need -= got.shape[0]
    inner = np.concatenate(inner) if inner else np.zeros((0, 2), np.int64)
    # points strictly inside edges
    S = np.array(steps, dtype=np.int64)
    ke = rng.integers(0, h, size=n_edge)
    je = rng.integers(1, scale, size=n_edge) if scale > 1 else np.zeros(n_edge, np.int64)
    on_edge = V[ke] + je[:, None] * S[ke]
    extras = np.concatenate([inner, on_edge])
    extras = extras[rng.permutation(extras.shape[0])]
    n_extra = extras.shape[0]
    n = h + n_extra + n_dup
    # vertex slots: random distinct positions among the first h + n_extra
    slots = np.sort(rng.choice(h + n_extra, size=h, replace=False))
    perm_v = rng.permutation(h)
    pts = np.zeros((n, 2), dtype=np.int64)
    mask = np.zeros(h + n_extra, dtype=bool)
    mask[slots] = True
    pts[:h + n_extra][mask] = V[perm_v]
    pts[:h + n_extra][~mask] = extras
    vert_index = np.empty(h, dtype=np.int64)
    vert_index[perm_v] = slots
    # duplicates of vertices after every vertex copy
    if n_dup:
        pts[h + n_extra:] = V[rng.integers(0, h, size=n_dup)]
    return pts.astype(np.float32), vert_index.astype(np.int32)
