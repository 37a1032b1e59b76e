"""The rule the multi-workgroup device finish applies (k_finish_wide),
checked on the CPU against the oracle: a region's chain is cut into pieces;
each piece's lower hull H in the region's frame; sigma_L the largest slope
of the lower tangents to H from the region's points left of the piece and
its start extreme point, sigma_R the smallest slope of the tangents from H
to the points right of it and its end extreme point (tangents by binary
search over H, points skipped when the bounding box of their piece lies
strictly above the line found from the two neighbouring pieces); a vertex of
H with edge slopes s_in < s_out is a strict hull vertex iff
max(s_in, sigma_L) < min(s_out, sigma_R).  Emitted in the order
E_1, R2, E_2, R3, E_3, R4, E_0, R1, the result must be the oracle's hull
on every non-degenerate input (degenerate ones never reach the wide
finish: it only takes polygons of thousands of vertices).  This pins the
geometry of the kernel's rule; the GPU tests pin the kernel itself."""
import random

import numpy as np

from oracle import hull as oracle
from oracle import steps
from paper_1508_05488_amd import workloads as wl


def turn(o, a, b):
    return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])


def less(a, b):  # slopes (dy, dx) with dx >= 0; dx == 0 is -inf (dy < 0) or +inf
    if a[1] == 0 and b[1] == 0:
        return a[0] < 0 < b[0]
    if a[1] == 0:
        return a[0] < 0
    if b[1] == 0:
        return b[0] > 0
    return a[0] * b[1] < b[0] * a[1]


def slope(a, b):
    return (b[1] - a[1], b[0] - a[0])


def tangent_from_left(H, a):
    lo, hi = 0, len(H) - 1
    while lo < hi:
        mid = (lo + hi) // 2
        if turn(a, H[mid], H[mid + 1]) < 0:
            lo = mid + 1
        else:
            hi = mid
    return lo


def tangent_to_right(H, b):
    lo, hi = 0, len(H) - 1
    while lo < hi:
        mid = (lo + hi) // 2
        if turn(H[mid], b, H[mid + 1]) < 0:
            lo = mid + 1
        else:
            hi = mid
    return lo


def wide_rule(points, maxpiece, seed):
    rnd = random.Random(seed)
    X, Y = steps.to_int(points)
    ext = steps.extreme_points(X, Y)
    code, _ = steps.regions(X, Y, ext)
    _, chains, _, _ = steps.simple_polygon(X, Y, ext, code)
    qv = steps.quad_vertices(ext)
    out, prev = [], []
    for r in (2, 3, 4, 1):
        E, F = qv[r - 1], qv[r % 4]
        if not any(X[E] == X[p] and Y[E] == Y[p] for p in prev):
            out.append(int(E))
        prev.append(E)
        k1, k2 = steps.frame(r, X, Y)

        def pt(i):
            return (int(k1[i]), int(k2[i]))

        e, f = pt(E), pt(F)
        ch = list(chains[r])
        pieces, i = [], 0
        while i < len(ch):
            m = rnd.randint(1, maxpiece)
            pieces.append(ch[i:i + m])
            i += m
        for pi, P in enumerate(pieces):
            H, Hi = [], []
            for j in P:
                p = pt(j)
                while len(H) >= 2 and turn(H[-2], H[-1], p) <= 0:
                    H.pop()
                    Hi.pop()
                H.append(p)
                Hi.append(j)

            def best(cands, left, cur=None):
                for a in cands:
                    if left:
                        ln = (a, H[tangent_from_left(H, a)])
                        better = cur is None or less(slope(*cur), slope(*ln))
                    else:
                        ln = (H[tangent_to_right(H, a)], a)
                        better = cur is None or less(slope(*ln), slope(*cur))
                    if better:
                        cur = ln
                return cur

            def above(ln, Q):  # the bounding box of piece Q strictly above the line
                f0, l0 = pt(Q[0]), pt(Q[-1])
                if ln[0][0] == ln[1][0]:
                    return False
                return turn(ln[0], ln[1], (f0[0], l0[1])) > 0 and turn(ln[0], ln[1], (l0[0], l0[1])) > 0

            near = [pieces[j] for j in (pi - 1, pi - 2) if j >= 0]
            cur = best([e] + [pt(j) for Q in near for j in Q], True)
            far = [Q for Q in pieces[:max(pi - 2, 0)] if not above(cur, Q)]
            sl = slope(*best([pt(j) for Q in far for j in Q], True, cur))
            near = [pieces[j] for j in (pi + 1, pi + 2) if j < len(pieces)]
            cur = best([f] + [pt(j) for Q in near for j in Q], False)
            far = [Q for Q in pieces[pi + 3:] if not above(cur, Q)]
            sr = slope(*best([pt(j) for Q in far for j in Q], False, cur))
            for k, (p, j) in enumerate(zip(H, Hi)):
                sin = slope(H[k - 1], p) if k > 0 else (-1, 0)
                sout = slope(p, H[k + 1]) if k + 1 < len(H) else (1, 0)
                lo = sl if less(sin, sl) else sin
                hi = sr if less(sr, sout) else sout
                if less(lo, hi):
                    out.append(int(j))
    return np.array(out, dtype=np.int32)


def test_wide_rule_equals_oracle():
    checked = 0
    for t in range(240):
        rng = np.random.default_rng(t)
        kind = t % 4
        n = int(rng.integers(3, 400))
        if kind == 0:
            pts = rng.integers(0, 8, (n, 2)).astype(np.float32)       # a small lattice: ties everywhere
        elif kind == 1:
            pts = wl.generate("adversarial", n, t)                    # points on a rounded circle
        elif kind == 2:
            pts = wl.generate("disk", n, t)
        else:
            pts = rng.integers(0, 40, (n, 2)).astype(np.float32)
        want = oracle.hull(pts)
        if len(want) < 3:
            continue
        got = wide_rule(pts, maxpiece=int(rng.integers(1, 9)), seed=t)
        assert np.array_equal(got, want), (t, kind, n)
        checked += 1
    for t in range(12):
        pts = wl.generate(("adversarial", "disk", "square", "gaussian")[t % 4], 3000 + 331 * t, 1000 + t)
        got = wide_rule(pts, maxpiece=(3, 17, 64, 200)[t % 4], seed=t)
        assert np.array_equal(got, oracle.hull(pts)), t
        checked += 1
    assert checked > 200
