// Step 7 of the method (Section 2.1.3): the convex hull of the simple polygon
// formed by the four region chains, with Melkman's deque algorithm (the
// paper's reference [19]), on the host.
//
// Conventions (the paper outputs coordinates and leaves these open):
//  * consecutive coincident vertices are dropped (cyclically) first;
//  * two or fewer distinct vertices are returned as they are;
//  * a run of collinear vertices at the start is replaced by the segment
//    between its two far ends before the deque is seeded;
//  * turns are exact (int64) and a vertex is popped on a non-left turn, so
//    collinear boundary points are excluded;
//  * the newest vertex, kept at both deque ends, is finally dropped when it
//    lies on the segment joining its two neighbours;
//  * the result is rotated to start at the smallest (y, x).
#include <cstddef>
#include <cstdint>
#include <vector>

#include "finish.h"

namespace chainhull {

namespace {

struct V {
    int64_t x, y;
    int32_t idx;
};

inline int64_t turn(const V& a, const V& b, const V& c)
{
    return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}

}  // namespace

int melkman_finish(const int32_t* xy, const int32_t* idx, int64_t m, int32_t* out, int64_t* out_count)
{
    *out_count = 0;
    // working arrays kept per thread: their memory is reused by later calls
    // instead of being mapped and faulted in afresh
    thread_local std::vector<V> p, hull, d;
    p.clear();
    hull.clear();
    p.reserve(static_cast<size_t>(m));
    for (int64_t i = 0; i < m; ++i) {
        V v{xy[2 * i], xy[2 * i + 1], idx[i]};
        if (v.x < 0 || v.y < 0 || v.x >= (1 << 23) || v.y >= (1 << 23)) return -1;
        if (!p.empty() && p.back().x == v.x && p.back().y == v.y) continue;
        p.push_back(v);
    }
    while (p.size() > 1 && p.back().x == p.front().x && p.back().y == p.front().y) p.pop_back();

    const size_t np = p.size();
    if (np <= 2) {
        hull = p;
    } else {
        // Seed: the first vertex that leaves the line through p[0], p[1].
        size_t k = 2;
        while (k < np && turn(p[0], p[1], p[k]) == 0) ++k;
        const int64_t dx = p[1].x - p[0].x, dy = p[1].y - p[0].y;
        size_t lo = 0, hi = 0;
        int64_t tlo = 0, thi = 0;
        for (size_t i = 0; i < k; ++i) {
            const int64_t t = dx * (p[i].x - p[0].x) + dy * (p[i].y - p[0].y);
            if (t < tlo) { tlo = t; lo = i; }
            if (t > thi) { thi = t; hi = i; }
        }
        if (k == np) {
            hull.push_back(p[lo]);
            hull.push_back(p[hi]);
        } else {
            // Deque in a flat array with room to grow by one slot per vertex
            // at either end: d[bot] .. d[top], with d[bot] == d[top].
            const int64_t cap = 2 * static_cast<int64_t>(np) + 8;
            if (d.size() < static_cast<size_t>(cap)) d.resize(static_cast<size_t>(cap));
            int64_t bot = static_cast<int64_t>(np) + 2, top = bot + 3;
            d[bot] = p[k];
            d[top] = p[k];
            if (turn(p[lo], p[hi], p[k]) > 0) {
                d[bot + 1] = p[lo];
                d[bot + 2] = p[hi];
            } else {
                d[bot + 1] = p[hi];
                d[bot + 2] = p[lo];
            }
            for (size_t i = k + 1; i < np; ++i) {
                const V& v = p[i];
                if (turn(d[bot], d[bot + 1], v) > 0 && turn(d[top - 1], d[top], v) > 0) continue;
                while (turn(d[bot], d[bot + 1], v) <= 0) {
                    if (top - bot < 2) return -1;  // not a simple polygon
                    ++bot;
                }
                if (bot < 1) return -1;
                d[--bot] = v;
                while (turn(d[top - 1], d[top], v) <= 0) {
                    if (top - bot < 2) return -1;
                    --top;
                }
                if (top + 1 >= cap) return -1;
                d[++top] = v;
            }
            // d[bot .. top-1] is the hull; drop the newest vertex d[bot] when
            // it lies on the segment between d[top-1] and d[bot+1].
            int64_t first = bot;
            if (turn(d[top - 1], d[bot], d[bot + 1]) <= 0) first = bot + 1;
            hull.assign(d.begin() + first, d.begin() + top);
        }
    }

    const size_t h = hull.size();
    size_t start = 0;
    for (size_t i = 1; i < h; ++i) {
        if (hull[i].y < hull[start].y || (hull[i].y == hull[start].y && hull[i].x < hull[start].x)) start = i;
    }
    for (size_t i = 0; i < h; ++i) out[i] = hull[(start + i) % h].idx;
    *out_count = static_cast<int64_t>(h);
    return 0;
}

}  // namespace chainhull
