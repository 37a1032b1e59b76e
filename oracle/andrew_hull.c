/*
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct CPU reference for
 * the exact planar convex hull that the CudaChain method (Mei, "CudaChain: A
 * Practical GPU-accelerated 2D Convex Hull Algorithm") computes.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never links or calls it, and it shares no code with the
 * GPU library.
 *
 * What is computed (the plain definition; Section 2.1 states that the result
 * is exactly the convex hull of the input, and Section 4.2 argues it):
 *   - the strict vertices of conv(P) (an input coordinate that is not in the
 *     convex hull of the other distinct coordinates), each reported once by
 *     the minimum index among its exact duplicates;
 *   - in counter-clockwise order (y axis up), starting at the vertex with the
 *     smallest Y and, among those, the smallest X;
 *   - n == 0 -> empty; one distinct coordinate -> [its min index]; all
 *     distinct coordinates collinear -> [lowest-then-leftmost endpoint, the
 *     other endpoint].
 *
 * How: Andrew's monotone chain (the paper's reference [4], Section 1) with
 * exact 64-bit integer orientation tests.  Coordinates are integer-valued
 * float32 in [0, 2^23), so every difference fits in 24 bits and every cross
 * product in 48 bits.
 *
 * Input outside that domain (NaN, +-Inf, a fractional value, a negative value
 * or a value >= 2^23) is rejected; -0.0 is accepted as 0.  The paper does not
 * define behaviour outside the domain; this is the chosen reading.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

#define ORACLE_OK 0
#define ORACLE_EDOMAIN (-2)
#define ORACLE_ENOMEM (-3)
#define ORACLE_EINVAL (-1)

typedef struct {
    int32_t x, y, idx;
} opt_t;

/* 1 if v is an integer value in [0, 2^23), else 0.  NaN fails v >= 0. */
static int in_domain(float v)
{
    if (!(v >= 0.0f && v < 8388608.0f)) return 0;
    return floorf(v) == v;
}

/* Lexicographic order on (x, y, idx). */
static int cmp_xy_idx(const void* pa, const void* pb)
{
    const opt_t* a = (const opt_t*)pa;
    const opt_t* b = (const opt_t*)pb;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* Twice the signed area of triangle (o, a, b); > 0 for a left turn. */
static int64_t cross3(const opt_t* o, const opt_t* a, const opt_t* b)
{
    int64_t ax = (int64_t)a->x - o->x, ay = (int64_t)a->y - o->y;
    int64_t bx = (int64_t)b->x - o->x, by = (int64_t)b->y - o->y;
    return ax * by - ay * bx;
}

/* Index of the first point outside the domain, or -1 if all are valid. */
int64_t oracle_first_invalid(const float* xy, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        if (!in_domain(xy[2 * i]) || !in_domain(xy[2 * i + 1])) return i;
    }
    return -1;
}

/*
 * xy:      n interleaved (x, y) float32 pairs (host memory).
 * out_idx: capacity >= n (the hull never has more vertices than points).
 * out_h:   receives the number of hull vertices written.
 * Returns ORACLE_OK, ORACLE_EDOMAIN, ORACLE_EINVAL or ORACLE_ENOMEM.
 */
int oracle_hull(const float* xy, int64_t n, int32_t* out_idx, int64_t* out_h)
{
    if (n < 0 || !out_h || (n > 0 && (!xy || !out_idx))) return ORACLE_EINVAL;
    if (n > INT32_MAX) return ORACLE_EINVAL;
    *out_h = 0;
    if (n == 0) return ORACLE_OK;
    if (oracle_first_invalid(xy, n) >= 0) return ORACLE_EDOMAIN;

    opt_t* p = (opt_t*)malloc((size_t)n * sizeof(opt_t));
    opt_t** chain = (opt_t**)malloc((size_t)(2 * n + 2) * sizeof(opt_t*));
    if (!p || !chain) {
        free(p);
        free(chain);
        return ORACLE_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        p[i].x = (int32_t)xy[2 * i];
        p[i].y = (int32_t)xy[2 * i + 1];
        p[i].idx = (int32_t)i;
    }
    qsort(p, (size_t)n, sizeof(opt_t), cmp_xy_idx);

    /* Keep the first of every run of equal coordinates: it has the min idx. */
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (m > 0 && p[m - 1].x == p[i].x && p[m - 1].y == p[i].y) continue;
        p[m++] = p[i];
    }

    int64_t h = 0;
    if (m == 1) {
        chain[h++] = &p[0];
    } else {
        /* Lower chain, left to right; pop on non-left turns so that
         * collinear points are excluded. */
        for (int64_t i = 0; i < m; ++i) {
            while (h >= 2 && cross3(chain[h - 2], chain[h - 1], &p[i]) <= 0) --h;
            chain[h++] = &p[i];
        }
        /* Upper chain, right to left, stacked on top of the lower one. */
        int64_t lower = h;
        for (int64_t i = m - 2; i >= 0; --i) {
            while (h > lower && cross3(chain[h - 2], chain[h - 1], &p[i]) <= 0) --h;
            chain[h++] = &p[i];
        }
        --h; /* the last point repeats the first */
    }

    /* Rotate so the output starts at the smallest (y, x). */
    int64_t start = 0;
    for (int64_t k = 1; k < h; ++k) {
        const opt_t* a = chain[k];
        const opt_t* b = chain[start];
        if (a->y < b->y || (a->y == b->y && a->x < b->x)) start = k;
    }
    for (int64_t k = 0; k < h; ++k) out_idx[k] = chain[(start + k) % h]->idx;
    *out_h = h;

    free(chain);
    free(p);
    return ORACLE_OK;
}
