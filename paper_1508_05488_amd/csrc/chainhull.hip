// chainhull: the CudaChain hot path (Section 2.1, steps 1-7) as hand-written
// gfx950 kernels, the pipeline around them and the C ABI.
//
// Kernels of one hull (all on the caller's stream):
//   k_sample        a sample of the points: per-frame slot minima, merged
//                   into the call's table by atomic maxima of complements
//   k_stream        the one full pass over the points: each workgroup turns
//                   the table into the sampled staircases (prefix minima),
//                   then the domain check and the staircase dominance test;
//                   lists the points that pass it (the extreme points are
//                   among them) and its extreme keys
//   k_cand          step 1's reduction of the extreme keys (every
//                   workgroup; the first publishes the quadrilateral and
//                   starts the call's header), step 2's exact region test on
//                   the listed points, a chunk staircase; each workgroup
//                   sorts its records by sort bucket (region, top k1 bits) in
//                   its own part and writes its row of the bucket table
//   k_scan          the bucket table's columns: bucket sizes, where each
//                   bucket starts, the SPA threshold entering it
//   k_bucket_spa    steps 3-5: each bucket gathered from the rows' parts,
//                   ordered by its low k1 bits and filtered by SPA
//   k_chain         step 6: the chains concatenated, shortened by a
//                   pre-hull per segment
//   k_finish_wide   step 7 across workgroups: every kept point tested
//                   against tangents to its neighbours' hulls
// (hull2d falls back to Melkman on the host only if the device finish gives
// up; chainhull_polygon stops after k_chain and returns the polygon.)
//
// Data layout in HBM (one workspace per device and stream):
//   points           caller's n x float32[2], read once in full (k_stream)
//   DevHeader        extreme points, quadrilateral edges, frames, counters;
//                    with the look-back states and the sample table it is
//                    zeroed when the workspace is allocated
//   stab             the sample's slot minima, complemented (4 x 1024 words,
//                    then 4 x 256 for the frames' first slots; zero again
//                    after every call)
//   ExtPartial[G]    per-workgroup extreme keys
//   open lists       per k_stream workgroup: index; x | y << 23 | mask << 46
//   key[2], val[2]   records: u32 q << 23 | k1, u64 k2 << 32 | index; per
//                    k_cand workgroup a part in each: [0] in chunk order,
//                    [1] by bucket
//   rowoff, rowmin   the bucket table: per k_cand workgroup and bucket the
//                    first position in its part, the smallest k2
//   bucket arrays    sizes, starts, thresholds, survivors (8192 buckets)
//   chain, kept      SPA survivors (index, x, y) at their bucket's place;
//                    the pre-hull's kept points per 1024-point segment
//
// Regions follow the paper (R1 lower left, R2 lower right, R3 upper right,
// R4 upper left); q = r - 1 is the region code in the sort key, so ascending
// keys list the chains in the polygon's counter-clockwise order
// P_minx -> R1 -> P_miny -> R2 -> P_maxx -> R3 -> P_maxy -> R4.
//
// Each region is sorted and filtered in its own frame (k1, k2), a rotation of
// R1's frame (x, y): ascending k1 is Table 1's primary order, and SPA
// (Figure 2) keeps a point iff its k2 is strictly below the k2 of every
// earlier point of the region and of the region's first point.
//   R1: k1 = x,     k2 = y        first point P_minx
//   R2: k1 = y,     k2 = M - x    first point P_miny
//   R3: k1 = M - x, k2 = M - y    first point P_maxx
//   R4: k1 = M - y, k2 = x        first point P_maxy
// with M = 2^23 - 1 (so M - v == v ^ M for 0 <= v <= M).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "chainhull.h"
#include "finish.h"

// The fixed device buffer of hull2d_noalloc (callers that cannot allocate):
// one copy per device, held from the code object's load until the process
// ends.  Host code never uses this name as an address: it takes the
// device's address from hipGetSymbolAddress (noalloc_base).
static __device__ __align__(256) unsigned char scratch[CH_NOALLOC_SCRATCH_BYTES];

namespace chainhull {

typedef float v2f __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef unsigned long long u64;
typedef long long i64;

constexpr uint32_t kM = (1u << 23) - 1;
constexpr int kBlock = 256;        // threads per workgroup (4 waves of 64)
constexpr int kWaves = kBlock / 64;
// Chunk-filter slots of region q, by u = k1 minus the k1 of the region's
// first point: kFineSlots slots of 2^kFineShift values at the region's start
// (where the sampled staircase knows nothing, and where open points crowd
// on inputs that fill their bounding box), then slots of 2^kCoarseShift.
constexpr int kFineSlots = 128;
constexpr int kFineShift = 7;
constexpr int kCoarseShift = 14;
constexpr int kSlots = kFineSlots + (1 << (23 - kCoarseShift));  // 640 per region
__device__ inline uint32_t chunk_slot(uint32_t u)
{
    constexpr uint32_t kFineEnd = (uint32_t)kFineSlots << kFineShift;
    return u < kFineEnd ? (u >> kFineShift) : kFineSlots + ((u - kFineEnd) >> kCoarseShift);
}
// Buckets of the region sort: region q and the top kBucketBits bits of k1;
// inside a bucket, k1's low kLowBits bits address an LDS table directly.
constexpr int kBucketBits = 11;
constexpr int kLowBits = 23 - kBucketBits;
constexpr int kBuckets = 4 << kBucketBits;        // 8192
constexpr int kLowSize = 1 << kLowBits;           // 4096

constexpr uint32_t kErrDomain = 1;   // a coordinate is outside the domain
constexpr int32_t kBatchRedo = INT32_MIN;  // a count: the batched kernel left the set to the single-hull path

// The small-input path runs the batched kernel on the one set first and the
// single-hull kernels after it gated on its count (gate): they do their work
// only if it left kBatchRedo, and return at once otherwise.
__device__ inline bool gated_off(const int32_t* gate) { return gate && *gate != kBatchRedo; }

#ifdef CH_PHASE_TIMING
// Instrumented builds only: the batched kernel's time per phase, summed over
// the sets that finish ([0, 8): batched path, [8, 16): list mode; 100 MHz
// ticks of the workgroup's thread 0), and the sets counted ([16], [17]).
__device__ unsigned long long g_phase_ticks[18];
#define CH_PHASE_MARK(k) (ph[k] = __builtin_amdgcn_s_memrealtime())
#else
#define CH_PHASE_MARK(k) ((void)0)
#endif

struct DevHeader {
    double ec[4];        // ex*E_q.y - ey*E_q.x for the edge E_q -> E_{q+1}
    int32_t ex[4], ey[4];
    uint32_t ext_x[4], ext_y[4], ext_idx[4];  // P_minx, P_miny, P_maxx, P_maxy
    uint32_t sigma[4];   // k2 of each region's first point
    uint32_t err;
    uint32_t s1[4];      // round-1 survivors per region (chainhull_polygon)
    uint32_t cand;       // sort records (after the dominance filters)
    uint32_t open;       // points listed by k_stream
    uint32_t s2[4];      // SPA survivors per region
    uint32_t chain;      // SPA survivors in all (chain points before the pre-hull)
    uint32_t fin_done;   // 1 when the device finish wrote the hull
    int32_t fin_hull;    // its size
    uint32_t fin_w2[4];  // polygon vertices per region it finished from
    uint32_t gat_count;  // polygon vertices k_gather wrote for the host finish
    uint32_t unused0;
    uint32_t epoch;      // calls on this workspace so far (tags the look-back states)
    uint32_t wide_ticket;  // k_finish_wide's next item
    uint32_t fin_fail;   // 1 when k_finish_wide gave up (the host finishes)
    int32_t list_count;  // (host copy only) the list mode's count, for hull2d
    uint32_t pad[3];
};

// Extreme keys: key 0 = x << 32 | (M - y), key 1 = y << 32 | x; P_minx and
// P_maxx are the minimum and maximum of key 0, P_miny and P_maxy of key 1.
struct ExtPartial {
    u64 kmin[2], kmax[2];
    uint32_t imin[2], imax[2];
    uint32_t err;
    uint32_t pad[3];
};

struct PolyRec {
    int32_t idx, x, y;
};

// Per-bucket arrays of one call (device memory).
struct Buckets {
    uint32_t* cnt;     // records per bucket (k_scan)
    uint32_t* off;     // first record of each bucket in bucket order (k_bucket_spa)
    uint32_t* surv;    // SPA survivors per bucket (k_bucket_spa)
    uint32_t* lstart;  // first record of the bucket among its k_scan workgroup's buckets
    uint32_t* lthr;    // smallest k2 over the earlier buckets of its k_scan workgroup
    uint32_t* bmin;    // smallest k2 of the bucket's records (k_scan)
    uint32_t* wtot;    // per k_scan workgroup: records
    uint32_t* wmin;    // per k_scan workgroup: smallest k2
};

// ---------------------------------------------------------------------------
// Wave and workgroup helpers (wave64)
// ---------------------------------------------------------------------------

__device__ inline uint32_t lane_id() { return __lane_id(); }

// The lanes whose predicate holds.
__device__ inline u64 ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

// The lanes with a > b (unsigned): the comparison's lane mask as it is (a
// ballot of a combination of comparisons goes through a register and a
// second comparison).
__device__ inline u64 cmp_mask_gt(uint32_t a, uint32_t b) { return __builtin_amdgcn_uicmp(a, b, 34 /* ugt */); }

// Cross-workgroup hand-offs inside one kernel.  The last workgroup to
// arrive reads what the others wrote: they store it with device-scope
// stores (written through to where every XCD sees it, instead of a
// device-scope release fence, which would write back the whole L2 of the
// XCD), wait until those stores have completed, and only then count their
// arrival; the last arrival takes a device-scope acquire and reads.
__device__ inline void st_dev(uint32_t* p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void st_dev(u64* p, u64 v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void stores_done()
{
    // (a workgroup-scope release orders the compiler but waits for nothing:
    // the explicit wait makes the device-scope stores complete first)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}
// The last arrival, before it reads what the others stored: a device-scope
// acquire (drops stale cache lines once; the reads are plain loads, issued
// together).
__device__ inline void last_arrival_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
// Arrival counter: returns the count before this arrival.
__device__ inline uint32_t arrive(uint32_t* ctr) { return __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

__device__ inline void take_min(u64& k, uint32_t& i, u64 ok, uint32_t oi)
{
    if (ok < k || (ok == k && oi < i)) {
        k = ok;
        i = oi;
    }
}

__device__ inline void take_max(u64& k, uint32_t& i, u64 ok, uint32_t oi)
{
    if (ok > k || (ok == k && oi < i)) {
        k = ok;
        i = oi;
    }
}


// Inclusive and exclusive minimum scans over the wave without the LDS
// crossbar: DPP row shifts inside each row of 16 lanes, then the rows'
// totals by readlane.  (DPP row_shr:n, control 0x110 + n; a lane whose
// source lies outside its row keeps the identity.)
__device__ inline uint32_t dpp_row_shr(uint32_t v, int ctrl_n)
{
    switch (ctrl_n) {
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x111, 0xf, 0xf, false);
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x112, 0xf, 0xf, false);
    case 4: return (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x114, 0xf, 0xf, false);
    default: return (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x118, 0xf, 0xf, false);
    }
}

__device__ inline void wave_min_scan(uint32_t v, uint32_t& incl, uint32_t& excl, uint32_t& total)
{
    const uint32_t lane = lane_id();
    v = min(v, dpp_row_shr(v, 1));
    v = min(v, dpp_row_shr(v, 2));
    v = min(v, dpp_row_shr(v, 4));
    v = min(v, dpp_row_shr(v, 8));
    // v: inclusive minimum inside the row; the rows' totals
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = min(r0, (uint32_t)__builtin_amdgcn_readlane((int)v, 31));
    const uint32_t r2 = min(r1, (uint32_t)__builtin_amdgcn_readlane((int)v, 47));
    const uint32_t before = lane < 16 ? ~0u : lane < 32 ? r0 : lane < 48 ? r1 : r2;
    incl = min(v, before);
    total = min(r2, (uint32_t)__builtin_amdgcn_readlane((int)v, 63));
    // exclusive: the row's shifted inclusive value, the earlier rows' total
    // at a row's first lane
    const uint32_t sh = dpp_row_shr(v, 1);
    excl = (lane & 15u) == 0 ? before : min(sh, before);
}

// DPP row shift by n with 0 for the lanes whose source lies outside the row.
__device__ inline uint32_t dpp_row_shr0(uint32_t v, int ctrl_n)
{
    switch (ctrl_n) {
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
    case 4: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
    default: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
    }
}

// Inclusive sum and minimum scans over the wave (every lane active), by DPP
// row shifts and the rows' totals through readlane.
__device__ inline uint32_t wave_incl_sum(uint32_t v)
{
    const uint32_t lane = lane_id();
    v += dpp_row_shr0(v, 1);
    v += dpp_row_shr0(v, 2);
    v += dpp_row_shr0(v, 4);
    v += dpp_row_shr0(v, 8);
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = r0 + (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t r2 = r1 + (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    return v + (lane < 16 ? 0u : lane < 32 ? r0 : lane < 48 ? r1 : r2);
}

__device__ inline uint32_t wave_incl_min(uint32_t v)
{
    uint32_t incl, excl, total;
    wave_min_scan(v, incl, excl, total);
    return incl;
}

// The sum over the wave, in every lane (every lane active).
__device__ inline uint32_t wave_sum(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_sum(v), 63); }

// Exclusive workgroup sum of one value per thread (W waves); `total` gets
// the sum.
template <int W = kWaves>
__device__ inline uint32_t block_excl_sum(uint32_t v, uint32_t* scratch, uint32_t& total)
{
    const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
    const uint32_t incl = wave_incl_sum(v);
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t s = scratch[w];
        before += (w < (int)wave) ? s : 0u;
        all += s;
    }
    __syncthreads();
    total = all;
    return before + incl - v;
}

// Exclusive workgroup minimum (identity ~0u, W waves); `total` gets the
// minimum.
template <int W = kWaves>
__device__ inline uint32_t block_excl_min(uint32_t v, uint32_t* scratch, uint32_t& total)
{
    const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
    const uint32_t incl = wave_incl_min(v);
    uint32_t excl = __shfl_up(incl, 1);
    if (lane == 0) excl = ~0u;
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    uint32_t before = ~0u, all = ~0u;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t s = scratch[w];
        if (w < (int)wave) before = min(before, s);
        all = min(all, s);
    }
    __syncthreads();
    total = all;
    return min(before, excl);
}

// ---------------------------------------------------------------------------
// Step 1 (Section 2.1 step 1; Section 2.2.1): the four extreme points by a
// parallel reduction, fused with domain validation.  Two lexicographic keys
// serve all four: K0 = (x, M - y) has its minimum at P_minx (min x, then max
// y) and its maximum at P_maxx (max x, then min y); K1 = (y, x) has its
// minimum at P_miny and its maximum at P_maxy.  Ties go to the smallest index.
// ---------------------------------------------------------------------------

// Per-lane extreme keys (with indices), the domain flag and the largest
// coordinate.  A maximum still at its initial (0, ~0u) after the reduction
// means that every key is 0; the minimum's index is then the answer
// (make_quad).
struct ExtAcc {
    u64 kmin[2], kmax[2];
    uint32_t imin[2], imax[2];
    uint32_t hi;
    bool bad;
};

__device__ inline void ext_init(ExtAcc& a)
{
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        a.kmin[e] = ~0ull;
        a.kmax[e] = 0;
        a.imin[e] = ~0u;
        a.imax[e] = ~0u;
    }
    a.bad = false;
    a.hi = 0;
}

// Integer value of a coordinate clamped to [0, 2^24]; NaN gives 0.
__device__ inline uint32_t coord_u32(float v) { return (uint32_t)fminf(fmaxf(v, 0.0f), 16777216.0f); }

// The hardware conversion: truncates, saturates to [0, 2^32 - 1], NaN gives 0.
__device__ inline uint32_t cvt_u32_sat(float v)
{
    uint32_t r;
    asm("v_cvt_u32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// Domain check of one point, X and Y its conversions: a coordinate is in
// the domain iff its conversion converts back to it exactly (so it is an
// integer, not NaN, not negative apart from -0) and the maximum over all
// coordinates is at most M.
__device__ inline void ext_check(ExtAcc& a, float fx, float fy, uint32_t X, uint32_t Y)
{
    a.bad = a.bad | ((float)X != fx) | ((float)Y != fy);
    a.hi = max(a.hi, max(X, Y));
}

// One candidate for the extreme points, in any order: ties of a key go to
// the smaller index.
__device__ inline void ext_take(ExtAcc& a, uint32_t X, uint32_t Y, uint32_t idx)
{
    const u64 k0 = ((u64)X << 32) | (Y ^ kM);
    const u64 k1 = ((u64)Y << 32) | X;
    take_min(a.kmin[0], a.imin[0], k0, idx);
    take_max(a.kmax[0], a.imax[0], k0, idx);
    take_min(a.kmin[1], a.imin[1], k1, idx);
    take_max(a.kmax[1], a.imax[1], k1, idx);
}

__device__ inline void ext_combine(ExtAcc& a, const ExtAcc& b)
{
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        take_min(a.kmin[e], a.imin[e], b.kmin[e], b.imin[e]);
        take_max(a.kmax[e], a.imax[e], b.kmax[e], b.imax[e]);
    }
    a.bad |= b.bad;
    a.hi = max(a.hi, b.hi);
}

// The smallest value over the wave, in every lane: DPP row shifts inside
// each row of 16 lanes, then the four rows' minima by readlane (no LDS
// crossbar round trips).
__device__ inline uint32_t wave_min_all(uint32_t v)
{
    v = min(v, dpp_row_shr(v, 1));
    v = min(v, dpp_row_shr(v, 2));
    v = min(v, dpp_row_shr(v, 4));
    v = min(v, dpp_row_shr(v, 8));
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    return min(min(r0, r1), min(r2, r3));
}

__device__ inline uint32_t wave_min(uint32_t v) { return wave_min_all(v); }

// The lexicographically smallest (hi, lo) over the wave and, among the lanes
// holding it, the smallest index: three wave minima.
__device__ inline void wave_lex_min(uint32_t& hi, uint32_t& lo, uint32_t& idx)
{
    const uint32_t mh = wave_min_all(hi);
    const uint32_t ml = wave_min_all(hi == mh ? lo : ~0u);
    idx = wave_min_all(hi == mh && lo == ml ? idx : ~0u);
    hi = mh;
    lo = ml;
}

// The smallest 64-bit value over the wave, in every lane (high words, then
// the low words of the lanes holding the smallest high word).
__device__ inline u64 wave_min_u64(u64 v)
{
    const uint32_t h = (uint32_t)(v >> 32), l = (uint32_t)v;
    const uint32_t mh = wave_min_all(h);
    const uint32_t ml = wave_min_all(h == mh ? l : ~0u);
    return ((u64)mh << 32) | ml;
}

// Every lane ends with the wave's result (ties of a key to the smaller index,
// as take_min / take_max); maxima as minima of the complements.
__device__ inline void ext_wave_reduce(ExtAcc& a)
{
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        uint32_t h = (uint32_t)(a.kmin[e] >> 32), l = (uint32_t)a.kmin[e];
        wave_lex_min(h, l, a.imin[e]);
        a.kmin[e] = ((u64)h << 32) | l;
        h = ~(uint32_t)(a.kmax[e] >> 32);
        l = ~(uint32_t)a.kmax[e];
        wave_lex_min(h, l, a.imax[e]);
        a.kmax[e] = ((u64)~h << 32) | ~l;
    }
    a.hi = ~wave_min_all(~a.hi);
    a.bad = ballot(a.bad) != 0;
}

// Reduce over the workgroup (W waves); thread 0 gets the result.
template <int W = kWaves>
__device__ inline void ext_block_reduce(ExtAcc& a, ExtAcc* sh)
{
    ext_wave_reduce(a);
    if (lane_id() == 0) sh[threadIdx.x / 64] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < W; ++w) ext_combine(a, sh[w]);
    }
}

// ---------------------------------------------------------------------------
// Steps 1-2 (Section 2.1 step 1; Section 2.1.1) in one pass over the points,
// with the SPA dominance rule used as an early filter.
//
// A point p of region q is dominated by another point p' of the region when
// k1' <= k1 and k2' <= k2 and p' precedes p in (k1, k2, index) order; then p
// lies in the triangle (first point, p', last point) and is not a hull vertex
// (the argument of Figure 3).  Dropping dominated points leaves the result of
// the region sort and SPA unchanged, so any filter that only drops dominated
// points may run before them.
//
// Sampled staircases.  k_sample takes a sample of up to kSamplePts points
// (up to kSampleBlocks evenly spaced runs of consecutive points, about one
// run per eight of the input) and records, in
// each of the four region frames, the smallest k2 per slot of 2^kStairShift
// k1 values, over all sample points (not only the region's), then turns them
// into exclusive prefix minima over the slots.  A sample
// point p' with smaller k1 and k2 <= k2 of p in the frame of p's region lies
// in that region as well (moving towards the corner never re-enters the
// quadrilateral), so it dominates p there.  A point whose k2 is not below
// the staircase in any of the four frames is therefore dominated in its own
// region, or lies in no region, whatever the extreme points turn out to be:
// the test needs no extreme point and runs in the same pass that finds them.
//
// k_stream reads every point once: the domain check and the staircase test;
// the points that pass it ("open" points) go, with their 4-bit frame mask,
// to a per-wave list in LDS that is flushed to the workgroup's region.  The
// extreme points are found among the open points only: every point with the
// smallest x is open in frame R1 (no sample has a smaller x, so the
// staircase is empty up to its slot), and likewise every point with the
// smallest y (R2), the largest x (R3) and the largest y (R4); so the
// lexicographic extremes of the open points, ties to the smallest index,
// are those of all points.  The last k_stream workgroup reduces them; k_cand
// runs the exact region test on the open points only (a point counts for its region only if
// it passed that region's frame), and filters again with a staircase over
// chunks of kCandChunk records: per region and k1-slot (chunk_slot) the smallest
// (k2, k1) in LDS; a record is dropped when the region's first point or a
// record of an earlier slot has k2 <= its k2, or when its slot's smallest
// record precedes it with k1 <= its k1.  The rest become sort records.
// ---------------------------------------------------------------------------

constexpr int kSampleBlocks = 128;
constexpr int kSamplePerThread = 16;
constexpr uint32_t kSamplePts = (uint32_t)kSampleBlocks * kBlock * kSamplePerThread;
// An input of at most kSelfSampleMax points skips k_sample: every k_stream
// workgroup takes its own sample, kBlock * kSamplePerThread evenly spaced
// points, into LDS (one launch less; such an input leaves few open points
// with that sample too).
constexpr uint32_t kSelfSampleMax = 1u << 18;
constexpr int kStairBits = 10;
constexpr int kStairSlots = 1 << kStairBits;
constexpr int kStairShift = 23 - kStairBits;
// Each frame's first slot (k1 below 2^kStairShift) again at a finer step:
// its test has no earlier slot, so without these every point of it would
// pass (the four edge strips of a uniform input hold 4 / kStairSlots of it).
constexpr int kEdgeBits = 8;
constexpr int kEdgeSub = 1 << kEdgeBits;
constexpr int kEdgeShift = kStairShift - kEdgeBits;
constexpr int kStabWords = 4 * kStairSlots + 4 * kEdgeSub;  // the sample table
constexpr int kStreamGrid = 1024;   // k_stream workgroups at most (the partials' room)
constexpr int kWaveList = 256;      // open points listed per wave before a flush

// A slot pair's two frames as one interval of the other coordinate: the
// point is dominated in both iff that coordinate lies in [lo, M - cf]
// (lo: the lower frame's staircase, cf: the upper frame's), stored as
// a | w << 32 with w = M - cf - a; an empty interval as a = ~0u, w = 0.
__device__ inline u64 stair_interval(uint32_t lo, uint32_t cf)
{
    const bool some = cf <= kM && lo <= kM - cf;
    return some ? ((u64)(kM - cf - lo) << 32) | lo : (u64)~0u;
}

// The frames in which a point outside its slots' intervals is open (bit
// f - 1 for frame Rf): R1 below the y interval [ax, ax + wx], R3 above it,
// R4 below the x interval [ay, ay + wy], R2 above it; an empty interval
// (a = ~0u) opens both of its frames.
__device__ inline uint32_t open_frames(uint32_t X, uint32_t Y, uint32_t ax, uint32_t wx, uint32_t ay, uint32_t wy)
{
    const bool ex = ax == ~0u, ey = ay == ~0u;
    const bool o1 = ex | (Y < ax), o3 = ex | (Y > ax + wx);
    const bool o4 = ey | (X < ay), o2 = ey | (X > ay + wy);
    return (o1 ? 1u : 0u) | (o2 ? 2u : 0u) | (o3 ? 4u : 0u) | (o4 ? 8u : 0u);
}

// Open-point record: X | Y << 23 | frame mask << 46.
__device__ inline u64 open_rec(uint32_t X, uint32_t Y, uint32_t mask)
{
    return (u64)X | ((u64)Y << 23) | ((u64)mask << 46);
}

// One sample point (X, Y) into the slot minima st (LDS, the table layout
// below, ~0u: no point yet).  Every lane of the wave calls it together.
__device__ inline void sample_point(uint32_t* st, uint32_t X, uint32_t Y)
{
    const uint32_t xm = X ^ kM, ym = Y ^ kM;
    atomicMin(&st[0 * kStairSlots + (X >> kStairShift)], Y);   // R1: (x, y)
    atomicMin(&st[1 * kStairSlots + (Y >> kStairShift)], xm);  // R2: (y, M-x)
    atomicMin(&st[2 * kStairSlots + (xm >> kStairShift)], ym); // R3: (M-x, M-y)
    atomicMin(&st[3 * kStairSlots + (ym >> kStairShift)], X);  // R4: (M-y, x)
    // a frame's first slot by sub-slot as well (few points: one wave-wide
    // test first)
    constexpr uint32_t E = 4 * kStairSlots;
    const bool ex0 = (X >> kStairShift) == 0, ey0 = (Y >> kStairShift) == 0;
    const bool ex1 = (xm >> kStairShift) == 0, ey1 = (ym >> kStairShift) == 0;
    if (ballot(ex0 | ey0 | ex1 | ey1)) {
        if (ex0) atomicMin(&st[E + 0 * kEdgeSub + (X >> kEdgeShift)], Y);
        if (ey0) atomicMin(&st[E + 1 * kEdgeSub + (Y >> kEdgeShift)], xm);
        if (ex1) atomicMin(&st[E + 2 * kEdgeSub + (xm >> kEdgeShift)], ym);
        if (ey1) atomicMin(&st[E + 3 * kEdgeSub + (ym >> kEdgeShift)], X);
    }
}

// k_sample: workgroup b reads a run of kBlock * kSamplePerThread consecutive
// points (coalesced), the runs evenly spaced (a smaller input is sampled with
// repeats at evenly spaced indices), takes its per-frame slot minima in LDS
// and merges them into the call's table stab by atomic maxima of their
// complements (so that zero, the cleared state, stands for an empty slot).
// Table layout: frame f's slots at [f*S, (f+1)*S), S = kStairSlots; R1 by
// x-slot, R2 by y-slot, R3 by (M-x)-slot, R4 by (M-y)-slot.  k_cand clears
// the table again once k_stream has read it.
__global__ __launch_bounds__(kBlock) void k_sample(const float* __restrict__ pts, uint32_t n, uint32_t runs,
                                                   uint32_t step, uint64_t mul, uint32_t* __restrict__ stab,
                                                   const int32_t* __restrict__ gate)
{
    __shared__ __align__(16) uint32_t st[kStabWords];
    const uint32_t tid = threadIdx.x;
    if (gated_off(gate)) return;
    for (int e = tid; e < kStabWords; e += kBlock) st[e] = ~0u;
    __syncthreads();
    // runs: workgroup b's run starts at b * step; otherwise (an input smaller
    // than the gridDim.x runs) sample j reads point floor(j * mul / 2^32),
    // mul = floor(n * 2^32 / (gridDim.x * kBlock * kSamplePerThread)) < n
    const uint32_t start = blockIdx.x * step;
    uint32_t X[kSamplePerThread], Y[kSamplePerThread];  // every point load of a thread in flight together
#pragma unroll
    for (int k = 0; k < kSamplePerThread; ++k) {
        const uint32_t sidx = (blockIdx.x * kBlock + tid) * kSamplePerThread + k;
        const uint32_t i = runs ? start + k * kBlock + tid : (uint32_t)(((u64)sidx * mul) >> 32);
        const v2f p = *reinterpret_cast<const v2f*>(pts + 2 * (size_t)i);
        // out-of-domain values only need to stay in range here: such a call
        // fails with a domain error
        X[k] = coord_u32(p.x) & kM;
        Y[k] = coord_u32(p.y) & kM;
    }
#pragma unroll
    for (int k = 0; k < kSamplePerThread; ++k) sample_point(st, X[k], Y[k]);
    __syncthreads();
    for (int e = tid; e < kStabWords; e += kBlock)
        if (st[e] != ~0u) atomicMax(stab + e, ~st[e]);
}

// The quadrilateral: extreme points, edges and frames, from the reduced
// extreme keys.
struct Quad {
    uint32_t X[4], Y[4], idx[4];  // P_minx, P_miny, P_maxx, P_maxy
    int32_t ex[4], ey[4];         // edge q runs from E_q to E_{q+1}
    double ec[4];                 // ex*E_q.y - ey*E_q.x
    uint32_t sigma[4];            // k2 of each region's first point
    uint32_t err;
};

// The edges and the regions' first keys from the extreme points Q.X, Q.Y.
__device__ inline void quad_edges(Quad& Q)
{
    // region q lies strictly right of edge q: ex*(y - E_q.y) - ey*(x - E_q.x) < 0
    for (int q = 0; q < 4; ++q) {
        const int s = (q + 1) & 3;
        Q.ex[q] = (int32_t)Q.X[s] - (int32_t)Q.X[q];
        Q.ey[q] = (int32_t)Q.Y[s] - (int32_t)Q.Y[q];
        Q.ec[q] = (double)Q.ex[q] * (double)Q.Y[q] - (double)Q.ey[q] * (double)Q.X[q];
    }
    Q.sigma[0] = Q.Y[0];        // R1 starts at P_minx
    Q.sigma[1] = Q.X[1] ^ kM;   // R2 starts at P_miny
    Q.sigma[2] = Q.Y[2] ^ kM;   // R3 starts at P_maxx
    Q.sigma[3] = Q.X[3];        // R4 starts at P_maxy
}

__device__ inline void make_quad(ExtAcc r, Quad& Q)
{
    for (int e = 0; e < 2; ++e) {
        if (r.imax[e] == ~0u) {  // every key is 0: the minimum is the answer
            r.kmax[e] = r.kmin[e];
            r.imax[e] = r.imin[e];
        }
    }
    // masked so that a rejected input still gives in-range values
    const u64 key[4] = {r.kmin[0], r.kmin[1], r.kmax[0], r.kmax[1]};
    Q.idx[0] = r.imin[0];
    Q.idx[1] = r.imin[1];
    Q.idx[2] = r.imax[0];
    Q.idx[3] = r.imax[1];
    Q.X[0] = (uint32_t)(key[0] >> 32) & kM; Q.Y[0] = ((uint32_t)key[0] & kM) ^ kM;
    Q.Y[1] = (uint32_t)(key[1] >> 32) & kM; Q.X[1] = (uint32_t)key[1] & kM;
    Q.X[2] = (uint32_t)(key[2] >> 32) & kM; Q.Y[2] = ((uint32_t)key[2] & kM) ^ kM;
    Q.Y[3] = (uint32_t)(key[3] >> 32) & kM; Q.X[3] = (uint32_t)key[3] & kM;
    quad_edges(Q);
    Q.err = r.bad ? kErrDomain : 0u;
}

// The quadrilateral from k_stream's per-workgroup extreme partials (a few
// tens of KB): thread t of a workgroup of W waves takes partial t (nparts
// <= 64 W); every thread returns with it in *sq.
template <int W>
__device__ inline void quad_from_partials(const ExtPartial* __restrict__ part, uint32_t nparts, ExtAcc* sh,
                                          Quad* sq)
{
    ExtAcc r;
    ext_init(r);
    if (threadIdx.x < nparts) {
        const ExtPartial p = part[threadIdx.x];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            r.kmin[e] = p.kmin[e];
            r.kmax[e] = p.kmax[e];
            r.imin[e] = p.imin[e];
            r.imax[e] = p.imax[e];
        }
        r.bad = p.err != 0;
    }
    ext_block_reduce<W>(r, sh);
    if (threadIdx.x == 0) make_quad(r, *sq);
    __syncthreads();
}

// `head` leading points (0 or 1) are visited singly so that the rest of the
// array is 16-byte aligned for float4 loads; an odd last point likewise.
// Workgroup b writes its open points to its own region [b*region, ...) of
// the open arrays and their number to wgcount[b]: no two workgroups share a
// counter (same-address atomics from many workgroups serialise).  `per`
// float4s per workgroup, a multiple of kBlock*kStreamUnroll (the float4
// loads in flight per thread).  kSelfSample: the workgroup takes its own
// sample instead of reading stab: kSamplePerThread runs of kBlock
// consecutive points (coalesced), run k from floor(k * smul / 2^32), smul =
// floor(max(n - kBlock, 0) * 2^32 / (kSamplePerThread - 1)).
template <int kStreamUnroll, bool kSelfSample = false>
__global__ __launch_bounds__(kBlock) void k_stream(const float* __restrict__ pts, uint32_t n, uint32_t head,
                                                   const uint32_t* __restrict__ stab, ExtPartial* __restrict__ part,
                                                   uint32_t* __restrict__ open_idx, u64* __restrict__ open_xym,
                                                   uint32_t per, uint32_t region, uint32_t* __restrict__ wgcount,
                                                   uint64_t smul, const int32_t* __restrict__ gate)
{
    if (gated_off(gate)) return;
    __shared__ __align__(16) uint32_t sst[4 * kStairSlots];
    __shared__ uint32_t own_tab[kSelfSample ? kStabWords : 1];  // the own sample's slot minima
    __shared__ __align__(16) u64 ssub[4 * kEdgeSub];  // the first slots' intervals by sub-slot
    __shared__ uint32_t s_last[4];                      // each frame's staircase at its last slot
    __shared__ uint32_t lidx[kWaves][kWaveList];
    __shared__ u64 lxym[kWaves][kWaveList];
    __shared__ ExtAcc sh[kWaves];
    __shared__ uint32_t s_fill;
    const uint32_t tid = threadIdx.x, wave = tid / 64, lane = lane_id();
    const u64 lt = (1ull << lane) - 1ull;

    // Workgroup b streams float4s [b*per, (b+1)*per) of the aligned part, a
    // round of kBlock*kStreamUnroll at a time.  Every lane runs the same
    // number of rounds (the list append is wave-wide); lanes past the range
    // reread its last float4, which changes nothing and lists nothing.  The
    // sample table's loads go first and the first round's point loads right
    // after them, so that the wait for the table (loads complete in issue
    // order) leaves the point loads in flight while the staircases are built.
    const v4f* p4 = reinterpret_cast<const v4f*>(pts + 2 * head);
    const uint32_t n4 = (n - head) / 2;
    constexpr uint32_t kRound = kBlock * kStreamUnroll;
    const uint32_t lo = min(n4, blockIdx.x * per), hi = min(n4, lo + per);
    const uint32_t rounds = (hi - lo + kRound - 1) / kRound;
    auto load_round = [&](uint32_t r, v4f* v) {
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u)
            v[u] = __builtin_nontemporal_load(p4 + min(lo + r * kRound + u * kBlock + tid, hi - 1));
    };
    // wave f holds frame f, lane l its slots l, l + 64, ..., l + 960
    // (coalesced loads; consecutive lanes write neighbouring LDS words)
    constexpr int kPer = kStairSlots / 64;  // 16
    static_assert(4 * 64 == kBlock, "one wave per frame");
    constexpr int kEdgePer = kEdgeSub / 64;  // 4
    uint32_t sv[kPer], ev[kEdgePer];
    if constexpr (!kSelfSample) {
#pragma unroll
        for (int k = 0; k < kPer; ++k) sv[k] = stab[wave * kStairSlots + k * 64 + lane];
#pragma unroll
        for (int k = 0; k < kEdgePer; ++k) ev[k] = stab[4 * kStairSlots + wave * kEdgeSub + k * 64 + lane];
    }
    v4f va[kStreamUnroll];
    {
        // unconditional, so that no branch joins before the table wait (a
        // workgroup without points reads the table's first bytes instead)
        const v4f* src = rounds ? p4 : reinterpret_cast<const v4f*>(stab);
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u)
            va[u] = __builtin_nontemporal_load(src + (rounds ? min(lo + u * kBlock + tid, hi - 1) : 0u));
    }
    if constexpr (kSelfSample) {
        // k_sample's slot minima of the workgroup's own sample, in LDS (the
        // first round's loads above stay in flight meanwhile); the table as
        // k_sample leaves it holds their complements
        for (int e = tid; e < kStabWords; e += kBlock) own_tab[e] = ~0u;
        uint32_t X[kSamplePerThread], Y[kSamplePerThread];
#pragma unroll
        for (int k = 0; k < kSamplePerThread; ++k) {
            const uint32_t i = min((uint32_t)(((u64)k * smul) >> 32) + tid, n - 1);
            const v2f p = *reinterpret_cast<const v2f*>(pts + 2 * (size_t)i);
            X[k] = coord_u32(p.x) & kM;  // (out of domain: in range here, the call fails)
            Y[k] = coord_u32(p.y) & kM;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSamplePerThread; ++k) sample_point(own_tab, X[k], Y[k]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPer; ++k) sv[k] = ~own_tab[wave * kStairSlots + k * 64 + lane];
#pragma unroll
        for (int k = 0; k < kEdgePer; ++k) ev[k] = ~own_tab[4 * kStairSlots + wave * kEdgeSub + k * 64 + lane];
    }
    {
        // The staircases: per frame the exclusive prefix minimum of the slot
        // minima (the table holds their complements; zero: no sample).  LDS
        // layout: sst[2s], sst[2s+1] = R1 at x-slot s, R3 at its own slot of
        // the same x; sst[2S + 2s], sst[2S + 2s + 1] = R2 at y-slot s, R4 at
        // its own slot of the same y (S = kStairSlots), so that one 64-bit
        // LDS read per coordinate serves two frames.
        const uint32_t q = wave, S = kStairSlots;
        uint32_t carry = ~0u;  // over the earlier rows of 64 slots
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            uint32_t incl, excl, tot;
            wave_min_scan(~sv[k], incl, excl, tot);
            excl = min(excl, carry);
            carry = min(carry, tot);
            const uint32_t sl = k * 64 + lane;
            const uint32_t at = q == 0 ? 2 * sl : q == 1 ? 2 * S + 2 * sl : q == 2 ? 2 * (S - 1 - sl) + 1 : 2 * S + 2 * (S - 1 - sl) + 1;
            sst[at] = excl;
            if (k == kPer - 1 && lane == 63) s_last[q] = excl;
        }
        // the frame's first slot by sub-slot: prefix minima over its sub-slots
        carry = ~0u;
#pragma unroll
        for (int k = 0; k < kEdgePer; ++k) {
            uint32_t incl, excl, tot;
            wave_min_scan(~ev[k], incl, excl, tot);
            excl = min(excl, carry);
            carry = min(carry, tot);
            ssub[q * kEdgeSub + k * 64 + lane] = excl;
        }
    }
    __syncthreads();
    {
        // Each slot's two frames as one interval of the other coordinate: a
        // point is dominated in both iff y (x-slots: R1 and R3) or x (y-slots:
        // R4 and R2) lies in [a, a + w].  R1 holds y < s1 open and R3 y >
        // M - s3, so the interval is [s1, M - s3]; R4 and R2 give [s4, M - s2].
        // Stored as a | w << 32; an empty interval as a = ~0u, w = 0 (every
        // point of the slot is open).
        const auto interval = stair_interval;
        u64* const s64 = reinterpret_cast<u64*>(sst);
        for (int e = tid; e < 2 * kStairSlots; e += kBlock) {
            const u64 v = s64[e];
            const bool xs = e < kStairSlots;
            const uint32_t lo = xs ? (uint32_t)v : (uint32_t)(v >> 32);   // s1 or s4
            const uint32_t cf = xs ? (uint32_t)(v >> 32) : (uint32_t)v;   // s3 or s2
            s64[e] = interval(lo, cf);
        }
        // The first slots by sub-slot: frame R1's first slot is x-slot 0,
        // whose interval of y is [s1, M - s3] with s3 of that x-slot (R3's
        // last slot); R2's is y-slot 0 ([s4, M - s2], s4 of R4's last slot);
        // R3's x-slot S - 1 (s1 of R1's last slot); R4's y-slot S - 1 (s2 of
        // R2's last slot).
        for (int e = tid; e < 4 * kEdgeSub; e += kBlock) {
            const uint32_t f = e / kEdgeSub, v = (uint32_t)ssub[e];
            ssub[e] = f == 0 ? interval(v, s_last[2])
                    : f == 1 ? interval(s_last[3], v)
                    : f == 2 ? interval(s_last[0], v)
                             : interval(v, s_last[1]);
        }
    }
    if (tid == 0) s_fill = 0;
    __syncthreads();
    uint32_t* const my_idx = open_idx + (size_t)blockIdx.x * region;
    u64* const my_xym = open_xym + (size_t)blockIdx.x * region;
    const u64* const sx64 = reinterpret_cast<const u64*>(sst);
    const u64* const sy64 = sx64 + kStairSlots;

    ExtAcc a;
    ext_init(a);
    uint32_t wcount = 0;  // the same in every lane of a wave

    // Flush the wave's list: a listed point of a frame's first slot is
    // tested again with that frame by sub-slot (the other frames as
    // before); the points that stay open are compacted in place (an entry
    // moves only to a position at or before its own, after every lane has
    // read its entry) and written to the workgroup's region.
    auto flush = [&]() {
        constexpr uint32_t S = kStairSlots;
        uint32_t kept = 0;  // the same in every lane
        for (uint32_t e0 = 0; e0 < wcount; e0 += 64) {
            const uint32_t e = e0 + lane;
            bool keep = false;
            uint32_t i = 0;
            u64 r = 0;
            if (e < wcount) {
                i = lidx[wave][e];
                r = lxym[wave][e];
                keep = true;
                const uint32_t X = (uint32_t)r & kM, Y = (uint32_t)(r >> 23) & kM;
                const uint32_t xs = X >> kStairShift, ys = Y >> kStairShift;
                if (xs == 0 || xs == S - 1 || ys == 0 || ys == S - 1) {
                    const u64 sxv = xs == 0       ? ssub[0 * kEdgeSub + (X >> kEdgeShift)]
                                    : xs == S - 1 ? ssub[2 * kEdgeSub + ((X ^ kM) >> kEdgeShift)]
                                                  : sx64[xs];
                    const u64 syv = ys == 0       ? ssub[1 * kEdgeSub + (Y >> kEdgeShift)]
                                    : ys == S - 1 ? ssub[3 * kEdgeSub + ((Y ^ kM) >> kEdgeShift)]
                                                  : sy64[ys];
                    const uint32_t ax = (uint32_t)sxv, wx = (uint32_t)(sxv >> 32);
                    const uint32_t ay = (uint32_t)syv, wy = (uint32_t)(syv >> 32);
                    keep = (Y - ax > wx) || (X - ay > wy);
                    r = open_rec(X, Y, open_frames(X, Y, ax, wx, ay, wy));
                }
            }
            const u64 kb = ballot(keep);
            const uint32_t at = kept + (uint32_t)__popcll(kb & lt);
            if (keep) {
                lidx[wave][at] = i;
                lxym[wave][at] = r;
            }
            kept += (uint32_t)__popcll(kb);
        }
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&s_fill, kept);
        base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);  // (every lane is active here)
        __builtin_amdgcn_wave_barrier();
        for (uint32_t e = lane; e < kept; e += 64) {
            const uint32_t i = lidx[wave][e];
            const u64 r = lxym[wave][e];
            ext_take(a, (uint32_t)r & kM, (uint32_t)(r >> 23) & kM, i);
            my_idx[base + e] = i;
            my_xym[base + e] = r;
        }
        __builtin_amdgcn_wave_barrier();
        wcount = 0;
    };
    // (out-of-domain coordinates only need to index the staircase in range:
    // such a call fails with a domain error)
    auto slot_of = [](uint32_t v) { return __builtin_amdgcn_ubfe(v, kStairShift, kStairBits); };
    // One point of every lane: list it if it is open.  Every lane of the
    // wave calls it together (the list append is wave-wide); the branch is
    // taken when some lane of the wave has an open point.
    auto list_point = [&](uint32_t X, uint32_t Y, uint32_t idx, bool valid, u64 sxv, u64 syv) {
        const uint32_t ax = (uint32_t)sxv, wx = (uint32_t)(sxv >> 32);
        const uint32_t ay = (uint32_t)syv, wy = (uint32_t)(syv >> 32);
        // outside an interval (below a wraps around past w); the lane masks
        // of the comparisons combine as they are
        const u64 bal = (cmp_mask_gt(Y - ax, wx) | cmp_mask_gt(X - ay, wy)) & ballot(valid);
        if (bal) {
            if ((bal >> lane) & 1u) {
                const uint32_t mask = open_frames(X, Y, ax, wx, ay, wy);
                const uint32_t slot = wcount + (uint32_t)__popcll(bal & lt);
                lidx[wave][slot] = idx;
                lxym[wave][slot] = open_rec(X & kM, Y & kM, mask);
            }
            wcount += (uint32_t)__popcll(bal);
            if (wcount > (uint32_t)(kWaveList - 64)) flush();
        }
    };
    auto visit_one = [&](float fx, float fy, uint32_t idx, bool valid) {
        const uint32_t X = cvt_u32_sat(fx), Y = cvt_u32_sat(fy);
        ext_check(a, fx, fy, X, Y);
        list_point(X, Y, idx, valid, sx64[slot_of(X)], sy64[slot_of(Y)]);
    };

    if (blockIdx.x == 0 && wave == 0 && head) visit_one(pts[0], pts[1], 0, lane == 0);
    // One round: the conversions and the domain checks take the loaded
    // values first, then the next round's loads reuse their registers, so
    // that the staircase reads, the tests and the list appends run with the
    // next round in flight.  The loads are unconditional (past the last
    // round they reread the range's last float4).
    constexpr int kP = 2 * kStreamUnroll;
    for (uint32_t r = 0; r < rounds; ++r) {
        uint32_t X[kP], Y[kP];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const float f[4] = {va[u].x, va[u].y, va[u].z, va[u].w};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                X[2 * u + h] = cvt_u32_sat(f[2 * h]);
                Y[2 * u + h] = cvt_u32_sat(f[2 * h + 1]);
                ext_check(a, f[2 * h], f[2 * h + 1], X[2 * u + h], Y[2 * u + h]);
            }
        }
        load_round(r + 1, va);
        // all staircase reads first, then the tests: one wait per round
        u64 sxv[kP], syv[kP];
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            sxv[p] = sx64[slot_of(X[p])];
            syv[p] = sy64[slot_of(Y[p])];
        }
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            const uint32_t g0 = lo + r * kRound + (p / 2) * kBlock + tid, g = min(g0, n4 - 1);
            list_point(X[p], Y[p], head + 2 * g + (p & 1), g0 < hi, sxv[p], syv[p]);
        }
    }
    if (blockIdx.x == 0 && wave == 0 && ((n - head) & 1u))
        visit_one(pts[2 * (n - 1)], pts[2 * (n - 1) + 1], n - 1, lane == 0);
    if (wcount) flush();

    ext_block_reduce(a, sh);  // ends with a workgroup barrier: s_fill is final
    if (tid == 0) {
        wgcount[blockIdx.x] = s_fill;
        ExtPartial p;
        for (int e = 0; e < 2; ++e) {
            p.kmin[e] = a.kmin[e];
            p.kmax[e] = a.kmax[e];
            p.imin[e] = a.imin[e];
            p.imax[e] = a.imax[e];
        }
        p.err = (a.bad || a.hi > kM) ? 1u : 0u;
        part[blockIdx.x] = p;  // (k_cand reduces the partials)
    }
}

// Region (0..3, or 4 for none) of a point by the exact test: every product is
// below 2^46 and every sum below 2^47, so fp64 is exact.
__device__ inline uint32_t region_of(const Quad& Q, uint32_t X, uint32_t Y)
{
    const double dx = (double)X, dy = (double)Y;
    const bool t0 = fma((double)Q.ex[0], dy, -((double)Q.ey[0] * dx)) < Q.ec[0];
    const bool t1 = fma((double)Q.ex[1], dy, -((double)Q.ey[1] * dx)) < Q.ec[1];
    const bool t2 = fma((double)Q.ex[2], dy, -((double)Q.ey[2] * dx)) < Q.ec[2];
    const bool t3 = fma((double)Q.ex[3], dy, -((double)Q.ey[3] * dx)) < Q.ec[3];
    return t0 ? 0u : t1 ? 1u : t2 ? 2u : t3 ? 3u : 4u;
}

// Frame coordinates (k1, k2) of a point (X, Y) in region q's frame.
__device__ inline void to_frame(uint32_t q, uint32_t X, uint32_t Y, uint32_t& k1, uint32_t& k2)
{
    const uint32_t a = (q & 1u) ? Y : X;
    const uint32_t b = (q & 1u) ? X : Y;
    k1 = (q & 2u) ? a ^ kM : a;
    k2 = ((q ^ (q >> 1)) & 1u) ? b ^ kM : b;
}

// Bucket arrays that threads read with the ownership "thread t: buckets
// kPerThreadBuckets*t .. kPerThreadBuckets*(t+1)-1" sit in LDS at bpad(b):
// one pad word per 32 puts the lanes of one read step in distinct banks.
constexpr int kPerThreadBuckets = kBuckets / kBlock;  // 32
__device__ inline uint32_t bpad(uint32_t b) { return b + (b >> 5); }
constexpr int kBucketsPadded = kBuckets + kBuckets / 32;

// k_cand: workgroup j takes the open lists of k_stream workgroups
// L*j .. L*(j+1)-1 (L = lists, a launch shape).  It runs the exact region test
// and the chunk filter on them, then sorts its records by sort bucket
// (region q and the top kBucketBits bits of k1) inside its own part of the
// record arrays: a counting sort with its histogram in LDS, so no two
// workgroups share a counter.  Its row of the bucket table receives, per
// bucket, the first position of the bucket's records in its part (and the
// total at the end) and their smallest k2.
//   pass 1  the records, in chunk order, to part A (key[0], val[0]); LDS
//           counts and smallest k2 per bucket;
//   pass 2  the counts' exclusive prefix sum: the row;
//   pass 3  the records again from part A, each to part B (key[1], val[1])
//           at its bucket's next position.
// One workgroup of 16 waves per CU (its LDS holds the histogram, the slot
// minima and the list starts): four waves per SIMD to hide the latency of
// the record loads and the region test.
constexpr int kCandBlock = 1024;
constexpr int kCandWaves = kCandBlock / 64;
constexpr int kCandChunk = 4096;                              // records filtered together
constexpr int kCandPer = kCandChunk / kCandBlock;             // 4 per thread
constexpr int kCandBucketsPer = kBuckets / kCandBlock;        // buckets per thread in pass 2
static_assert(kCandBlock >= kStreamGrid, "one list per thread");
// LDS position of bucket b in the histogram: thread t reads buckets
// 8t .. 8t+7 in pass 2, so one pad word per 8 puts a read step's lanes in
// distinct banks
__device__ inline uint32_t cpad(uint32_t b) { return b + (b >> 3); }
constexpr int kBucketsCPadded = kBuckets + kBuckets / 8;
constexpr int kCandMaxRows = 256;  // rows of the bucket table (k_cand workgroups) at most

// Rows of the bucket table for a call: one per cand_per_row open points (a
// launch shape), at least one, at most kCandMaxRows and the k_stream grid;
// row r takes lists [r*lists, min((r+1)*lists, grid)), so the rows' parts
// tile the open lists' regions.  The open count comes from k_stream, so
// k_cand, k_scan and k_bucket_spa all derive the same rows from it.
__device__ inline uint32_t cand_rows(uint32_t open, uint32_t grid, uint32_t per_row, uint32_t& lists)
{
    uint32_t r = (open + per_row - 1) / per_row;
    r = max(1u, min(r, min((uint32_t)kCandMaxRows, grid)));
    lists = (grid + r - 1) / r;
    return (grid + lists - 1) / lists;
}

__global__ __launch_bounds__(kCandBlock) void k_cand(DevHeader* __restrict__ hdr, uint32_t* __restrict__ stab,
                                                     const ExtPartial* __restrict__ parts,
                                                     const uint32_t* __restrict__ open_idx,
                                                     const u64* __restrict__ open_xym, uint32_t region,
                                                     const uint32_t* __restrict__ wgcount, uint32_t grid,
                                                     uint32_t per_row, uint32_t* __restrict__ key_a,
                                                     u64* __restrict__ val_a, uint32_t* __restrict__ key_b,
                                                     u64* __restrict__ val_b, uint32_t* __restrict__ rowoff,
                                                     uint32_t* __restrict__ rowmin, const int32_t* __restrict__ gate)
{
    __shared__ u64 smin[4 * kSlots];
    __shared__ uint32_t sexc[4 * kSlots];
    __shared__ uint32_t scratch[kCandWaves];
    __shared__ uint32_t lcnt[kBucketsCPadded];  // per bucket (at cpad): counts, then next positions
    __shared__ uint32_t lmin[kBuckets];         // smallest k2 per bucket
    __shared__ uint32_t s_start[kStreamGrid + 1];  // the lists' first positions in the concatenation
    __shared__ ExtAcc s_ext[kCandWaves];
    __shared__ Quad s_q;
    __shared__ uint32_t s_base;
    const uint32_t tid = threadIdx.x, wave = tid / 64, lane = lane_id();
    if (gated_off(gate)) return;
    // every workgroup: the open count and the quadrilateral, from k_stream's
    // per-workgroup counts and extreme partials (thread t: workgroup t)
    const uint32_t mine = tid < grid ? wgcount[tid] : 0u;
    quad_from_partials<kCandWaves>(parts, grid, s_ext, &s_q);
    uint32_t open;
    const uint32_t gpre = block_excl_sum<kCandWaves>(mine, scratch, open);  // open points of lists < tid
    if (blockIdx.x == 0) {
        // k_stream has read the sample table: cleared for the next call
        for (int e = tid; e < kStabWords; e += kCandBlock) stab[e] = 0;
    }
    if (blockIdx.x == 0 && tid == 0) {
        // the call's header: the quadrilateral and the open count for the
        // later steps, the call's counters cleared, the call counter advanced
        for (int q = 0; q < 4; ++q) {
            hdr->ext_x[q] = s_q.X[q];
            hdr->ext_y[q] = s_q.Y[q];
            hdr->ext_idx[q] = s_q.idx[q];
            hdr->ex[q] = s_q.ex[q];
            hdr->ey[q] = s_q.ey[q];
            hdr->ec[q] = s_q.ec[q];
            hdr->sigma[q] = s_q.sigma[q];
            hdr->s1[q] = 0;
        }
        hdr->err = s_q.err;
        hdr->open = open;
        hdr->cand = 0;
        hdr->wide_ticket = 0;
        hdr->fin_fail = 0;
        hdr->epoch = hdr->epoch + 1;
    }
    if (s_q.err) return;
    uint32_t lists;
    const uint32_t rows = cand_rows(open, grid, per_row, lists);
    if (blockIdx.x >= rows) return;
    Quad Q;
    uint32_t kfirst[4];  // k1 of each region's first point: the smallest of the region
    for (int q = 0; q < 4; ++q) {
        Q.ex[q] = s_q.ex[q];
        Q.ey[q] = s_q.ey[q];
        Q.ec[q] = s_q.ec[q];
        Q.sigma[q] = s_q.sigma[q];
        uint32_t k2;
        to_frame((uint32_t)q, s_q.X[q], s_q.Y[q], kfirst[q], k2);
    }
    for (int b = tid; b < kBuckets; b += kCandBlock) {
        lcnt[cpad(b)] = 0;
        lmin[b] = ~0u;
    }
    // the workgroup's lists, concatenated: their starts from the prefix over
    // all lists (thread t: list t)
    const uint32_t first = blockIdx.x * lists, nl = min(lists, grid - first);
    if (tid == first) s_base = gpre;
    __syncthreads();
    if (tid >= first && tid < first + nl) s_start[tid - first] = gpre - s_base;
    if (tid == first + nl - 1) s_start[nl] = gpre + mine - s_base;
    __syncthreads();
    const uint32_t count = s_start[nl];
    const size_t part = (size_t)first * region;
    uint32_t* const my_ka = key_a + part;
    u64* const my_va = val_a + part;
    uint32_t written = 0;  // records of the chunks before the last, in part A

    // ---- pass 1 (the last chunk's records stay in registers) ----
    uint32_t lk[kCandPer], keep = 0;  // the last chunk's kept records: q << 23 | k1, k2 << 32 | index
    u64 lv[kCandPer];
    for (uint32_t c0 = 0; c0 < count; c0 += kCandChunk) {
        uint32_t k1s[kCandPer], k2s[kCandPer], idxs[kCandPer], addrs[kCandPer];
        const bool last = c0 + kCandChunk >= count;
        for (int e = tid; e < 4 * kSlots; e += kCandBlock) smin[e] = ~0ull;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCandPer; ++k) {
            const uint32_t e = c0 + k * kCandBlock + tid;
            addrs[k] = ~0u;
            if (e < count) {
                // the list holding e: the last with start <= e
                uint32_t l = 0;
                for (uint32_t st = kStreamGrid / 2; st > 0; st >>= 1)
                    if (l + st < nl && s_start[l + st] <= e) l += st;
                const size_t at = ((size_t)first + l) * region + (e - s_start[l]);
                const u64 r = open_xym[at];
                const uint32_t ix = open_idx[at];  // (with the record, not after the test: one round trip)
                const uint32_t X = (uint32_t)r & kM, Y = (uint32_t)(r >> 23) & kM, mask = (uint32_t)(r >> 46);
                const uint32_t q = region_of(Q, X, Y);
                if (q < 4 && ((mask >> q) & 1u)) {
                    uint32_t k1, k2;
                    to_frame(q, X, Y, k1, k2);
                    k1s[k] = k1;
                    k2s[k] = k2;
                    idxs[k] = ix;
                    const uint32_t kf = q == 0 ? kfirst[0] : q == 1 ? kfirst[1] : q == 2 ? kfirst[2] : kfirst[3];
                    addrs[k] = q * kSlots + chunk_slot(k1 - kf);
                    atomicMin(&smin[addrs[k]], ((u64)k2 << 23) | k1);
                }
            }
        }
        __syncthreads();
        // Wave w < 4 scans region w's slots: sexc becomes the smallest k2
        // over earlier slots and the region's first point.
        if (wave < 4) {
            const uint32_t q = wave;
            constexpr int per = kSlots / 64;
            uint32_t v[per];
            uint32_t run = ~0u;
#pragma unroll
            for (int k = 0; k < per; ++k) {
                const u64 m = smin[q * kSlots + lane * per + k];
                v[k] = m == ~0ull ? ~0u : (uint32_t)(m >> 23);
                run = min(run, v[k]);
            }
            const uint32_t incl = wave_incl_min(run);
            uint32_t before = __shfl_up(incl, 1);
            if (lane == 0) before = ~0u;
            const uint32_t sigma = q == 0 ? Q.sigma[0] : q == 1 ? Q.sigma[1] : q == 2 ? Q.sigma[2] : Q.sigma[3];
            before = min(before, sigma);
#pragma unroll
            for (int k = 0; k < per; ++k) {
                sexc[q * kSlots + lane * per + k] = before;
                before = min(before, v[k]);
            }
        }
        __syncthreads();
        keep = 0;
#pragma unroll
        for (int k = 0; k < kCandPer; ++k) {
            if (addrs[k] != ~0u) {
                const u64 me = ((u64)k2s[k] << 23) | k1s[k];
                const u64 best = smin[addrs[k]];
                bool ok = k2s[k] < sexc[addrs[k]];
                ok = ok && !(best < me && (uint32_t)(best & kM) <= k1s[k]);
                if (ok) keep |= 1u << k;
            }
        }
        uint32_t pos = written, total = 0;
        if (!last) pos += block_excl_sum<kCandWaves>(__popc(keep), scratch, total);
#pragma unroll
        for (int k = 0; k < kCandPer; ++k) {
            if ((keep >> k) & 1u) {
                const uint32_t q = addrs[k] / kSlots;
                if (!last) {
                    my_ka[pos] = (q << 23) | k1s[k];
                    my_va[pos] = ((u64)k2s[k] << 32) | idxs[k];
                    ++pos;
                }
                const uint32_t b = (q << kBucketBits) | (k1s[k] >> kLowBits);
                atomicAdd(&lcnt[cpad(b)], 1u);
                atomicMin(&lmin[b], k2s[k]);
            }
            lk[k] = ((addrs[k] / kSlots) << 23) | k1s[k];
            lv[k] = ((u64)k2s[k] << 32) | idxs[k];
        }
        written += total;
        __syncthreads();
    }

    // ---- pass 2: the row (thread t owns buckets 8t .. 8t+7) ----
    __syncthreads();  // (the counts' set-up, when there was no chunk)
    uint32_t* const my_off = rowoff + (size_t)blockIdx.x * (kBuckets + 1);
    {
        uint32_t c[kCandBucketsPer], sum = 0;
#pragma unroll
        for (int k = 0; k < kCandBucketsPer; ++k) {
            c[k] = lcnt[cpad(tid * kCandBucketsPer + k)];
            sum += c[k];
        }
        uint32_t total;
        uint32_t run = block_excl_sum<kCandWaves>(sum, scratch, total);  // (its barriers follow every read above)
#pragma unroll
        for (int k = 0; k < kCandBucketsPer; ++k) {
            lcnt[cpad(tid * kCandBucketsPer + k)] = run;
            run += c[k];
        }
        if (tid == 0) my_off[kBuckets] = total;
    }
    __syncthreads();
    for (int b = tid; b < kBuckets; b += kCandBlock) {
        my_off[b] = lcnt[cpad(b)];
        rowmin[(size_t)blockIdx.x * kBuckets + b] = lmin[b];
    }

    // ---- pass 3: the last chunk's records from registers, the earlier
    // ones from part A, each to part B at its bucket's next position ----
    __syncthreads();  // (a workgroup-scope fence and barrier: part A's stores, before other threads read them)
    uint32_t* const my_kb = key_b + part;
    u64* const my_vb = val_b + part;
#pragma unroll
    for (int k = 0; k < kCandPer; ++k) {
        if ((keep >> k) & 1u) {
            const uint32_t b = ((lk[k] >> 23) << kBucketBits) | ((lk[k] & kM) >> kLowBits);
            const uint32_t p = atomicAdd(&lcnt[cpad(b)], 1u);
            my_kb[p] = lk[k];
            my_vb[p] = lv[k];
        }
    }
    for (uint32_t i0 = 0; i0 < written; i0 += 4 * kCandBlock) {
        uint32_t kk[4];
        u64 vv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = i0 + u * kCandBlock + tid;
            kk[u] = i < written ? my_ka[i] : ~0u;
            vv[u] = i < written ? my_va[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (kk[u] == ~0u) continue;
            const uint32_t b = ((kk[u] >> 23) << kBucketBits) | ((kk[u] & kM) >> kLowBits);
            const uint32_t p = atomicAdd(&lcnt[cpad(b)], 1u);
            my_kb[p] = kk[u];
            my_vb[p] = vv[u];
        }
    }
}

// Round-1 survivor counts per region (Section 2.1.1), for chainhull_polygon:
// the exact region test on every point.
__global__ __launch_bounds__(kBlock) void k_count_regions(const float* __restrict__ pts, uint32_t n,
                                                          DevHeader* __restrict__ hdr)
{
    __shared__ uint32_t wc[kWaves][4];
    if (hdr->err) return;
    Quad Q;
    for (int q = 0; q < 4; ++q) {
        Q.ex[q] = hdr->ex[q];
        Q.ey[q] = hdr->ey[q];
        Q.ec[q] = hdr->ec[q];
    }
    uint32_t c[4] = {0, 0, 0, 0};
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const v2f p = *reinterpret_cast<const v2f*>(pts + 2 * (size_t)i);
        const uint32_t q = region_of(Q, (uint32_t)p.x, (uint32_t)p.y);
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] += q == (uint32_t)r;
    }
    const uint32_t wave = threadIdx.x / 64;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        c[r] = wave_sum(c[r]);
        if (lane_id() == 0) wc[wave][r] = c[r];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        uint32_t tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += wc[w][threadIdx.x];
        if (tot) atomicAdd(&hdr->s1[threadIdx.x], tot);
    }
}
// ---------------------------------------------------------------------------
// Steps 3-6 (Section 2.1; Table 1; Figure 2): the region sort, SPA and the
// chain order, as a two-level sort fused with SPA.
//
// Level 1: the records are grouped by bucket, the region code and the top
// kBucketBits bits of k1 (a counting sort): k_cand sorts each workgroup's
// records by bucket in its own part of the record arrays and writes its
// row of the bucket table (first position per bucket, smallest k2 per
// bucket); k_scan sums the rows per bucket (bucket sizes, where each
// bucket's records start in the concatenated order) and takes, per region,
// the exclusive prefix minimum of the buckets' smallest k2 seeded with the
// region's first point (the threshold entering each bucket).  Buckets in
// ascending order list the regions in Table 1's order and each region by
// ascending k1.
//
// Level 2 (k_bucket_spa): a bucket's records are gathered from the rows'
// parts; inside a bucket the low kLowBits bits of k1 address an LDS table
// directly, and a 64-bit atomic minimum of (k2 << 32 | index) per entry
// leaves each group of equal k1 with its smallest (k2, index): the order
// Table 1 asks for, restricted to what SPA can keep.  SPA keeps a record iff
// its k2 is below the k2 of every earlier record of its region and of the
// region's first point (Figure 2's threshold t is exactly that running
// minimum, since a discarded record never lowers it); within an equal-k1
// group only the group's smallest (k2, index) can qualify.  The running
// minimum entering a bucket is the threshold above; inside the bucket it is
// an exclusive prefix minimum over the table.  Survivors are written, in k1
// order, as (index, x, y) at the bucket's first record position of the
// chain buffer; their number per bucket goes to bk.surv.
// ---------------------------------------------------------------------------

// k_scan: workgroup j owns buckets [64j, 64j+64) (within one region, since
// a region has 2048 buckets); wave w sums rows w, w+4, ... of them, one
// bucket per lane.  Per bucket: its size and smallest k2 over the rows;
// then, inside the workgroup, the exclusive prefix sum of the sizes
// (lstart) and exclusive prefix minimum of the smallest k2 (lthr), and the
// workgroup's totals (wtot, wmin).  k_bucket_spa combines the totals of the
// earlier workgroups itself: a bucket's first record is lstart plus the
// records of the earlier workgroups, its threshold the minimum of lthr, the
// earlier workgroups' of its region and the region's first point.
constexpr int kScanBuckets = 64;                    // buckets per k_scan workgroup
constexpr int kScanGrid = kBuckets / kScanBuckets;  // 128
constexpr int kScanPerRegion = kScanGrid / 4;       // 32
static_assert(kScanGrid == 2 * 64, "k_bucket_spa's combine: two workgroup totals per lane");

__global__ __launch_bounds__(kBlock) void k_scan(DevHeader* __restrict__ hdr, const uint32_t* __restrict__ rowoff,
                                                 const uint32_t* __restrict__ rowmin, uint32_t grid,
                                                 uint32_t per_row, Buckets bk, const int32_t* __restrict__ gate)
{
    __shared__ uint32_t s_c[kWaves][64], s_m[kWaves][64];
    const uint32_t tid = threadIdx.x, wave = tid / 64, lane = lane_id();
    if (gated_off(gate) || hdr->err) return;
    uint32_t lists;
    const uint32_t rows = cand_rows(hdr->open, grid, per_row, lists);
    const uint32_t b = blockIdx.x * kScanBuckets + lane;
    uint32_t c = 0, m = ~0u;
    constexpr int kBatch = 8;  // rows loaded together per wave
    for (uint32_t r0 = wave; r0 < rows; r0 += kWaves * kBatch) {
        uint32_t lo[kBatch], hi[kBatch], mn[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const uint32_t r = min(r0 + k * kWaves, rows - 1);
            lo[k] = rowoff[(size_t)r * (kBuckets + 1) + b];
            hi[k] = rowoff[(size_t)r * (kBuckets + 1) + b + 1];
            mn[k] = rowmin[(size_t)r * kBuckets + b];
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            if (r0 + k * kWaves < rows) {
                c += hi[k] - lo[k];
                m = min(m, mn[k]);
            }
        }
    }
    s_c[wave][lane] = c;
    s_m[wave][lane] = m;
    __syncthreads();
    if (wave == 0) {
        c = 0;
        m = ~0u;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            c += s_c[w][lane];
            m = min(m, s_m[w][lane]);
        }
        bk.cnt[b] = c;
        bk.bmin[b] = m;
        const uint32_t incl = wave_incl_sum(c);
        bk.lstart[b] = incl - c;
        const uint32_t mincl = wave_incl_min(m);
        uint32_t mexcl = __shfl_up(mincl, 1);
        if (lane == 0) mexcl = ~0u;
        bk.lthr[b] = mexcl;
        const uint32_t tot = __shfl(incl, 63), mtot = __shfl(mincl, 63);
        if (lane == 0) {
            bk.wtot[blockIdx.x] = tot;
            bk.wmin[blockIdx.x] = mtot;
        }
    }
}

// Workgroup g takes buckets 4g .. 4g+3, wave w bucket 4g + w.  A bucket
// whose smallest k2 is not below the threshold entering it keeps nothing.
// Otherwise its records are gathered from the rows' parts (row r: part B of
// k_cand workgroup r, positions [rowoff[r][b], rowoff[r][b+1]); each lane
// holds up to four rows).  A bucket of at most kWaveBucket records is
// sorted and filtered by its wave alone (wave_spa); larger ones use the
// table, the whole workgroup on one bucket at a time.  Survivors go, as
// (index, x, y), to dev_chain at the bucket's first record position (also
// written to bk.off); their number to bk.surv.
constexpr int kSpaHalves = 1;                      // tables per large bucket (parts of its k1 range)
constexpr int kSpaTab = kLowSize / kSpaHalves;     // 4096 entries
constexpr int kPerThreadTab = kSpaTab / kBlock;    // 16
constexpr int kBucketsPerSpa = kWaves;
constexpr uint32_t kWaveBucket = 512;  // records of a bucket one wave sorts (eight per lane)

__device__ inline PolyRec chain_rec(uint32_t q, uint32_t k1, uint32_t k2, uint32_t idx)
{
    // invert the frame: x = (k1, M-k2, M-k1, k2), y = (k2, k1, M-k2, M-k1)
    const uint32_t a = (q & 1u) ? k2 : k1;
    const uint32_t b = (q & 1u) ? k1 : k2;
    const uint32_t X = ((q ^ (q >> 1)) & 1u) ? a ^ kM : a;
    const uint32_t Y = (q & 2u) ? b ^ kM : b;
    return PolyRec{(int32_t)idx, (int32_t)X, (int32_t)Y};
}

// Sorts the 64*PER (key, index) pairs that one wave holds, element
// e = lane*PER + s, ascending by key, then index: a bitonic network, with
// shuffles across lanes (partner distance j >= PER) and register swaps inside
// a lane (j < PER).
template <int PER>
__device__ inline void bitonic_in_lane(u64 (&key)[PER], uint32_t (&ix)[PER], uint32_t lane, uint32_t k)
{
#pragma unroll
    for (int j = PER / 2; j > 0; j >>= 1) {
        if ((uint32_t)j >= k) continue;
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            const int t = s ^ j;
            if (t <= s) continue;
            const uint32_t e = lane * PER + s;
            const bool t_less = key[t] < key[s] || (key[t] == key[s] && ix[t] < ix[s]);
            const bool s_less = key[s] < key[t] || (key[s] == key[t] && ix[s] < ix[t]);
            if ((e & k) == 0 ? t_less : s_less) {
                const u64 tk = key[s];
                key[s] = key[t];
                key[t] = tk;
                const uint32_t ti = ix[s];
                ix[s] = ix[t];
                ix[t] = ti;
            }
        }
    }
}

template <int PER>
__device__ inline void wave_bitonic(u64 (&key)[PER], uint32_t (&ix)[PER])
{
    const uint32_t lane = lane_id();
    for (uint32_t k = 2; k <= 64u * PER; k <<= 1) {
        for (uint32_t j = k >> 1; j >= (uint32_t)PER; j >>= 1) {
            // partner e ^ j: lane ^ (j / PER), same register
            const int d = (int)(j / PER);
#pragma unroll
            for (int s = 0; s < PER; ++s) {
                const uint32_t e = lane * PER + s;
                const u64 pk = __shfl_xor(key[s], d);
                const uint32_t pi = __shfl_xor(ix[s], d);
                const bool less = key[s] < pk || (key[s] == pk && ix[s] < pi);
                // an ascending pair's lower element keeps the smaller pair,
                // its upper one the larger; descending the reverse
                if (less != (((e & k) == 0) == ((e & j) == 0))) {
                    key[s] = pk;
                    ix[s] = pi;
                }
            }
        }
        bitonic_in_lane<PER>(key, ix, lane, k);
    }
}

// Sorts keys[0 .. n) (distinct, n <= 64*PER) ascending in one wave.
template <int PER>
__device__ inline void wave_sort_keys(u64* keys, uint32_t n)
{
    const uint32_t lane = lane_id();
    u64 k[PER];
    uint32_t ix[PER];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const uint32_t e = lane * PER + s;
        k[s] = e < n ? keys[e] : ~0ull;
        ix[s] = 0;
    }
    wave_bitonic<PER>(k, ix);
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const uint32_t e = lane * PER + s;
        if (e < n) keys[e] = k[s];
    }
}

// SPA of one bucket of m <= 64*PER records by one wave: the records,
// gathered from the rows' parts (seg, pre: the bucket's first position in
// each row's part and the records before each row), sorted by (k1, k2,
// index); a record is kept iff its k2 is below the threshold entering the
// bucket and below every earlier record's k2 (so of a run of equal (k1, k2)
// at most the first, the smallest index).  Survivors go, in order, to
// dev_chain at off; their number to surv[b].
template <int PER>
__device__ inline void wave_spa(uint32_t m, uint32_t b, uint32_t off, uint32_t thr,
                                const uint32_t* __restrict__ key, const u64* __restrict__ val, size_t part,
                                const uint32_t* seg, const uint32_t* pre, uint32_t rows,
                                PolyRec* __restrict__ dev_chain, uint32_t* __restrict__ surv)
{
    const uint32_t lane = lane_id();
    u64 kk[PER];  // k1 << 23 | k2
    uint32_t ix[PER];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const uint32_t i = lane * PER + s;
        kk[s] = ~0ull;
        ix[s] = ~0u;
        if (i < m) {
            // the row holding record i: the last with pre <= i
            uint32_t r = 0;
            for (uint32_t st = kCandMaxRows / 2; st > 0; st >>= 1)
                if (r + st < rows && pre[r + st] <= i) r += st;
            const size_t at = (size_t)r * part + seg[r] + (i - pre[r]);
            const u64 v = val[at];
            kk[s] = ((u64)(key[at] & kM) << 23) | (v >> 32);
            ix[s] = (uint32_t)v;
        }
    }
    wave_bitonic<PER>(kk, ix);
    uint32_t low = ~0u;
#pragma unroll
    for (int s = 0; s < PER; ++s) low = min(low, kk[s] != ~0ull ? (uint32_t)kk[s] & kM : ~0u);
    const uint32_t incl = wave_incl_min(low);
    uint32_t run = __shfl_up(incl, 1);
    if (lane == 0) run = ~0u;
    run = min(run, thr);
    uint32_t keep = 0;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const uint32_t k2 = (uint32_t)kk[s] & kM;
        if (kk[s] != ~0ull && k2 < run) keep |= 1u << s;
        if (kk[s] != ~0ull) run = min(run, k2);
    }
    const uint32_t cnt = (uint32_t)__popc(keep);
    const uint32_t sum = wave_incl_sum(cnt);
    uint32_t pos = off + sum - cnt;
    const uint32_t q = b >> kBucketBits;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        if ((keep >> s) & 1u) dev_chain[pos++] = chain_rec(q, (uint32_t)(kk[s] >> 23), (uint32_t)kk[s] & kM, ix[s]);
    }
    if (lane == 63) surv[b] = sum;
}

__global__ __launch_bounds__(kBlock) void k_bucket_spa(const uint32_t* __restrict__ key,
                                                       const u64* __restrict__ val, uint32_t region, uint32_t grid,
                                                       uint32_t per_row, const uint32_t* __restrict__ rowoff,
                                                       DevHeader* __restrict__ hdr, Buckets bk,
                                                       PolyRec* __restrict__ dev_chain, const int32_t* __restrict__ gate)
{
    constexpr int kRowsPerLane = kCandMaxRows / 64;
    __shared__ u64 tab[kSpaTab];
    __shared__ uint32_t scratch[kWaves];
    __shared__ uint32_t s_m[kBucketsPerSpa], s_off[kBucketsPerSpa], s_thr[kBucketsPerSpa];
    // per bucket and row: first position in the row's part, records before the row
    __shared__ uint32_t s_seg[kBucketsPerSpa][kCandMaxRows], s_pre[kBucketsPerSpa][kCandMaxRows];
    const uint32_t tid = threadIdx.x, wave = tid / 64, lane = lane_id();
    if (gated_off(gate) || hdr->err) return;
    uint32_t lists;
    const uint32_t rows = cand_rows(hdr->open, grid, per_row, lists);
    const size_t part = (size_t)lists * region;  // records in one row's part
    // the row holding record i of bucket kb: the last row with pre <= i
    auto row_of = [&](uint32_t kb, uint32_t i) {
        uint32_t r = 0;
        for (uint32_t st = kCandMaxRows / 2; st > 0; st >>= 1)
            if (r + st < rows && s_pre[kb][r + st] <= i) r += st;
        return r;
    };
    {
        // wave w: bucket 4g + w: where it starts, its threshold, its
        // segments (rows lane, lane + 64, ...; loaded with the rest, before
        // the bucket is known to be live).  A bucket whose smallest k2 is not
        // below the threshold entering it keeps nothing (every record is
        // dominated by an earlier bucket's record or the region's first
        // point).
        const uint32_t b = blockIdx.x * kBucketsPerSpa + wave;
        // k_scan workgroup g holds the bucket; lane l combines the totals of
        // workgroups l and l + 64: the records before g, the smallest k2 over
        // the earlier workgroups of the region (q*32 .. g-1)
        const uint32_t g = b / kScanBuckets, q = b >> kBucketBits;
        const uint32_t t0 = bk.wtot[lane], t1 = bk.wtot[lane + 64];
        const uint32_t m0 = bk.wmin[lane], m1 = bk.wmin[lane + 64];
        const uint32_t ls = bk.lstart[b], lt = bk.lthr[b], bm = bk.bmin[b];
        const uint32_t sigma = hdr->sigma[q];
        uint32_t lo[kRowsPerLane], n[kRowsPerLane];
#pragma unroll
        for (int k = 0; k < kRowsPerLane; ++k) {
            const uint32_t r = lane + 64 * k;
            lo[k] = 0;
            n[k] = 0;
            if (r < rows) {
                lo[k] = rowoff[(size_t)r * (kBuckets + 1) + b];
                n[k] = rowoff[(size_t)r * (kBuckets + 1) + b + 1] - lo[k];
            }
        }
        const uint32_t first = q * kScanPerRegion;
        uint32_t before = (lane < g ? t0 : 0u) + (lane + 64 < g ? t1 : 0u);
        uint32_t mprev = min((lane >= first && lane < g) ? m0 : ~0u, (lane + 64 >= first && lane + 64 < g) ? m1 : ~0u);
        before = wave_sum(before);
        mprev = wave_min(mprev);
        if (blockIdx.x == 0 && wave == 0) {
            const uint32_t all = wave_sum(t0 + t1);
            if (lane == 0) hdr->cand = all;
        }
        const uint32_t off = ls + before;
        const uint32_t thr = min(min(lt, mprev), sigma);
        const bool live = bm < thr;
        uint32_t m = 0;
        if (live) {
#pragma unroll
            for (int k = 0; k < kRowsPerLane; ++k) {
                const uint32_t incl = wave_incl_sum(n[k]);
                s_seg[wave][lane + 64 * k] = lo[k];
                s_pre[wave][lane + 64 * k] = m + incl - n[k];
                m += __shfl(incl, 63);
            }
        }
        if (lane == 0) {
            s_m[wave] = m;
            s_off[wave] = off;
            s_thr[wave] = thr;
            bk.off[b] = off;
            if (!live) bk.surv[b] = 0;
        }
        __builtin_amdgcn_wave_barrier();
        if (live && m <= kWaveBucket) {
            const uint32_t* seg = s_seg[wave];
            const uint32_t* pre = s_pre[wave];
            if (m <= 64) wave_spa<1>(m, b, off, thr, key, val, part, seg, pre, rows, dev_chain, bk.surv);
            else if (m <= 128) wave_spa<2>(m, b, off, thr, key, val, part, seg, pre, rows, dev_chain, bk.surv);
            else if (m <= 256) wave_spa<4>(m, b, off, thr, key, val, part, seg, pre, rows, dev_chain, bk.surv);
            else wave_spa<8>(m, b, off, thr, key, val, part, seg, pre, rows, dev_chain, bk.surv);
        }
    }
    __syncthreads();
    for (int kb = 0; kb < kBucketsPerSpa; ++kb) {
        const uint32_t b = blockIdx.x * kBucketsPerSpa + kb, m = s_m[kb];
        if (m <= kWaveBucket) continue;
        const uint32_t off = s_off[kb];
        // the bucket's k1 range in kSpaHalves parts, one table each; the
        // running minimum and the output position carry over
        uint32_t run_in = s_thr[kb], pos_base = off;
        const uint32_t q = b >> kBucketBits;
        const uint32_t k1base = (b & ((1u << kBucketBits) - 1)) << kLowBits;
        for (uint32_t h = 0; h < (uint32_t)kSpaHalves; ++h) {
            for (int e = tid; e < kSpaTab; e += kBlock) tab[e] = ~0ull;
            __syncthreads();
            constexpr int kBatch = 8;  // records loaded together per thread
            for (uint32_t i0 = 0; i0 < m; i0 += kBatch * kBlock) {
                uint32_t k1[kBatch];
                u64 v[kBatch];  // k2 << 32 | index
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const uint32_t i = i0 + u * kBlock + tid;
                    k1[u] = 0u;
                    v[u] = ~0ull;
                    if (i < m) {
                        const uint32_t r = row_of(kb, i);
                        const size_t at = (size_t)r * part + s_seg[kb][r] + (i - s_pre[kb][r]);
                        k1[u] = key[at];
                        v[u] = val[at];
                    }
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const uint32_t low = k1[u] & (kLowSize - 1);
                    if (v[u] != ~0ull && low / kSpaTab == h) atomicMin(&tab[low % kSpaTab], v[u]);
                }
            }
            __syncthreads();
            // exclusive prefix minimum of k2 over the table, seeded with the
            // running minimum entering it; survivors in table order
            u64 e[kPerThreadTab];
            uint32_t lo = ~0u;
#pragma unroll
            for (int k = 0; k < kPerThreadTab; ++k) {
                e[k] = tab[tid * kPerThreadTab + k];
                lo = min(lo, (uint32_t)(e[k] >> 32));
            }
            uint32_t tmin;
            uint32_t run = min(run_in, block_excl_min(lo, scratch, tmin));
            uint32_t keep = 0;
#pragma unroll
            for (int k = 0; k < kPerThreadTab; ++k) {
                const uint32_t k2 = (uint32_t)(e[k] >> 32);
                if (e[k] != ~0ull && k2 < run) keep |= 1u << k;
                run = min(run, k2);
            }
            uint32_t total;
            uint32_t pos = pos_base + block_excl_sum(__popc(keep), scratch, total);
#pragma unroll
            for (int k = 0; k < kPerThreadTab; ++k) {
                if ((keep >> k) & 1u)
                    dev_chain[pos++] = chain_rec(q, k1base + h * kSpaTab + tid * kPerThreadTab + k,
                                                 (uint32_t)(e[k] >> 32), (uint32_t)e[k]);
            }
            pos_base += total;
            run_in = min(run_in, tmin);
            __syncthreads();
        }
        if (tid == 0) bk.surv[b] = pos_base - off;
    }
}

// ---------------------------------------------------------------------------
// Step 6 (Section 2.1; Section 2.2.2): the chains concatenated in bucket
// order, cut into segments of kSeg points, each shortened by a pre-hull and
// written to pinned host memory.
//
// Pre-hull: a chain point that makes no left turn, in its region's frame,
// with two other points of its region around it (in chain order) lies on or
// above the segment joining them, so its support value never strictly
// exceeds theirs for any outward direction of that corner: it is not a
// strict hull vertex.  All such points (with their current neighbours) go
// at once, round after round, until the segment's chains are convex.  Only
// non-vertices go, so the hull of the polygon the finish scans is
// unchanged; the frames are rotations, so turns keep their sign.
//
// Segment s keeps its points at [s*kSeg, ...) of the device copy (and, when
// host_chain is given, of the host chain buffer) and writes how many of
// each region it kept to dev_segcnt[4s .. 4s+3] (and segcnt).  Workgroup
// 0 also publishes the SPA survivor counts per region.
// ---------------------------------------------------------------------------
constexpr int kSeg = 1024;
constexpr int kPerThreadSeg = kSeg / kBlock;  // 4
constexpr int kPrehullRounds = 16;

// Frame cross product (o, a, b): > 0 for a left turn.
__device__ inline i64 frame_turn(uint32_t o1, uint32_t o2, uint32_t a1, uint32_t a2, uint32_t b1, uint32_t b2)
{
    return (i64)((int32_t)a1 - (int32_t)o1) * (i64)((int32_t)b2 - (int32_t)o2) -
           (i64)((int32_t)a2 - (int32_t)o2) * (i64)((int32_t)b1 - (int32_t)o1);
}

__global__ __launch_bounds__(kBlock) void k_chain(const PolyRec* __restrict__ dev_chain,
                                                  DevHeader* __restrict__ hdr, Buckets bk,
                                                  PolyRec* __restrict__ host_chain, uint32_t host_cap,
                                                  PolyRec* __restrict__ spill, uint32_t* __restrict__ segcnt,
                                                  DevHeader* __restrict__ host_hdr, int prehull,
                                                  PolyRec* __restrict__ dev_kept, uint32_t* __restrict__ dev_segcnt,
                                                  const int32_t* __restrict__ gate)
{
    __shared__ uint32_t pre[kBucketsPadded];  // chain points before each bucket (at bpad)
    __shared__ uint32_t ka[kSeg], kb[kSeg];
    __shared__ int32_t sidx[kSeg];  // the points' indices (the output needs no second read of the chain)
    __shared__ uint16_t lst[kSeg];
    __shared__ uint8_t reg[kSeg], alive[kSeg];
    __shared__ uint32_t scratch[kWaves];
    __shared__ uint32_t s_removed[2], s_cnt[4];
    const uint32_t tid = threadIdx.x;
    if (gated_off(gate)) return;
    // the header, for the host, once every field is final
    auto publish_header = [&]() {
        if (blockIdx.x != 0) return;
        __syncthreads();
        const uint32_t* src = reinterpret_cast<const uint32_t*>(hdr);
        uint32_t* dst = reinterpret_cast<uint32_t*>(host_hdr);
        for (uint32_t e = tid; e < sizeof(DevHeader) / 4; e += kBlock) dst[e] = src[e];
    };
    if (hdr->err) {
        publish_header();
        return;
    }
    // the chain is at most the sort records long: workgroups past its last
    // segment have nothing to do (workgroup 0 still publishes the header)
    if (blockIdx.x > 0 && blockIdx.x >= (hdr->cand + kSeg - 1) / kSeg) return;

    uint32_t total;
    {
        {
            uint32_t v[kPerThreadBuckets];  // staged, all loads in flight together
#pragma unroll
            for (int k = 0; k < kPerThreadBuckets; ++k) v[k] = bk.surv[k * kBlock + tid];
#pragma unroll
            for (int k = 0; k < kPerThreadBuckets; ++k) pre[bpad(k * kBlock + tid)] = v[k];
        }
        __syncthreads();
        uint32_t c[kPerThreadBuckets], sum = 0;
#pragma unroll
        for (int k = 0; k < kPerThreadBuckets; ++k) {
            c[k] = pre[bpad(tid * kPerThreadBuckets + k)];
            sum += c[k];
        }
        uint32_t run = block_excl_sum(sum, scratch, total);  // (its barriers follow every read above)
#pragma unroll
        for (int k = 0; k < kPerThreadBuckets; ++k) {
            pre[bpad(tid * kPerThreadBuckets + k)] = run;
            run += c[k];
        }
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < 4) {
        const uint32_t first = pre[bpad(tid << kBucketBits)];
        const uint32_t last = tid == 3 ? total : pre[bpad((tid + 1) << kBucketBits)];
        hdr->s2[tid] = last - first;
        if (tid == 0) hdr->chain = total;
    }
    const uint32_t nseg = (total + kSeg - 1) / kSeg;
    for (uint32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const uint32_t base = sg * kSeg, len = min((uint32_t)kSeg, total - base);
        // every point: its bucket (the last with pre <= position: its range
        // holds the position), region, place in dev_chain, frame coordinates;
        // all loads of a kind issued together
        uint32_t bb[kPerThreadSeg], aa[kPerThreadSeg];
        const int kmax = (int)((len + kBlock - 1) / kBlock);  // rounds that hold points
#pragma unroll
        for (int k = 0; k < kPerThreadSeg; ++k) {
            bb[k] = 0;
            if (k >= kmax) continue;
            const uint32_t i = k * kBlock + tid, g = base + min(i, len - 1);
            uint32_t lo = 0, hi = kBuckets - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) / 2;
                if (pre[bpad(mid)] <= g) lo = mid;
                else hi = mid - 1;
            }
            bb[k] = lo;
        }
#pragma unroll
        for (int k = 0; k < kPerThreadSeg; ++k) aa[k] = k < kmax ? bk.off[bb[k]] : 0u;
        PolyRec rr[kPerThreadSeg];
#pragma unroll
        for (int k = 0; k < kPerThreadSeg; ++k) {
            if (k >= kmax) continue;
            const uint32_t i = k * kBlock + tid, g = base + min(i, len - 1);
            aa[k] += g - pre[bpad(bb[k])];
            rr[k] = dev_chain[aa[k]];
        }
#pragma unroll
        for (int k = 0; k < kPerThreadSeg; ++k) {
            const uint32_t i = k * kBlock + tid;
            if (k < kmax && i < len) {
                const uint32_t q = bb[k] >> kBucketBits;
                uint32_t k1, k2;
                to_frame(q, (uint32_t)rr[k].x, (uint32_t)rr[k].y, k1, k2);
                sidx[i] = rr[k].idx;
                reg[i] = (uint8_t)q;
                ka[i] = k1;
                kb[i] = k2;
                alive[i] = 1;
            }
        }
        if (tid < 4) s_cnt[tid] = 0;
        __syncthreads();
        // alive points in order: thread t owns positions [4t, 4t+4)
        auto compact = [&]() -> uint32_t {
            uint32_t mine = 0;
#pragma unroll
            for (int k = 0; k < kPerThreadSeg; ++k) {
                const uint32_t i = tid * kPerThreadSeg + k;
                mine += (i < len && alive[i]) ? 1u : 0u;
            }
            uint32_t n_alive;
            uint32_t o = block_excl_sum(mine, scratch, n_alive);
#pragma unroll
            for (int k = 0; k < kPerThreadSeg; ++k) {
                const uint32_t i = tid * kPerThreadSeg + k;
                if (i < len && alive[i]) lst[o++] = (uint16_t)i;
            }
            __syncthreads();
            return n_alive;
        };
        // Pre-hull rounds: every alive point that makes no left turn with
        // its alive neighbours of the same region goes at once; repeat
        // until none does (at most kPrehullRounds times).  First inside
        // each wave's window of 256 positions (lane l: 4l .. 4l+3; the
        // alive flags stay in registers, the neighbours come from wave
        // scans, no workgroup barrier), then over the whole segment.
        if (prehull) {
            // in registers: lane l holds positions 4l .. 4l+3 (k1; region << 23
            // | k2); a lane's neighbours outside it are the last alive point
            // of the nearest lane before with one and the first of the
            // nearest lane after (lane scans, then one shuffle per value)
            const uint32_t p0 = tid * kPerThreadSeg;
            const int lane = (int)lane_id();
            bool al[kPerThreadSeg];
            uint32_t c1[kPerThreadSeg], c2[kPerThreadSeg];
#pragma unroll
            for (int k = 0; k < kPerThreadSeg; ++k) {
                const uint32_t i = p0 + k;
                al[k] = i < len;
                c1[k] = al[k] ? ka[i] : 0u;
                c2[k] = al[k] ? (((uint32_t)reg[i] << 23) | kb[i]) : 0u;
            }
            for (int round = 0; round < kPrehullRounds; ++round) {
                uint32_t f1 = 0, f2 = 0, l1 = 0, l2 = 0;  // the lane's first and last alive point
                bool has = false;
#pragma unroll
                for (int k = kPerThreadSeg - 1; k >= 0; --k) {
                    if (al[k]) {
                        f1 = c1[k];
                        f2 = c2[k];
                    }
                }
#pragma unroll
                for (int k = 0; k < kPerThreadSeg; ++k) {
                    if (al[k]) {
                        l1 = c1[k];
                        l2 = c2[k];
                        has = true;
                    }
                }
                int before = has ? lane : -1, after = has ? lane : 64;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const int bv = __shfl_up(before, off), av = __shfl_down(after, off);
                    if (lane >= off) before = max(before, bv);
                    if (lane + off < 64) after = min(after, av);
                }
                int pl = __shfl_up(before, 1), nl = __shfl_down(after, 1);
                if (lane == 0) pl = -1;
                if (lane == 63) nl = 64;
                const uint32_t q1 = (uint32_t)__shfl(l1, max(pl, 0)), q2 = (uint32_t)__shfl(l2, max(pl, 0));
                const uint32_t n1 = (uint32_t)__shfl(f1, min(nl, 63)), n2 = (uint32_t)__shfl(f2, min(nl, 63));
                // walk the lane: the previous alive point so far, then the
                // next one from the lane's end
                bool hp = pl >= 0;
                uint32_t a1 = q1, a2 = q2;
                bool hpv[kPerThreadSeg];
                uint32_t pv1[kPerThreadSeg], pv2[kPerThreadSeg];
#pragma unroll
                for (int k = 0; k < kPerThreadSeg; ++k) {
                    hpv[k] = hp;
                    pv1[k] = a1;
                    pv2[k] = a2;
                    if (al[k]) {
                        hp = true;
                        a1 = c1[k];
                        a2 = c2[k];
                    }
                }
                bool hn = nl < 64;
                uint32_t b1 = n1, b2 = n2;
                bool any = false;
                bool gone[kPerThreadSeg];
#pragma unroll
                for (int k = kPerThreadSeg - 1; k >= 0; --k) {
                    gone[k] = false;
                    if (al[k] && hpv[k] && hn && (pv2[k] >> 23) == (c2[k] >> 23) && (b2 >> 23) == (c2[k] >> 23) &&
                        frame_turn(pv1[k], pv2[k] & kM, c1[k], c2[k] & kM, b1, b2 & kM) <= 0) {
                        gone[k] = true;
                        any = true;
                    }
                    if (al[k]) {
                        hn = true;
                        b1 = c1[k];
                        b2 = c2[k];
                    }
                }
#pragma unroll
                for (int k = 0; k < kPerThreadSeg; ++k) al[k] = al[k] && !gone[k];
                if (!__ballot(any)) break;
            }
#pragma unroll
            for (int k = 0; k < kPerThreadSeg; ++k)
                if (p0 + k < len) alive[p0 + k] = al[k] ? 1 : 0;
        }
        if (tid < 2) s_removed[tid] = 0;
        uint32_t n_alive = compact();
        for (int round = 0; prehull && round < kPrehullRounds; ++round) {
            if (tid == 0) s_removed[(round + 1) & 1] = 0;  // the flag of the next round
            bool removed = false;
            for (uint32_t p = tid + 1; p + 1 < n_alive; p += kBlock) {
                const uint32_t a = lst[p - 1], i = lst[p], c = lst[p + 1];
                if (reg[a] == reg[i] && reg[c] == reg[i] &&
                    frame_turn(ka[a], kb[a], ka[i], kb[i], ka[c], kb[c]) <= 0) {
                    alive[i] = 0;
                    removed = true;
                }
            }
            if (removed) s_removed[round & 1] = 1;
            __syncthreads();
            const bool any = s_removed[round & 1] != 0;
            n_alive = compact();
            if (!any) break;
        }
        // the kept points, in order, at base + rank
        for (uint32_t p = tid; p < n_alive; p += kBlock) {
            const uint32_t i = lst[p];
            const PolyRec r = chain_rec(reg[i], ka[i], kb[i], (uint32_t)sidx[i]);
            const uint32_t o = base + p;
            if (host_chain) {  // (the host polygon of chainhull_polygon)
                if (o < host_cap) host_chain[o] = r;
                else spill[o - host_cap] = r;
            }
            dev_kept[o] = r;  // k_finish_wide and k_gather read these
            atomicAdd(&s_cnt[reg[i]], 1u);
        }
        __syncthreads();
        if (tid < 4) {
            if (segcnt) segcnt[4 * sg + tid] = s_cnt[tid];
            dev_segcnt[4 * sg + tid] = s_cnt[tid];
        }
        __syncthreads();
    }
    publish_header();
}

// ---------------------------------------------------------------------------
// Batched hulls: the method on many independent point sets in one launch,
// one workgroup of kBatchBlock threads per set (larger sets first), every
// step inside the workgroup, the finish included.
//
//   stream   one read of the set: the domain check and the four-frame
//            staircase test of k_stream, against a staircase that tightens
//            itself.  It starts from a sample (kBatchChunks runs of
//            kBatchChunk consecutive points) and every listed point lowers
//            the slot minima it falls in.  Listed ("open") point indices go
//            to an LDS list.  When the next round could overflow the list,
//            the staircase is rebuilt from the slot minima and the list is
//            tested against it again; a point that fails is dominated in
//            every frame by a point of the set, as in k_stream.  The extreme
//            points are found among the listed points (they are always
//            open).
//   regions  the exact region test on the listed points; per region and
//            slot the smallest (k2, k1).  A record goes when the region's
//            first point or a record of an earlier slot has k2 <= its k2,
//            or when its slot's smallest point precedes it with k1 <= its
//            k1 (the dominance argument of Figure 3).
//   sort     bitonic, in LDS, by (region, k1, k2, list position).
//   SPA      a tagged exclusive prefix minimum (Figure 2's running
//            threshold); the run of exact duplicates reports its smallest
//            index.
//   polygon  [P_minx, R1, P_miny, R2, P_maxx, R3, P_maxy, R4] in LDS.  After
//            the SPA every region chain is monotone in both frame keys, so
//            the polygon is monotone in x above and below: simple.
//   pre-hull rounds: a chain vertex whose turn with its current neighbours
//            (chain points of its region or the region's two extreme
//            points) is not a left turn lies between the chord of those
//            neighbours and the quadrilateral edge, inside the convex hull
//            of four points of the set, so it goes; all such vertices go
//            together.  When a round removes nothing and every vertex,
//            extreme points included, is a strict left turn, the simple
//            polygon is convex: it is the hull, written out in parallel from
//            P_miny (the lowest, then leftmost, point).  Otherwise one
//            thread finishes with Melkman (Section 2.1.3).
// A set whose list, sort records or chain exceed the LDS capacities gets
// kBatchRedo in out_counts and is run by the single-hull path afterwards, as
// are sets larger than kBatchMaxSet (one workgroup would stream them for a
// long time while the rest of the device idles).
// ---------------------------------------------------------------------------
constexpr int kBatchBlock = 512;                                   // two workgroups per CU
constexpr int kBatchWaves = kBatchBlock / 64;
constexpr int kBatchWavesPerSimd = 4;                              // 128 VGPRs: two workgroups fit
constexpr int kBatchUnrollMax = 2;                                 // float4 loads per thread and round, at most
constexpr uint32_t kBatchRoundMax = 2u * kBatchUnrollMax * kBatchBlock;  // points per round, at most
constexpr int kBatchList = 8192;                                   // listed points per set
constexpr int kBatchPerList = kBatchList / kBatchBlock;
constexpr int kBatchCand = 4096;                                   // sort records per set
constexpr int kBatchPolyMax = 3584;                                // polygon vertices per set
constexpr int kBatchSlots = 512;                                   // k1 slots per region (exact filter)
constexpr int kBatchSlotShift = 23 - 9;                            // log2(kBatchSlots) = 9
constexpr int kBatchPosBits = 14;                                  // list position in a sort key
static_assert(kBatchSlots == 1 << (23 - kBatchSlotShift) && kBatchList <= 1 << kBatchPosBits, "slots");

// The list mode's filter slot of a record: d = k1 minus the k1 of its
// region's first point (the region's smallest); exact below 16, then 16
// slots per power of two up to 2^19 (a relative step of 1/16, from the
// float exponent and the top mantissa bits), then steps of 2^15.  Fine where
// a region's chain starts steep (k_stream's open points of a uniform input
// crowd there: its edge strips), no coarser than 2^15 further on;
// non-decreasing in d, so an earlier slot still means a smaller k1.  (The
// batched path keeps even steps of 2^kBatchSlotShift.)
__device__ inline uint32_t list_slot(uint32_t d)
{
    if (d < 16u) return d;
    if (d < (1u << 19)) return (__float_as_uint((float)d) >> 19) - (131u << 4) + 16u;  // exact float
    return 256u + (min(d, (1u << 23) - 1u) >> 15) - 16u;
}
// (2^19 - 1 maps to slot 255, 2^19 to 256; any d, an out-of-domain set's
// too, below 256 + 2^8 - 16)
static_assert(((145u - 131u) << 4) + 15u + 16u == 255u && 256u + 256u - 16u <= (uint32_t)kBatchSlots, "list_slot range");
constexpr int kBatchChunks = 64, kBatchChunk = 128;                // the first staircase sample
constexpr int kBatchRounds = 32;                                   // pre-hull rounds at most
constexpr int64_t kBatchMaxSet = 1 << 22;                          // larger sets: single-hull path
static_assert(kBatchList >= 2 * (int)kBatchRoundMax, "a round must fit beside a compacted list");
static_assert(kBatchCand / kBatchBlock <= 8 && kBatchPolyMax % kBatchBlock == 0, "per-thread shares");
// LDS: [staircase u32 x 4S][raw slot minima u32 x 4S] [list u32 x
// kBatchList].  Once the stream is done the region slot minima (u64 x
// 4*kBatchSlots) and region staircase (u32 x 4*kBatchSlots) take the
// staircase's place, the sort keys (u64 x kBatchCand) theirs once the
// regions are filtered, and the polygon view everything once the SPA is
// done.  The staircase sits at offset 0 so that its reads need no base
// address.
constexpr size_t kBatchOffStair = 0;
constexpr size_t kBatchOffRaw = kBatchOffStair + 4 * 4 * (size_t)kStairSlots;
constexpr size_t kBatchOffSmin = 0;
constexpr size_t kBatchOffSexc = kBatchOffSmin + 8 * 4 * (size_t)kBatchSlots;
constexpr size_t kBatchOffKey = 0;
constexpr size_t kBatchOffList =
    std::max(std::max(kBatchOffRaw + 4 * 4 * (size_t)kStairSlots, kBatchOffSexc + 4 * 4 * (size_t)kBatchSlots),
             8 * (size_t)kBatchCand);
// (the polygon view may reach past the list: it is built after the list's
// last read)
constexpr size_t kBatchLds = std::max(kBatchOffList + 4 * (size_t)kBatchList,
                                      16 * (size_t)kBatchPolyMax + 2 * (2 * (size_t)kBatchPolyMax + 8));
static_assert(kBatchLds <= 78 * 1024, "two workgroups per CU");

struct BatchPoly {  // polygon view of the LDS
    int32_t* x;
    int32_t* y;
    int32_t* idx;
    uint8_t* reg;  // region 0..3, 4 for an extreme point
    uint8_t* alive;
    uint16_t* lst;
    uint16_t* dq;
};

// The polygon view of LDS at b: x, y, idx (int32), the pre-hull list
// (u16), Melkman's deque (u16, 2 * kBatchPolyMax + 8), region and alive
// flags (u8).
__device__ inline BatchPoly poly_view(unsigned char* b)
{
    BatchPoly Pl;
    Pl.x = reinterpret_cast<int32_t*>(b);
    b += 4 * kBatchPolyMax;
    Pl.y = reinterpret_cast<int32_t*>(b);
    b += 4 * kBatchPolyMax;
    Pl.idx = reinterpret_cast<int32_t*>(b);
    b += 4 * kBatchPolyMax;
    Pl.lst = reinterpret_cast<uint16_t*>(b);
    b += 2 * kBatchPolyMax;
    Pl.dq = reinterpret_cast<uint16_t*>(b);
    b += 2 * (2 * kBatchPolyMax + 8);
    Pl.reg = b;
    b += kBatchPolyMax;
    Pl.alive = b;
    return Pl;
}

__device__ inline i64 turn_xy(const BatchPoly& P, uint32_t a, uint32_t b, uint32_t c)
{
    return (i64)(P.x[b] - P.x[a]) * (i64)(P.y[c] - P.y[a]) - (i64)(P.y[b] - P.y[a]) * (i64)(P.x[c] - P.x[a]);
}

// Melkman on the polygon lst[0..n) of vertices (x, y, idx) by one thread,
// with the conventions of the host finish (consecutive duplicates dropped,
// collinear prefix, newest vertex dropped when collinear).  Writes the hull,
// rotated to the lowest-then-leftmost vertex, to out; returns its size, or
// -1 when the deque would leave its room (not a simple polygon).
__device__ int batch_melkman(const BatchPoly& P, uint32_t n0, int32_t* __restrict__ out)
{
    // consecutive duplicates, cyclically
    uint16_t* const p = P.lst;  // compacted in place
    uint32_t np = 0;
    for (uint32_t i = 0; i < n0; ++i) {
        const uint32_t v = p[i];
        if (np && P.x[p[np - 1]] == P.x[v] && P.y[p[np - 1]] == P.y[v]) continue;
        p[np++] = (uint16_t)v;
    }
    while (np > 1 && P.x[p[np - 1]] == P.x[p[0]] && P.y[p[np - 1]] == P.y[p[0]]) --np;
    uint16_t* const d = P.dq;
    uint32_t h = 0;
    if (np <= 2) {
        for (uint32_t i = 0; i < np; ++i) d[i] = p[i];
        h = np;
    } else {
        uint32_t k = 2;
        while (k < np && turn_xy(P, p[0], p[1], p[k]) == 0) ++k;
        const i64 dx = P.x[p[1]] - P.x[p[0]], dy = P.y[p[1]] - P.y[p[0]];
        uint32_t lo = 0, hi = 0;
        i64 tlo = 0, thi = 0;
        for (uint32_t i = 0; i < k; ++i) {
            const i64 t = dx * (P.x[p[i]] - P.x[p[0]]) + dy * (P.y[p[i]] - P.y[p[0]]);
            if (t < tlo) { tlo = t; lo = i; }
            if (t > thi) { thi = t; hi = i; }
        }
        if (k == np) {
            d[0] = p[lo];
            d[1] = p[hi];
            h = 2;
        } else {
            const int cap = 2 * (int)np + 8;
            int bot = (int)np + 2, top = bot + 3;
            d[bot] = p[k];
            d[top] = p[k];
            if (turn_xy(P, p[lo], p[hi], p[k]) > 0) {
                d[bot + 1] = p[lo];
                d[bot + 2] = p[hi];
            } else {
                d[bot + 1] = p[hi];
                d[bot + 2] = p[lo];
            }
            for (uint32_t i = k + 1; i < np; ++i) {
                const uint32_t v = p[i];
                if (turn_xy(P, d[bot], d[bot + 1], v) > 0 && turn_xy(P, d[top - 1], d[top], v) > 0) continue;
                while (turn_xy(P, d[bot], d[bot + 1], v) <= 0) {
                    if (top - bot < 2) return -1;
                    ++bot;
                }
                if (bot < 1) return -1;
                d[--bot] = (uint16_t)v;
                while (turn_xy(P, d[top - 1], d[top], v) <= 0) {
                    if (top - bot < 2) return -1;
                    --top;
                }
                if (top + 1 >= cap) return -1;
                d[++top] = (uint16_t)v;
            }
            int first = bot;
            if (turn_xy(P, d[top - 1], d[bot], d[bot + 1]) <= 0) first = bot + 1;
            h = 0;
            for (int i = first; i < top; ++i) d[h++] = d[i];
        }
    }
    uint32_t start = 0;
    for (uint32_t i = 1; i < h; ++i) {
        const uint32_t a = d[i], b = d[start];
        if (P.y[a] < P.y[b] || (P.y[a] == P.y[b] && P.x[a] < P.x[b])) start = i;
    }
    for (uint32_t i = 0; i < h; ++i) out[i] = P.idx[d[(start + i) % h]];
    return (int)h;
}

// The staircase of the batched stream from its slot minima raw[f*S + s]
// (frames R1..R4, S = kStairSlots): per frame the exclusive prefix minimum
// over the slots, stored in k_stream's layout.  Every thread of the
// workgroup takes part; ends with a workgroup barrier.
__device__ inline void batch_stair(const uint32_t* raw, uint32_t* sst, uint32_t* scratch)
{
    constexpr uint32_t S = kStairSlots, kPer = 4 * S / kBatchBlock, kThreadsPerFrame = S / kPer;
    constexpr uint32_t kWavesPerFrame = kThreadsPerFrame / 64;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / 64;
    const uint32_t f = tid / kThreadsPerFrame, j0 = (tid % kThreadsPerFrame) * kPer;
    uint32_t v[kPer];
    uint32_t m = ~0u;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        v[k] = raw[f * S + j0 + k];
        m = min(m, v[k]);
    }
    const uint32_t incl = wave_incl_min(m);
    uint32_t excl = __shfl_up(incl, 1);
    if (lane == 0) excl = ~0u;
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    for (uint32_t w = f * kWavesPerFrame; w < wave; ++w) excl = min(excl, scratch[w]);
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t s = j0 + k;
        const uint32_t at = f == 0 ? 2 * s : f == 1 ? 2 * S + 2 * s : f == 2 ? 2 * (S - 1 - s) + 1 : 2 * S + 2 * (S - 1 - s) + 1;
        sst[at] = excl;
        excl = min(excl, v[k]);
    }
    __syncthreads();
    // each slot pair as one interval (the test of k_stream)
    u64* const s64 = reinterpret_cast<u64*>(sst);
    for (uint32_t e = tid; e < 2 * S; e += kBatchBlock) {
        const u64 pv = s64[e];
        const bool xs = e < S;
        s64[e] = stair_interval(xs ? (uint32_t)pv : (uint32_t)(pv >> 32), xs ? (uint32_t)(pv >> 32) : (uint32_t)pv);
    }
    __syncthreads();
}

// poly_finish's rounds on a polygon of at most 64 vertices by one wave
// (the first; every lane calls it), vertex k of the current polygon in lane
// k: neighbours by lane exchange, removal by compaction of the kept lanes (a
// forward permute), no workgroup barrier.  A convex result is written to out
// (*s_flag = 1), else the polygon left is in Pl.lst (*s_flag = 0); *s_ext
// receives its size.  Kept out of line: it runs once per set.
__device__ __attribute__((noinline)) void wave_poly_rounds(BatchPoly Pl, uint32_t npoly, uint32_t first,
                                                           int32_t* __restrict__ out, uint32_t* s_flag,
                                                           uint32_t* s_ext)
{
    const uint32_t lane = lane_id();
    bool keep = lane < npoly && Pl.alive[lane] != 0;
    uint32_t vid = lane, rg = keep ? Pl.reg[lane] : 0u;
    int32_t x = keep ? Pl.x[lane] : 0, y = keep ? Pl.y[lane] : 0;
    uint32_t cnt = 0;
    bool convex = false;
    for (int round = 0;; ++round) {
        // kept lanes to lanes 0 .. cnt-1 in order, the others above
        const u64 km = ballot(keep);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
        cnt = (uint32_t)__popcll(km);
        const uint32_t to = keep ? below : cnt + (lane - below);
        vid = (uint32_t)__builtin_amdgcn_ds_permute((int)(to * 4), (int)vid);
        rg = (uint32_t)__builtin_amdgcn_ds_permute((int)(to * 4), (int)rg);
        x = __builtin_amdgcn_ds_permute((int)(to * 4), x);
        y = __builtin_amdgcn_ds_permute((int)(to * 4), y);
        if (round == kBatchRounds) break;  // (a removal in every round: Melkman)
        const bool act = lane < cnt;
        const uint32_t pl = lane == 0 ? (cnt ? cnt - 1 : 0u) : lane - 1, nl = lane + 1 >= cnt ? 0u : lane + 1;
        const int32_t px = __shfl(x, (int)pl), py = __shfl(y, (int)pl);
        const int32_t nx = __shfl(x, (int)nl), ny = __shfl(y, (int)nl);
        const i64 t = (i64)(x - px) * (i64)(ny - py) - (i64)(y - py) * (i64)(nx - px);
        const bool bad = act && t <= 0;
        const bool gone = bad && rg < 4;
        if (ballot(gone) == 0) {
            convex = ballot(bad) == 0 && cnt >= 3;
            break;
        }
        keep = act && !gone;
    }
    const bool act = lane < cnt;
    if (convex) {
        const u64 fm = ballot(act && vid == first);
        const uint32_t start = fm ? (uint32_t)__builtin_ctzll(fm) : 0u;
        if (act) out[lane >= start ? lane - start : lane + cnt - start] = Pl.idx[vid];
    } else if (act) {
        Pl.lst[lane] = (uint16_t)vid;
    }
    if (lane == 0) {
        *s_flag = convex ? 1u : 0u;
        *s_ext = cnt;
    }
}

// The polygon phase: pre-hull rounds on the polygon Pl[0 .. npoly) (x, y,
// idx, region 0..3 or 4 for an extreme point, all alive), then the hull into
// out.  A chain vertex whose turn with its current neighbours (points of its
// chain or the region's extreme points) is not a left turn lies between the
// chord of those neighbours and the quadrilateral edge, inside the hull of
// four points of the set: all such vertices go together, round after round.
// When a round removes nothing and every vertex, the extreme points
// included, is a strict left turn, the simple polygon is convex and is the
// hull: it is written out in parallel from polygon position `first`
// (P_miny, the lowest then leftmost point).  Otherwise one thread runs
// Melkman.  A polygon of at most 64 vertices takes the rounds in one wave
// (a vertex per lane), a larger one in the workgroup.  Every thread of the
// workgroup (kBatchBlock) calls it; returns the hull size, the same in every
// thread, or -1 when Melkman's deque would leave its room.  s_flag, s_ext,
// s_start: LDS words.
__device__ int poly_finish(const BatchPoly& Pl, uint32_t npoly, uint32_t first, int32_t* __restrict__ out,
                           uint32_t* scratch, uint32_t* s_flag, uint32_t* s_ext, uint32_t* s_start)
{
    const uint32_t tid = threadIdx.x;
    if (npoly <= 64) {
        // the rounds by the first wave
        if (tid < 64) wave_poly_rounds(Pl, npoly, first, out, s_flag, s_ext);
        __syncthreads();
        const bool convex = *s_flag != 0;
        const uint32_t cnt = *s_ext;
        if (convex) return (int)cnt;
        if (tid == 0) *s_start = (uint32_t)batch_melkman(Pl, cnt, out);
        __syncthreads();
        return (int)*s_start;
    }
    auto compact_poly = [&]() -> uint32_t {
        constexpr int kPer = kBatchPolyMax / kBatchBlock;
        uint32_t mine = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = tid * kPer + k;
            mine += (i < npoly && Pl.alive[i]) ? 1u : 0u;
        }
        uint32_t n_alive;
        uint32_t o = block_excl_sum<kBatchWaves>(mine, scratch, n_alive);
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = tid * kPer + k;
            if (i < npoly && Pl.alive[i]) Pl.lst[o++] = (uint16_t)i;
        }
        __syncthreads();
        return n_alive;
    };
    uint32_t n_alive = compact_poly();
    bool convex = false;
    for (int round = 0; round < kBatchRounds; ++round) {
        if (tid == 0) {
            *s_flag = 0;
            *s_ext = 0;
        }
        __syncthreads();
        for (uint32_t p = tid; p < n_alive; p += kBatchBlock) {
            const uint32_t u = Pl.lst[p == 0 ? n_alive - 1 : p - 1], i = Pl.lst[p],
                           c = Pl.lst[p + 1 == n_alive ? 0 : p + 1];
            if (turn_xy(Pl, u, i, c) <= 0) {
                if (Pl.reg[i] < 4) {
                    Pl.alive[i] = 0;
                    *s_flag = 1;
                } else {
                    *s_ext = 1;
                }
            }
        }
        __syncthreads();
        const bool removed = *s_flag != 0, ext_flat = *s_ext != 0;
        if (!removed) {
            convex = !ext_flat && n_alive >= 3;
            break;
        }
        n_alive = compact_poly();
    }
    if (convex) {
        for (uint32_t p = tid; p < n_alive; p += kBatchBlock) {
            if (Pl.lst[p] == first) *s_start = p;
        }
        __syncthreads();
        const uint32_t start = *s_start;
        for (uint32_t p = tid; p < n_alive; p += kBatchBlock) {
            const uint32_t o = p >= start ? p - start : p + n_alive - start;
            out[o] = Pl.idx[Pl.lst[p]];
        }
        return (int)n_alive;
    }
    if (tid == 0) *s_start = (uint32_t)batch_melkman(Pl, n_alive, out);
    __syncthreads();
    return (int)*s_start;
}

// The open lists of one k_stream call, for k_batch_hull's list mode: the
// lists (index per open point, region points apart), their counts, the
// per-workgroup extreme partials, and the pinned header the host reads.
struct ListSrc {
    const uint32_t* idx;
    const u64* xym;  // x | y << 23 | mask << 46 per open point
    const uint32_t* wgcount;
    const ExtPartial* parts;
    DevHeader* host_hdr;
    uint32_t* stab;  // the sample table, cleared here (k_cand, which also clears it, may not run)
    uint32_t region, nlists;
    uint32_t cap;    // open points the list mode takes at most (<= kBatchList)
};

template <int kBatchUnroll, bool kFromLists = false>
__global__ __launch_bounds__(kBatchBlock, kBatchWavesPerSimd) void k_batch_hull(const float* __restrict__ pts,
                                                            const int64_t* __restrict__ offsets,
                                                            const int32_t* __restrict__ order,
                                                            int32_t* __restrict__ out_idx,
                                                            int32_t* __restrict__ out_counts, uint32_t pts_odd,
                                                            int32_t num_sets, int64_t single_n, ListSrc src)
{
    __shared__ __align__(16) unsigned char smem[kBatchLds];
    __shared__ u64 s_ek[kBatchWaves][4];
    __shared__ uint32_t s_bad[kBatchWaves], s_eidx[4];
    __shared__ uint32_t scratch[kBatchWaves];
    __shared__ uint32_t wcnt[2][kBatchWaves];
    __shared__ Quad sq;
    __shared__ uint32_t s_n, s_flag, s_ext, s_start, s_rcnt[4];
    // list mode: the listed points' coordinates (x | y << 23), from the
    // open records, so that the later steps read no point twice
    __shared__ uint32_t s_lxy[kFromLists ? 2 * kBatchList : 1];
    uint32_t* const lidx = reinterpret_cast<uint32_t*>(smem + kBatchOffList);
    uint32_t* const raw = reinterpret_cast<uint32_t*>(smem + kBatchOffRaw);
    uint32_t* const sst = reinterpret_cast<uint32_t*>(smem + kBatchOffStair);
    const uint32_t tid = threadIdx.x, lane = lane_id();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid / 64);  // a scalar
    const u64 lt = (1ull << lane) - 1ull;
    // (order may be absent: set b; offsets are checked here because the
    // stream-ordered entry point cannot read them on the host)
    const int32_t set = order ? order[blockIdx.x] : (int32_t)blockIdx.x;
    if (set < 0 || set >= num_sets) return;
    // (without offsets: one set, points [0, single_n))
    const int64_t base = offsets ? offsets[set] : 0, end = offsets ? offsets[set + 1] : single_n;
    if (base < 0 || end < base) {
        if (threadIdx.x == 0) out_counts[set] = CH_EINVAL;
        return;
    }
    if (!kFromLists && end - base > kBatchMaxSet) {  // (list mode reads only the open points)
        if (threadIdx.x == 0) out_counts[set] = kBatchRedo;
        return;
    }
    const uint32_t m = (uint32_t)(end - base);
#ifdef CH_PHASE_TIMING
    u64 ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#endif
    CH_PHASE_MARK(0);
    const float* const ps = pts + 2 * base;
    const v2f* const p2 = reinterpret_cast<const v2f*>(ps);
    if (m == 0) {
        if (tid == 0) out_counts[set] = 0;
        return;
    }
    constexpr uint32_t S = kStairSlots;
    // the extreme keys of the listed points: K0 = (x, M - y), K1 = (y, x);
    // minima then maxima (coordinates only: the smallest index among a
    // point's exact duplicates is found later, in the list)
    u64 ek[4] = {~0ull, ~0ull, 0ull, 0ull};
    // the domain check: a coordinate is in the domain iff its conversion
    // converts back to the same float (up to the sign of 0) and is at most
    // M; differing bits and the largest conversion accumulate
    uint32_t err = 0, hi = 0;
    if constexpr (kFromLists) {
        // ---- list mode: k_stream's open points are the list (its
        // staircase test already ran); the extreme keys from its partials.
        // More open points than the list holds leave the input to the
        // single-hull kernels. ----
        uint32_t* const s_lst = reinterpret_cast<uint32_t*>(smem + kBatchOffRaw);  // list starts (the sample's room)
        const uint32_t nl = src.nlists;
        uint32_t c[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint32_t l = 2 * tid + u;
            c[u] = 0;
            if (l < nl) {
                c[u] = src.wgcount[l];
                const ExtPartial pp = src.parts[l];
                ek[0] = min(ek[0], pp.kmin[0]);
                ek[1] = min(ek[1], pp.kmin[1]);
                ek[2] = max(ek[2], pp.kmax[0]);
                ek[3] = max(ek[3], pp.kmax[1]);
                err |= pp.err;
            }
        }
        // starts: list l at s_lst[l] (thread t: lists 2t and 2t + 1)
        uint32_t L;
        const uint32_t e0 = block_excl_sum<kBatchWaves>(c[0] + c[1], scratch, L);
        if (2 * tid < nl) s_lst[2 * tid] = e0;
        if (2 * tid + 1 < nl) s_lst[2 * tid + 1] = e0 + c[0];
        if (L > src.cap) {
            if (tid == 0) out_counts[set] = kBatchRedo;
            return;
        }
        __syncthreads();
        // Entry e of the list: its list from an owner array (the
        // staircase's room, free in the list mode), which each thread fills
        // for its two lists; then every load of the thread in flight
        // together (past L: the first list's first slot, read and dropped),
        // then the LDS writes.  (A list longer than the others only makes
        // its thread's loop longer: at most L <= kBatchList entries.)
        uint16_t* const s_own = reinterpret_cast<uint16_t*>(smem + kBatchOffStair);
        static_assert(2 * (size_t)kBatchList <= 4 * 4 * (size_t)kStairSlots && kStreamGrid <= 65536, "owner array");
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint32_t l = 2 * tid + u, first = u == 0 ? e0 : e0 + c[0];
            for (uint32_t q = 0; q < c[u]; ++q) s_own[first + q] = (uint16_t)l;
        }
        __syncthreads();
        uint32_t lst[kBatchPerList];
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            const uint32_t e = k * kBatchBlock + tid;
            lst[k] = e < L ? s_own[e] : 0u;
        }
        size_t at[kBatchPerList];
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            const uint32_t e = k * kBatchBlock + tid, l = lst[k];
            at[k] = e < L ? (size_t)l * src.region + (e - s_lst[l]) : 0;
        }
        uint32_t gi[kBatchPerList];
        u64 gr[kBatchPerList];
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            gi[k] = src.idx[at[k]];
            gr[k] = src.xym[at[k]];
        }
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            const uint32_t e = k * kBatchBlock + tid;
            if (e < L) {
                lidx[e] = gi[k];
                s_lxy[2 * e] = (uint32_t)gr[k] & kM;
                s_lxy[2 * e + 1] = (uint32_t)(gr[k] >> 23) & kM;
            }
        }
        if (tid == 0) s_n = L;
        __syncthreads();
    } else {
    constexpr uint32_t S = kStairSlots;
    
        // ---- the first staircase, from a sample of runs of consecutive points ----
        for (uint32_t e = tid; e < 4 * S; e += kBatchBlock) raw[e] = ~0u;
        if (tid == 0) s_n = 0;
        __syncthreads();
        auto lower = [&](uint32_t x, uint32_t y) {  // x, y in [0, M]
            atomicMin(&raw[0 * S + (x >> kStairShift)], y);         // R1: (x, y)
            atomicMin(&raw[1 * S + (y >> kStairShift)], x ^ kM);    // R2: (y, M-x)
            atomicMin(&raw[2 * S + ((x ^ kM) >> kStairShift)], y ^ kM);  // R3: (M-x, M-y)
            atomicMin(&raw[3 * S + ((y ^ kM) >> kStairShift)], x);  // R4: (M-y, x)
        };
        if (m > (2u * kBatchUnroll * kBatchBlock)) {
            constexpr uint32_t kThreads = kBatchBlock / kBatchChunks, kPer = kBatchChunk / kThreads;
            const uint32_t c = tid / kThreads, sub = tid % kThreads;
            const uint32_t start = (uint32_t)(((u64)c * (m - kBatchChunk)) / (kBatchChunks - 1));
            v2f v[kPer];
    #pragma unroll
            for (uint32_t k = 0; k < kPer; ++k) v[k] = p2[start + k * kThreads + sub];
            // out-of-domain values only need to stay in range here: such a set
            // fails with a domain error
    #pragma unroll
            for (uint32_t k = 0; k < kPer; ++k) lower(coord_u32(v[k].x) & kM, coord_u32(v[k].y) & kM);
        }
        __syncthreads();
        batch_stair(raw, sst, scratch);
    
        // ---- stream: domain check, staircase test, list the open points ----
        // points before the first 16-byte boundary of the set (pts_odd: whether
        // pts itself starts 8 bytes past one)
        const uint32_t head = (uint32_t)(((uint64_t)base + pts_odd) & 1u);
        const uint32_t n4 = (m - head) / 2;
        const bool tail = ((m - head) & 1u) != 0;
        const v4f* const p4 = reinterpret_cast<const v4f*>(ps + 2 * head);
        const u64* const sx64 = reinterpret_cast<const u64*>(sst);
        const u64* const sy64 = sx64 + S;
        auto slot_of = [](uint32_t v) { return (v >> kStairShift) & (S - 1); };
        auto check = [&](float fx, float fy, uint32_t X, uint32_t Y) {
            err |= (__float_as_uint((float)X) ^ __float_as_uint(fx)) | (__float_as_uint((float)Y) ^ __float_as_uint(fy));
            hi = max(hi, max(X, Y));
        };
        uint32_t wtot = 0;  // points this wave listed since the last compaction (uniform in the wave)
    
        // one point of every lane, the whole wave together (the append is
        // wave-wide)
        auto list_point = [&](uint32_t X, uint32_t Y, uint32_t idx, bool valid, u64 sxv, u64 syv) {
            // outside the slots' intervals (the comparisons' lane masks as
            // they are)
            const u64 bal = (cmp_mask_gt(Y - (uint32_t)sxv, (uint32_t)(sxv >> 32)) |
                             cmp_mask_gt(X - (uint32_t)syv, (uint32_t)(syv >> 32))) &
                            ballot(valid);
            if (bal) {
                const bool open = (bal >> lane) & 1u;
                uint32_t first = 0;
                if (lane == 0) first = atomicAdd(&s_n, (uint32_t)__popcll(bal));
                first = __shfl(first, 0);
                if (open) {
                    lidx[first + (uint32_t)__popcll(bal & lt)] = idx;
                    const uint32_t x = X & kM, y = Y & kM;
                    lower(x, y);
                    const u64 k0 = ((u64)x << 32) | (y ^ kM), k1 = ((u64)y << 32) | x;
                    ek[0] = min(ek[0], k0);
                    ek[1] = min(ek[1], k1);
                    ek[2] = max(ek[2], k0);
                    ek[3] = max(ek[3], k1);
                }
                wtot += (uint32_t)__popcll(bal);
            }
        };
        auto visit_one = [&](float fx, float fy, uint32_t idx, bool valid) {
            const uint32_t X = cvt_u32_sat(fx), Y = cvt_u32_sat(fy);
            check(fx, fy, X, Y);  // a lane without a point rechecks point idx
            list_point(X, Y, idx, valid, sx64[slot_of(X)], sy64[slot_of(Y)]);
        };
        // the list again against the staircase rebuilt from the slot minima;
        // every thread takes part, after a workgroup barrier with no append
        // pending
        auto compact = [&]() -> uint32_t {
            batch_stair(raw, sst, scratch);
            const uint32_t n = s_n;
            uint32_t id[kBatchPerList];
            v2f v[kBatchPerList];
    #pragma unroll
            for (int k = 0; k < kBatchPerList; ++k) {
                const uint32_t e = k * kBatchBlock + tid;
                id[k] = e < n ? lidx[e] : 0u;
            }
    #pragma unroll
            for (int k = 0; k < kBatchPerList; ++k) v[k] = p2[id[k]];
            uint32_t keep = 0;
    #pragma unroll
            for (int k = 0; k < kBatchPerList; ++k) {
                const uint32_t X = cvt_u32_sat(v[k].x) & kM, Y = cvt_u32_sat(v[k].y) & kM;
                const u64 sxv = sx64[X >> kStairShift], syv = sy64[Y >> kStairShift];
                const bool open = Y - (uint32_t)sxv > (uint32_t)(sxv >> 32) || X - (uint32_t)syv > (uint32_t)(syv >> 32);
                if (k * kBatchBlock + tid < n && open) keep |= 1u << k;
            }
            uint32_t kept;
            uint32_t at = block_excl_sum<kBatchWaves>((uint32_t)__popc(keep), scratch, kept);
    #pragma unroll
            for (int k = 0; k < kBatchPerList; ++k) {
                if ((keep >> k) & 1u) lidx[at++] = id[k];
            }
            if (tid == 0) s_n = kept;
            wtot = wave == 0 ? kept : 0u;
            __syncthreads();
            return kept;
        };
    
        if (wave == 0) {
            if (head) visit_one(ps[0], ps[1], 0, lane == 0);
            if (tail) visit_one(ps[2 * (m - 1)], ps[2 * (m - 1) + 1], m - 1, lane == 0);
        }
        constexpr uint32_t kR4 = (uint32_t)kBatchUnroll * kBatchBlock;  // float4s per round
        const uint32_t rounds = (n4 + kR4 - 1) / kR4;
        auto load_round = [&](uint32_t r, v4f* v) {
    #pragma unroll
            for (int u = 0; u < kBatchUnroll; ++u)
                v[u] = __builtin_nontemporal_load(p4 + min(r * kR4 + u * kBatchBlock + tid, n4 - 1));
        };
        // loads run two rounds ahead of the tests
        v4f va[kBatchUnroll], vb[kBatchUnroll], vc[kBatchUnroll];
        if (rounds > 0) load_round(0, va);
        if (rounds > 1) load_round(1, vb);
        bool full = false;  // the same in every thread
        // (uniform) the fill at the last check, counting the two points the head
        // and tail visits may have listed before it; rounds since; the wcnt
        // buffer of the next check
        uint32_t known = 2, since = 0, par = 0;
        for (uint32_t r = 0; r < rounds; ++r) {
            if (r + 2 < rounds) load_round(r + 2, vc);
    #pragma unroll
            for (int u = 0; u < kBatchUnroll; ++u) {
                const uint32_t g = r * kR4 + u * kBatchBlock + tid;
                const bool valid = g < n4;
                const uint32_t i0 = head + 2 * min(g, n4 - 1);
                const uint32_t X0 = cvt_u32_sat(va[u].x), Y0 = cvt_u32_sat(va[u].y);
                const uint32_t X1 = cvt_u32_sat(va[u].z), Y1 = cvt_u32_sat(va[u].w);
                const u64 sx0 = sx64[slot_of(X0)], sy0 = sy64[slot_of(Y0)];
                const u64 sx1 = sx64[slot_of(X1)], sy1 = sy64[slot_of(Y1)];
                // (a lane past the end rechecks the last points)
                check(va[u].x, va[u].y, X0, Y0);
                check(va[u].z, va[u].w, X1, Y1);
                list_point(X0, Y0, i0, valid, sx0, sy0);
                list_point(X1, Y1, i0 + 1, valid, sx1, sy1);
            }
            // The list holds at most known + since * (2u * kBatchUnroll * kBatchBlock) points now and
            // the next round adds at most (2u * kBatchUnroll * kBatchBlock): only when that bound
            // could pass the list's room is the fill taken (a workgroup
            // barrier), the same in every thread: each wave posts its own count
            // (double-buffered: a wave that runs ahead to the next check writes
            // the other buffer).
            ++since;
            if (known + (since + 1) * (2u * kBatchUnroll * kBatchBlock) > (uint32_t)kBatchList) {
                if (lane == 0) wcnt[par][wave] = wtot;
                __syncthreads();
                uint32_t fill = 0;
    #pragma unroll
                for (int w = 0; w < kBatchWaves; ++w) fill += wcnt[par][w];
                par ^= 1u;
                if (fill > (uint32_t)kBatchList - (2u * kBatchUnroll * kBatchBlock)) {
                    fill = compact();
                    // a list still too full after the compaction: the set has
                    // too many open points for the workgroup
                    if (fill > (uint32_t)kBatchList - (2u * kBatchUnroll * kBatchBlock)) {
                        full = true;
                        break;
                    }
                }
                known = fill;
                since = 0;
            }
    #pragma unroll
            for (int u = 0; u < kBatchUnroll; ++u) {
                va[u] = vb[u];
                vb[u] = vc[u];
            }
        }
        __syncthreads();  // every append of the stream is in the list
        if (full) {
            if (tid == 0) out_counts[set] = kBatchRedo;
            return;
        }
    
    }
    CH_PHASE_MARK(1);
    // ---- the extreme points and the quadrilateral ----
    ek[0] = wave_min_u64(ek[0]);
    ek[1] = wave_min_u64(ek[1]);
    ek[2] = ~wave_min_u64(~ek[2]);
    ek[3] = ~wave_min_u64(~ek[3]);
    const bool wave_bad = ballot((err & 0x7fffffffu) != 0 || hi > kM) != 0;
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) s_ek[wave][e] = ek[e];
        s_bad[wave] = wave_bad ? 1u : 0u;
    }
    __syncthreads();
    if (tid < 4) {  // thread e combines key e over the waves
        u64 v = s_ek[0][tid];
        for (int w = 1; w < kBatchWaves; ++w) v = tid < 2 ? min(v, s_ek[w][tid]) : max(v, s_ek[w][tid]);
        const uint32_t hi = (uint32_t)(v >> 32) & kM, lo = (uint32_t)v & kM;
        // K0 gives (x, M - y) of P_minx and P_maxx, K1 (y, x) of P_miny and P_maxy
        const uint32_t e = tid == 0 ? 0u : tid == 1 ? 1u : tid == 2 ? 2u : 3u;
        sq.X[e] = (e & 1u) ? lo : hi;
        sq.Y[e] = (e & 1u) ? hi : lo ^ kM;
        s_eidx[tid] = ~0u;
        s_rcnt[tid] = 0;
    }
    __syncthreads();
    if (tid == 0) {
        quad_edges(sq);
        uint32_t any = 0;
        for (int w = 0; w < kBatchWaves; ++w) any |= s_bad[w];
        sq.err = any ? kErrDomain : 0u;
        s_flag = 0;
    }
    u64* const smin = reinterpret_cast<u64*>(smem + kBatchOffSmin);
    uint32_t* const sexc = reinterpret_cast<uint32_t*>(smem + kBatchOffSexc);
    for (int e = tid; e < 4 * kBatchSlots; e += kBatchBlock) smin[e] = ~0ull;
    __syncthreads();
    if (sq.err) {
        if (tid == 0) {
            out_counts[set] = CH_EDOMAIN;
            if constexpr (kFromLists) {
                src.host_hdr->err = kErrDomain;
                src.host_hdr->fin_done = 0;
            }
        }
        if constexpr (kFromLists)  // (the tail does not run after a domain error)
            for (int e = tid; e < kStabWords; e += kBatchBlock) src.stab[e] = 0;
        return;
    }
    const uint32_t L = s_n;
    const Quad Q = sq;

    CH_PHASE_MARK(2);
    // ---- exact regions and region slot minima of the listed points ----
    u64 rec[kBatchPerList];
    uint32_t rslot[kBatchPerList];  // a record's filter slot (0 without a record)
    uint32_t kf[4];  // k1 of each region's first point
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t k2;
        to_frame((uint32_t)q, Q.X[q], Q.Y[q], kf[q], k2);
    }
    {
        uint32_t id[kBatchPerList];
        v2f v[kBatchPerList];
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            const uint32_t e = k * kBatchBlock + tid;
            id[k] = e < L ? lidx[e] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            if constexpr (kFromLists) {
                const uint32_t e = min(k * kBatchBlock + tid, (uint32_t)kBatchList - 1);
                v[k] = v2f{(float)s_lxy[2 * e], (float)s_lxy[2 * e + 1]};
            } else {
                v[k] = p2[id[k]];
            }
        }
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            rec[k] = ~0ull;
            if constexpr (kFromLists) rslot[k] = 0;
            if (k * kBatchBlock + tid < L) {
                const uint32_t X = (uint32_t)v[k].x, Y = (uint32_t)v[k].y;
                // the extreme points' smallest indices among their duplicates
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (X == Q.X[e] && Y == Q.Y[e]) atomicMin(&s_eidx[e], id[k]);
                }
                const uint32_t q = region_of(Q, X, Y);
                if (q < 4) {
                    uint32_t k1, k2;
                    to_frame(q, X, Y, k1, k2);
                    const uint32_t f = q == 0 ? kf[0] : q == 1 ? kf[1] : q == 2 ? kf[2] : kf[3];
                    const uint32_t sl = kFromLists ? list_slot(k1 - f) : (k1 >> kBatchSlotShift);
                    atomicMin(&smin[q * kBatchSlots + sl], ((u64)k2 << 23) | k1);
                    rec[k] = ((u64)q << 46) | ((u64)k1 << 23) | k2;
                    if constexpr (kFromLists) rslot[k] = q * kBatchSlots + sl;
                }
            }
        }
    }
    __syncthreads();
    {
        // exclusive prefix minimum per region over its slots, seeded with the
        // region's first point (a quarter of the threads own each region,
        // kPer consecutive slots per thread)
        constexpr uint32_t kPer = 4 * kBatchSlots / kBatchBlock;
        constexpr uint32_t kThreadsPerRegion = kBatchSlots / kPer, kWavesPerRegion = kThreadsPerRegion / 64;
        const uint32_t q = tid / kThreadsPerRegion, j0 = (tid % kThreadsPerRegion) * kPer;
        uint32_t v[kPer];
        uint32_t mn = ~0u;
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) {
            const u64 mk = smin[q * kBatchSlots + j0 + k];
            v[k] = mk == ~0ull ? ~0u : (uint32_t)(mk >> 23);
            mn = min(mn, v[k]);
        }
        const uint32_t incl = wave_incl_min(mn);
        uint32_t excl = __shfl_up(incl, 1);
        if (lane == 0) excl = ~0u;
        if (lane == 63) scratch[wave] = incl;
        __syncthreads();
        for (uint32_t w = q * kWavesPerRegion; w < wave; ++w) excl = min(excl, scratch[w]);
        excl = min(excl, sq.sigma[q]);
#pragma unroll
        for (uint32_t k = 0; k < kPer; ++k) {
            sexc[q * kBatchSlots + j0 + k] = excl;
            excl = min(excl, v[k]);
        }
        __syncthreads();
    }
    // survivors become sort keys: record << kBatchPosBits | list position
    uint32_t keep = 0;
    if constexpr (kFromLists) {
        // (one workgroup: every row's two LDS reads issued together, then
        // the tests)
        u64 best[kBatchPerList];
        uint32_t exc[kBatchPerList];
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            best[k] = smin[rslot[k]];
            exc[k] = sexc[rslot[k]];
        }
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            const uint32_t k1 = (uint32_t)(rec[k] >> 23) & kM, k2 = (uint32_t)rec[k] & kM;
            const u64 me = ((u64)k2 << 23) | k1;
            if (rec[k] != ~0ull && k2 < exc[k] && !(best[k] < me && (uint32_t)(best[k] & kM) <= k1)) keep |= 1u << k;
        }
    } else {
        // (two workgroups per CU: registers are short, one row at a time)
#pragma unroll
        for (int k = 0; k < kBatchPerList; ++k) {
            if (rec[k] != ~0ull) {
                const uint32_t k1 = (uint32_t)(rec[k] >> 23) & kM, k2 = (uint32_t)rec[k] & kM;
                const uint32_t sl = ((uint32_t)(rec[k] >> 46)) * kBatchSlots + (k1 >> kBatchSlotShift);
                const u64 me = ((u64)k2 << 23) | k1, best = smin[sl];
                if (k2 < sexc[sl] && !(best < me && (uint32_t)(best & kM) <= k1)) keep |= 1u << k;
            }
        }
    }
    uint32_t nsort;
    uint32_t at = block_excl_sum<kBatchWaves>((uint32_t)__popc(keep), scratch, nsort);
    if (nsort > (uint32_t)kBatchCand) {
        if (tid == 0) out_counts[set] = kBatchRedo;
        return;
    }
    u64* const skey = reinterpret_cast<u64*>(smem + kBatchOffKey);
#pragma unroll
    for (int k = 0; k < kBatchPerList; ++k) {
        if ((keep >> k) & 1u) skey[at++] = (rec[k] << kBatchPosBits) | (u64)(k * kBatchBlock + tid);
    }
    uint32_t P2 = 1;
    while (P2 < nsort) P2 <<= 1;
    for (uint32_t e = nsort + tid; e < P2; e += kBatchBlock) skey[e] = ~0ull;
    __syncthreads();

    CH_PHASE_MARK(3);
    // ---- sort (ascending): up to 64 records in one wave's registers, more
    // by the workgroup's bitonic network in LDS (measured: a wave's network
    // over 256 records took 11 us against 7 us for the workgroup's) ----
    if (P2 <= 64) {
        if (wave == 0) wave_sort_keys<1>(skey, P2);
        __syncthreads();
    } else if (nsort <= (uint32_t)kBatchBlock) {
        // by rank: each thread counts the keys below its own (distinct keys)
        const u64 mine = tid < nsort ? skey[tid] : 0ull;
        uint32_t rank = 0;
        for (uint32_t j = 0; j < nsort; ++j) rank += skey[j] < mine ? 1u : 0u;
        __syncthreads();
        if (tid < nsort) skey[rank] = mine;
        __syncthreads();
    } else {
        for (uint32_t size = 2; size <= P2; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (uint32_t t = tid; t < P2 / 2; t += kBatchBlock) {
                    const uint32_t i = 2 * t - (t & (stride - 1)), j = i + stride;
                    const bool up = (i & size) == 0;
                    const u64 x = skey[i], y = skey[j];
                    if ((x > y) == up) {
                        skey[i] = y;
                        skey[j] = x;
                    }
                }
                __syncthreads();
            }
        }
    }

    CH_PHASE_MARK(4);
    // ---- SPA over the sorted records; chain positions ----
    // thread t holds sorted records [t*per, t*per + per), per <= 8
    const uint32_t per = (P2 + kBatchBlock - 1) / kBatchBlock;
    uint32_t run = ~0u;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t r = tid * per + k;
        if (r < nsort) {
            const u64 key = skey[r] >> kBatchPosBits;
            run = min(run, ((3u - (uint32_t)(key >> 46)) << 23) | (uint32_t)(key & kM));
        }
    }
    uint32_t unused;
    uint32_t pm = block_excl_min<kBatchWaves>(run, scratch, unused);
    uint32_t kmask = 0;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t r = tid * per + k;
        if (r >= nsort) break;
        const u64 key = skey[r] >> kBatchPosBits;
        const uint32_t q = (uint32_t)(key >> 46), k2 = (uint32_t)(key & kM);
        uint32_t thr = sq.sigma[q];
        if ((pm >> 23) == 3u - q) thr = min(thr, pm & kM);
        if (k2 < thr) kmask |= 1u << k;
        pm = min(pm, ((3u - q) << 23) | k2);
    }
    uint32_t nchain;
    const uint32_t rank = block_excl_sum<kBatchWaves>((uint32_t)__popc(kmask), scratch, nchain);
    if (nchain + 4 > (uint32_t)kBatchPolyMax) {
        if (tid == 0) out_counts[set] = kBatchRedo;
        return;
    }
    // the kept records and their smallest duplicate index, in registers
    u64 krec[8];
    uint32_t kidx[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        krec[k] = 0;
        kidx[k] = 0;
        if ((kmask >> k) & 1u) {
            const uint32_t r = tid * per + k;
            constexpr u64 kPosMask = (1ull << kBatchPosBits) - 1;
            const u64 key = skey[r], rc = key >> kBatchPosBits;
            uint32_t idx = lidx[(uint32_t)(key & kPosMask)];
            for (uint32_t j = r + 1; j < nsort && (skey[j] >> kBatchPosBits) == rc; ++j)
                idx = min(idx, lidx[(uint32_t)(skey[j] & kPosMask)]);
            krec[k] = rc;
            kidx[k] = idx;
            atomicAdd(&s_rcnt[(uint32_t)(rc >> 46)], 1u);
        }
    }
    __syncthreads();

    CH_PHASE_MARK(5);
    // ---- the polygon in LDS (everything above is dead now) ----
    const BatchPoly Pl = poly_view(smem);
    const uint32_t npoly = nchain + 4;
    uint32_t rbase[4];  // polygon position of E_q
    {
        uint32_t acc = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rbase[q] = acc;
            acc += 1 + s_rcnt[q];
        }
    }
    if (tid < 4) {
        const uint32_t q = tid, o = q == 0 ? rbase[0] : q == 1 ? rbase[1] : q == 2 ? rbase[2] : rbase[3];
        Pl.x[o] = (int32_t)sq.X[q];
        Pl.y[o] = (int32_t)sq.Y[q];
        Pl.idx[o] = (int32_t)s_eidx[q];
        Pl.reg[o] = 4;
        Pl.alive[o] = 1;
    }
    {
        // chain rank over all regions; E_0 .. E_q precede a record of region q
        uint32_t rr = rank;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if ((kmask >> k) & 1u) {
                const uint32_t q = (uint32_t)(krec[k] >> 46), k1 = (uint32_t)(krec[k] >> 23) & kM,
                               k2 = (uint32_t)krec[k] & kM;
                const uint32_t o = rr + q + 1;
                const uint32_t a2 = (q & 1u) ? k2 : k1;
                const uint32_t b2 = (q & 1u) ? k1 : k2;
                Pl.x[o] = (int32_t)(((q ^ (q >> 1)) & 1u) ? a2 ^ kM : a2);
                Pl.y[o] = (int32_t)((q & 2u) ? b2 ^ kM : b2);
                Pl.idx[o] = (int32_t)kidx[k];
                Pl.reg[o] = (uint8_t)q;
                Pl.alive[o] = 1;
                ++rr;
            }
        }
    }
    __syncthreads();

    CH_PHASE_MARK(6);
    // ---- pre-hull rounds, the finish ----
    const int h = poly_finish(Pl, npoly, rbase[1], out_idx + base, scratch, &s_flag, &s_ext, &s_start);
    if (tid == 0) out_counts[set] = h < 0 ? kBatchRedo : h;
#ifdef CH_PHASE_TIMING
    CH_PHASE_MARK(7);
    if (tid == 0 && h >= 0) {
        const int b = kFromLists ? 8 : 0;
        for (int k = 0; k < 7; ++k) atomicAdd(&g_phase_ticks[b + k], ph[k + 1] - ph[k]);
        atomicAdd(&g_phase_ticks[16 + (kFromLists ? 1 : 0)], 1ull);
    }
#endif
    if constexpr (kFromLists) {
        // the sample table, clear for the next call (after a hand-back the
        // tail's k_cand clears it)
        if (h >= 0)
            for (int e = tid; e < kStabWords; e += kBatchBlock) src.stab[e] = 0;
        if (tid == 0 && h >= 0) {
            // the counts for the host (the single-hull kernels, gated off,
            // publish nothing)
            DevHeader* const hh = src.host_hdr;
            for (int q = 0; q < 4; ++q) {
                hh->ext_x[q] = sq.X[q];
                hh->ext_y[q] = sq.Y[q];
                hh->ext_idx[q] = s_eidx[q];
                hh->s2[q] = s_rcnt[q];
                hh->fin_w2[q] = s_rcnt[q];
            }
            hh->err = 0;
            hh->open = s_n;
            hh->cand = nsort;
            hh->chain = nchain;
            hh->fin_hull = h;
            hh->fin_fail = 0;
            hh->fin_done = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Step 7 on the device (Section 2.1.3's hull, computed without Melkman's
// sequential deque), across workgroups.
//
// Every hull vertex of region q lies on the lower hull, in q's frame, of the
// region's kept points and its two extreme points E_q (start) and E_{q+1}
// (end): a point v is a strict hull vertex iff some line through v has every
// other of these points strictly on its inner side (larger k2); the points
// of the other regions and of the quadrilateral are then on that side too
// (the region's corner triangle holds everything below such a line).
//
// k_chain cut the region chain into segments; within a segment the kept
// points of one region form a piece P (ascending k1, descending k2).  Let H
// be P's lower hull (P itself when the pre-hull converged).  For a line
// touching H from below with slope s, a point a left of H is strictly above
// it iff s > slope of the lower tangent from a to H, and a point b right of
// H iff s < slope of the tangent from H to b.  With
//   sigma_L = max over the region's points left of P and E_q of the tangent
//             slope from a to H,
//   sigma_R = min over the points right of P and E_{q+1} of the tangent
//             slope from H to b,
// a vertex v of H with incoming and outgoing edge slopes s_in < s_out (minus
// and plus infinity at H's ends) is a strict hull vertex iff
//   max(s_in, sigma_L) < min(s_out, sigma_R).
// Tangents are binary searches over H in LDS.  A piece whose bounding box
// lies strictly above the line found from the neighbouring segments cannot
// raise sigma_L (or lower sigma_R) and is skipped.
//
// The output is written in the order E_1, R2, E_2, R3, E_3, R4, E_0, R1 (the
// hull from P_miny counter-clockwise): items (the extreme points and the
// pieces) are taken in that order by ticket, and each item's first output
// position is an exclusive prefix sum over the earlier items' vertex counts
// by decoupled look-back: an item publishes its count, then sums its
// predecessors' counts back to the nearest one that has published its
// inclusive prefix.  An item waits only on items with smaller tickets, which
// running workgroups hold and complete without waiting on later ones, so the
// look-back always ends.
// ---------------------------------------------------------------------------
constexpr int kWideBlock = 256;
constexpr int kWideWaves = kWideBlock / 64;
constexpr int kWideNear = 2;                // neighbouring segments searched before the pruning pass
constexpr int kWideList = 1024;             // segments left after pruning, processed per pass
constexpr uint32_t kWideSpinMax = 1u << 20; // safety bound of one look-back wait (never reached)
constexpr u64 kLookAgg = 1ull << 62, kLookIncl = 2ull << 62;

// A slope dy/dx with dx >= 0; dx == 0 stands for minus infinity (dy < 0) or
// plus infinity (dy > 0).  Every product is below 2^46.
struct Slope {
    i64 dy, dx;
};

__device__ inline bool slope_less(Slope a, Slope b)
{
    if (a.dx == 0 && b.dx == 0) return a.dy < 0 && b.dy > 0;
    if (a.dx == 0) return a.dy < 0;
    if (b.dx == 0) return b.dy > 0;
    return a.dy * b.dx < b.dy * a.dx;
}

// A line through two points of the region, from (a1, a2) to (b1, b2) with
// a1 <= b1 (frame coordinates): a tangent candidate.
struct Line {
    uint32_t a1, a2, b1, b2;
    uint32_t ok;
};

__device__ inline Slope line_slope(const Line& l) { return Slope{(i64)l.b2 - (i64)l.a2, (i64)l.b1 - (i64)l.a1}; }

// The better of two candidates: the larger slope (want_max) or the smaller.
__device__ inline Line line_better(const Line& x, const Line& y, bool want_max)
{
    const bool y_less = slope_less(line_slope(y), line_slope(x));
    const bool x_less = slope_less(line_slope(x), line_slope(y));
    const bool take_y = y.ok && (!x.ok || (want_max ? x_less : y_less));
    // (field by field: a select of whole structs goes through scratch memory)
    Line r;
    r.a1 = take_y ? y.a1 : x.a1;
    r.a2 = take_y ? y.a2 : x.a2;
    r.b1 = take_y ? y.b1 : x.b1;
    r.b2 = take_y ? y.b2 : x.b2;
    r.ok = take_y ? y.ok : x.ok;
    return r;
}

// Workgroup reduction of one candidate per thread; every thread gets the
// result.  sh: kWideWaves Lines of LDS.
__device__ inline Line line_reduce(Line v, bool want_max, Line* sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Line o;
        o.a1 = __shfl_xor(v.a1, off);
        o.a2 = __shfl_xor(v.a2, off);
        o.b1 = __shfl_xor(v.b1, off);
        o.b2 = __shfl_xor(v.b2, off);
        o.ok = __shfl_xor(v.ok, off);
        v = line_better(v, o, want_max);
    }
    if (lane_id() == 0) sh[threadIdx.x / 64] = v;
    __syncthreads();
    Line r = sh[0];
    for (int w = 1; w < kWideWaves; ++w) r = line_better(r, sh[w], want_max);
    __syncthreads();
    return r;
}

// The lower tangent from a point a left of the hull H[0 .. h) (ascending k1,
// strictly convex): the first k with H[k+1] not strictly below the line from
// a through H[k] (the predicate holds for a prefix of k).
__device__ inline uint32_t tangent_from_left(const uint32_t* hk1, const uint32_t* hk2, uint32_t h, uint32_t a1,
                                             uint32_t a2)
{
    uint32_t lo = 0, hi = h - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (frame_turn(a1, a2, hk1[mid], hk2[mid], hk1[mid + 1], hk2[mid + 1]) < 0) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The lower tangent from the hull to a point b right of it: the first k with
// H[k+1] not strictly below the line from H[k] to b.
__device__ inline uint32_t tangent_to_right(const uint32_t* hk1, const uint32_t* hk2, uint32_t h, uint32_t b1,
                                            uint32_t b2)
{
    uint32_t lo = 0, hi = h - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (frame_turn(hk1[mid], hk2[mid], b1, b2, hk1[mid + 1], hk2[mid + 1]) < 0) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Decoupled look-back by wave 0: publishes the item's count, sums the counts
// of the items before it back to the nearest published inclusive prefix,
// publishes its own inclusive prefix and returns the exclusive one (the same
// in every lane of wave 0).  state: flag (2 bits) | epoch (30 bits) | value.
__device__ inline uint32_t look_back(u64* states, uint32_t t, uint32_t epoch, uint32_t count, bool& fail)
{
    const uint32_t lane = lane_id();
    const u64 ep = (u64)(epoch & 0x3FFFFFFFu) << 32;
    if (lane == 0) __hip_atomic_store(states + t, kLookAgg | ep | count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0, spins = 0;
    int j = (int)t - 1;
    while (j >= 0) {
        const int at = j - (int)lane;
        u64 v = kLookIncl | ep;  // before the first item: an inclusive prefix of 0
        if (at >= 0) v = __hip_atomic_load(states + at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool ready = (v & 0x3FFFFFFF00000000ull) == ep && (v >> 62) != 0;
        const bool incl = ready && (v >> 62) == 2;
        const u64 im = __ballot(incl), rm = __ballot(ready);
        const uint32_t last = im ? (uint32_t)__builtin_ctzll(im) : 63u;
        const u64 need = last == 63 ? ~0ull : ((2ull << last) - 1ull);
        if ((rm & need) == need) {
            excl += wave_sum(lane <= last ? (uint32_t)v : 0u);
            if (im) break;
            j -= 64;
        } else {
            if (++spins > kWideSpinMax) {
                fail = true;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    if (lane == 0 && !fail)
        __hip_atomic_store(states + t, kLookIncl | ep | (u64)(excl + count), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// Region layout of the chain for the wide finish: region q's SPA survivors
// occupy chain positions [rs, rs + s2[q]), so its pieces lie in segments
// first .. first + nseg - 1.
struct WideRegion {
    uint32_t first, nseg;
};

// Segment s's kept points of region q: offset inside the segment and count.
__device__ inline void piece_of(const uint32_t* __restrict__ segcnt, uint32_t s, uint32_t q, uint32_t& off,
                                uint32_t& cnt)
{
    const v4u c = reinterpret_cast<const v4u*>(segcnt)[s];
    off = (q > 0 ? c.x : 0u) + (q > 1 ? c.y : 0u) + (q > 2 ? c.z : 0u);
    cnt = q == 0 ? c.x : q == 1 ? c.y : q == 2 ? c.z : c.w;
}

__global__ __launch_bounds__(kWideBlock) void k_finish_wide(DevHeader* __restrict__ hdr,
                                                            const uint32_t* __restrict__ segcnt,
                                                            const PolyRec* __restrict__ kept,
                                                            u64* __restrict__ states,
                                                            int32_t* __restrict__ out_idx,
                                                            int32_t* __restrict__ out_count,
                                                            DevHeader* __restrict__ host_hdr,
                                                            const int32_t* __restrict__ gate)
{
    __shared__ uint32_t hk1[kSeg], hk2[kSeg];
    __shared__ int32_t hidx[kSeg];
    __shared__ uint16_t hrank[kSeg];  // 1 + output rank of a strict vertex, 0 otherwise
    __shared__ uint32_t slist[kWideList], s_lo[kWideList], s_pre[kWideList];  // listed segments: id, offset, prefix
    __shared__ Line sh_line[kWideWaves];
    __shared__ uint32_t scratch[kWideWaves];
    __shared__ uint32_t s_t, s_h, s_nl, s_bad, s_base, s_fail;
    const uint32_t tid = threadIdx.x;
    if (gated_off(gate)) return;
    if (hdr->err) {
        // a failed step: the count is the call's status
        if (blockIdx.x == 0 && tid == 0) {
            host_hdr->fin_done = 0;
            *out_count = (hdr->err & kErrDomain) ? CH_EDOMAIN : CH_EHIP;
        }
        return;
    }
    const uint32_t epoch = hdr->epoch;
    // the region layout, in LDS (indexed by region)
    __shared__ WideRegion R[4];
    if (tid == 0) {
        uint32_t rs = 0;
        for (int q = 0; q < 4; ++q) {
            const uint32_t m = hdr->s2[q];
            R[q].first = rs / kSeg;
            R[q].nseg = m ? (rs + m - 1) / kSeg - rs / kSeg + 1 : 0u;
            rs += m;
        }
    }
    __syncthreads();
    uint32_t nitems = 4;
    for (int q = 0; q < 4; ++q) nitems += R[q].nseg;
    if (blockIdx.x >= nitems) return;  // (no ticket could be left for it)
    bool fail = false;

    for (;;) {
        if (tid == 0) s_t = __hip_atomic_fetch_add(&hdr->wide_ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t t = s_t;
        __syncthreads();
        if (t >= nitems) break;
        // the item: extreme point E_q, or region q's piece in segment s
        uint32_t q = 0, s = 0, rest = t;
        bool is_ext = false;
        for (int k = 0; k < 4; ++k) {
            const uint32_t qq = (uint32_t)(k + 1) & 3u;  // E_1, R2, E_2, R3, E_3, R4, E_0, R1
            if (rest == 0) {
                q = qq;
                is_ext = true;
                break;
            }
            rest -= 1;
            if (rest < R[qq].nseg) {
                q = qq;
                s = R[qq].first + rest;
                break;
            }
            rest -= R[qq].nseg;
        }
        uint32_t count = 0, h = 0;
        if (is_ext) {
            // a coincident earlier extreme point (in the order E_1, E_2, E_3,
            // E_0) has been written already
            auto same = [&](uint32_t a, uint32_t b) {
                return hdr->ext_x[a] == hdr->ext_x[b] && hdr->ext_y[a] == hdr->ext_y[b];
            };
            const bool dup = q == 2 ? same(2, 1) : q == 3 ? same(3, 2) : q == 0 ? (same(0, 3) || same(0, 1)) : false;
            count = dup ? 0u : 1u;
        } else {
            uint32_t off, cnt;
            piece_of(segcnt, s, q, off, cnt);
            // the piece in frame coordinates
            for (uint32_t j = tid; j < cnt; j += kWideBlock) {
                const PolyRec r = kept[(size_t)s * kSeg + off + j];
                uint32_t k1, k2;
                to_frame(q, (uint32_t)r.x, (uint32_t)r.y, k1, k2);
                hk1[j] = k1;
                hk2[j] = k2;
                hidx[j] = r.idx;
            }
            if (tid == 0) s_bad = 0;
            __syncthreads();
            for (uint32_t j = tid + 1; j + 1 < cnt; j += kWideBlock)
                if (frame_turn(hk1[j - 1], hk2[j - 1], hk1[j], hk2[j], hk1[j + 1], hk2[j + 1]) <= 0) s_bad = 1;
            __syncthreads();
            if (s_bad) {
                // not convex (the pre-hull stopped early): its lower hull, in place
                if (tid == 0) {
                    uint32_t m = 0;
                    for (uint32_t j = 0; j < cnt; ++j) {
                        const uint32_t k1 = hk1[j], k2 = hk2[j];
                        const int32_t ix = hidx[j];
                        while (m >= 2 && frame_turn(hk1[m - 2], hk2[m - 2], hk1[m - 1], hk2[m - 1], k1, k2) <= 0) --m;
                        hk1[m] = k1;
                        hk2[m] = k2;
                        hidx[m] = ix;
                        ++m;
                    }
                    s_h = m;
                }
            } else if (tid == 0) {
                s_h = cnt;
            }
            __syncthreads();
            h = s_h;
            if (h) {
                const uint32_t qn = (q + 1) & 3;
                uint32_t e1, e2, f1, f2;
                to_frame(q, hdr->ext_x[q], hdr->ext_y[q], e1, e2);    // E_q: left of every point
                to_frame(q, hdr->ext_x[qn], hdr->ext_y[qn], f1, f2);  // E_{q+1}: right of every point
                const uint32_t lo_seg = R[q].first, hi_seg = R[q].first + R[q].nseg;  // [lo_seg, hi_seg)
                Line best_l = Line{0, 0, 0, 0, 0u}, best_r = Line{0, 0, 0, 0, 0u};
                // the listed segments' points (slist[0 .. nl)) as candidates,
                // all at once: per segment its place and count, their prefix
                // sum, then every point by one thread, four loads in flight
                auto eval_list = [&](uint32_t nl, bool left) __attribute__((always_inline)) -> Line {
                    for (uint32_t e = tid; e < nl; e += kWideBlock) {
                        uint32_t o, c;
                        piece_of(segcnt, slist[e], q, o, c);
                        s_lo[e] = o;
                        s_pre[e] = c;
                    }
                    __syncthreads();
                    uint32_t total;
                    {
                        constexpr int kPer = kWideList / kWideBlock;
                        uint32_t c[kPer], sum = 0;
#pragma unroll
                        for (int k = 0; k < kPer; ++k) {
                            const uint32_t e = tid * kPer + k;
                            c[k] = e < nl ? s_pre[e] : 0u;
                            sum += c[k];
                        }
                        uint32_t run = block_excl_sum(sum, scratch, total);  // (its barriers follow the reads above)
#pragma unroll
                        for (int k = 0; k < kPer; ++k) {
                            const uint32_t e = tid * kPer + k;
                            if (e < nl) s_pre[e] = run;
                            run += c[k];
                        }
                    }
                    __syncthreads();
                    Line acc = Line{0, 0, 0, 0, 0u};
                    constexpr int kLoads = 4;
                    for (uint32_t i0 = 0; i0 < total; i0 += kLoads * kWideBlock) {
                        PolyRec r[kLoads];
#pragma unroll
                        for (int u = 0; u < kLoads; ++u) {
                            const uint32_t i = i0 + u * kWideBlock + tid;
                            if (i < total) {
                                uint32_t e = 0;  // the last listed segment with pre <= i
                                for (uint32_t st = kWideList / 2; st > 0; st >>= 1)
                                    if (e + st < nl && s_pre[e + st] <= i) e += st;
                                r[u] = kept[(size_t)slist[e] * kSeg + s_lo[e] + (i - s_pre[e])];
                            }
                        }
#pragma unroll
                        for (int u = 0; u < kLoads; ++u) {
                            if (i0 + u * kWideBlock + tid < total) {
                                uint32_t k1, k2;
                                to_frame(q, (uint32_t)r[u].x, (uint32_t)r[u].y, k1, k2);
                                Line l;
                                if (left) {
                                    const uint32_t k = tangent_from_left(hk1, hk2, h, k1, k2);
                                    l = Line{k1, k2, hk1[k], hk2[k], 1u};
                                } else {
                                    const uint32_t k = tangent_to_right(hk1, hk2, h, k1, k2);
                                    l = Line{hk1[k], hk2[k], k1, k2, 1u};
                                }
                                acc = line_better(acc, l, left);
                            }
                        }
                    }
                    return line_reduce(acc, left, sh_line);
                };
                // side 0: points left of the piece (E_q and earlier segments),
                // the largest tangent slope; side 1: points right of it (later
                // segments and E_{q+1}), the smallest
                for (int side = 0; side < 2; ++side) {
                    const bool left = side == 0;
                    // the extreme point and the neighbouring segments first
                    if (tid == 0) {
                        uint32_t nn = 0;
                        for (int d = 1; d <= kWideNear; ++d) {
                            const int64_t sg = left ? (int64_t)s - d : (int64_t)s + d;
                            if (sg >= (int64_t)lo_seg && sg < (int64_t)hi_seg) slist[nn++] = (uint32_t)sg;
                        }
                        s_nl = nn;
                    }
                    __syncthreads();
                    Line cur = eval_list(s_nl, left);
                    {
                        Line ext;
                        if (left) {
                            const uint32_t k = tangent_from_left(hk1, hk2, h, e1, e2);
                            ext = Line{e1, e2, hk1[k], hk2[k], 1u};
                        } else {
                            const uint32_t k = tangent_to_right(hk1, hk2, h, f1, f2);
                            ext = Line{hk1[k], hk2[k], f1, f2, 1u};
                        }
                        cur = line_better(cur, ext, left);
                    }
                    // the other segments: those whose bounding box is not
                    // strictly above the current line, in passes of at most
                    // kWideList segments
                    const uint32_t a0 = left ? lo_seg : (uint32_t)(s + kWideNear + 1);
                    const uint32_t a1 = left ? (s > lo_seg + kWideNear ? s - kWideNear : lo_seg) : hi_seg;
                    for (uint32_t p0 = a0; p0 < a1; p0 += kWideList) {
                        if (tid == 0) s_nl = 0;
                        __syncthreads();
                        const uint32_t p1 = min(a1, p0 + (uint32_t)kWideList);
                        const bool vertical = cur.b1 == cur.a1;  // (only E_q above the first point: nothing to prune)
                        for (uint32_t sg = p0 + tid; sg < p1; sg += kWideBlock) {
                            uint32_t o, c;
                            piece_of(segcnt, sg, q, o, c);
                            if (!c) continue;
                            bool keep = true;
                            if (!vertical) {
                                const PolyRec r0 = kept[(size_t)sg * kSeg + o];
                                const PolyRec r1 = kept[(size_t)sg * kSeg + o + c - 1];
                                uint32_t x1, x2, y1, y2;
                                to_frame(q, (uint32_t)r0.x, (uint32_t)r0.y, x1, x2);  // largest k2
                                to_frame(q, (uint32_t)r1.x, (uint32_t)r1.y, y1, y2);  // largest k1, smallest k2
                                // the box [x1, y1] x [y2, x2] is strictly above the
                                // line when its two lower corners are
                                keep = !(frame_turn(cur.a1, cur.a2, cur.b1, cur.b2, x1, y2) > 0 &&
                                         frame_turn(cur.a1, cur.a2, cur.b1, cur.b2, y1, y2) > 0);
                            }
                            if (keep) slist[atomicAdd(&s_nl, 1u)] = sg;
                        }
                        __syncthreads();
                        const uint32_t nl = s_nl;
                        if (nl) cur = line_better(cur, eval_list(nl, left), left);
                        __syncthreads();
                    }
                    if (left) best_l = cur;
                    else best_r = cur;
                }
                // strict vertices of the piece's hull, in order
                const Slope sl = best_l.ok ? line_slope(best_l) : Slope{-1, 0};
                const Slope sr = best_r.ok ? line_slope(best_r) : Slope{1, 0};
                for (uint32_t k0 = 0; k0 < h; k0 += kWideBlock) {
                    const uint32_t k = k0 + tid;
                    bool strict = false;
                    if (k < h) {
                        const Slope sin = k > 0 ? Slope{(i64)hk2[k] - (i64)hk2[k - 1], (i64)hk1[k] - (i64)hk1[k - 1]}
                                                : Slope{-1, 0};
                        const Slope sout = k + 1 < h ? Slope{(i64)hk2[k + 1] - (i64)hk2[k], (i64)hk1[k + 1] - (i64)hk1[k]}
                                                     : Slope{1, 0};
                        const Slope lo = slope_less(sin, sl) ? sl : sin;
                        const Slope hi = slope_less(sr, sout) ? sr : sout;
                        strict = slope_less(lo, hi);
                    }
                    uint32_t tot;
                    const uint32_t r = block_excl_sum(strict ? 1u : 0u, scratch, tot);
                    // (1 + rank in the piece; the output position needs the
                    // item's base from the look-back)
                    if (k < h) hrank[k] = (uint16_t)(strict ? count + r + 1 : 0u);
                    count += tot;
                    __syncthreads();
                }
            }
        }
        // the item's first output position (the first item's workgroup
        // first sets the count to a sentinel that only the last item's
        // total replaces, so that a failed item can never be overwritten)
        if (t == 0 && tid == 0) {
            st_dev(reinterpret_cast<uint32_t*>(out_count), (uint32_t)kBatchRedo);
            stores_done();
        }
        if (tid < 64) {
            bool f = false;
            const uint32_t base = look_back(states, t, epoch, count, f);
            if (tid == 0) {
                s_base = base;
                s_fail = f ? 1u : 0u;
            }
        }
        __syncthreads();
        const uint32_t base = s_base;
        fail = s_fail != 0;
        if (is_ext) {
            if (tid == 0 && count) out_idx[base] = (int32_t)hdr->ext_idx[q];
        } else {
            for (uint32_t k = tid; k < h; k += kWideBlock) {
                const uint32_t r = hrank[k];
                if (r) out_idx[base + r - 1] = hidx[k];
            }
        }
        if (t == nitems - 1 && tid == 0) {
            // the last item: the hull size and the counts for the host
            const int32_t total = (int32_t)(base + count);
            if (!fail) atomicCAS(out_count, kBatchRedo, total);
            host_hdr->fin_hull = total;
            for (int k = 0; k < 4; ++k) {
                uint32_t w = 0;
                const uint32_t first = R[k].first, ns = R[k].nseg;
                for (uint32_t sg = first; sg < first + ns; ++sg) {
                    uint32_t o, c;
                    piece_of(segcnt, sg, k, o, c);
                    w += c;
                }
                host_hdr->fin_w2[k] = w;
            }
            if (!fail) host_hdr->fin_done = 1u;
        }
        if (fail) {
            // a look-back wait ran out (not expected): the call reports an
            // error instead of a wrong hull, and hull2d finishes on the host
            if (tid == 0) {
                atomicExch(out_count, (int32_t)CH_EHIP);
                host_hdr->fin_fail = 1u;
            }
            break;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// The host finish's input when the device finish gave up (not expected): one
// workgroup gathers the polygon [P_minx, R1, P_miny, R2, P_maxx, R3, P_maxy,
// R4] from k_chain's device copy (per segment and region, the kept points at
// the segment's start) into pinned host memory, densely, as (x, y) pairs and
// indices, so that the host reads one contiguous array.
//   pass 1  the kept points per region (the polygon position of each
//           extreme point);
//   pass 2  per run of kBatchBlock segments, an exclusive scan of their
//           counts; each kept point of the run finds its segment by binary
//           search and goes to its polygon position.
// The header receives the vertex count (gat_count; 0 when it exceeds `cap`)
// and the per-region counts.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBatchBlock) void k_gather(const DevHeader* __restrict__ hdr,
                                                        const uint32_t* __restrict__ segcnt,
                                                        const PolyRec* __restrict__ kept, int32_t* __restrict__ out_xy,
                                                        int32_t* __restrict__ out_idx, uint32_t cap,
                                                        DevHeader* __restrict__ host_hdr)
{
    __shared__ uint32_t s_pre[kBatchBlock], s_cum[kBatchBlock][4], s_sg[kBatchBlock];
    __shared__ uint32_t scratch[kBatchWaves];
    __shared__ uint32_t s_reg[4];
    const uint32_t tid = threadIdx.x, lane = lane_id();
    const uint32_t chain = hdr->chain;
    const uint32_t nseg = (chain + kSeg - 1) / kSeg;
    if (tid < 4) s_reg[tid] = 0;
    __syncthreads();

    // ---- pass 1: points per region ----
    uint32_t reg[4] = {0, 0, 0, 0};
    for (uint32_t sg = tid; sg < nseg; sg += kBatchBlock) {
#pragma unroll
        for (int q = 0; q < 4; ++q) reg[q] += segcnt[4 * sg + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t v = wave_sum(reg[q]);
        if (lane == 0 && v) atomicAdd(&s_reg[q], v);
    }
    __syncthreads();
    uint32_t rbase[4], npoly = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        rbase[q] = npoly;
        npoly += 1 + s_reg[q];
    }
    if (npoly > cap) {  // the same in every thread
        if (tid == 0) host_hdr->gat_count = 0;
        return;
    }
    if (tid < 4) {
        const uint32_t q = tid, o = q == 0 ? rbase[0] : q == 1 ? rbase[1] : q == 2 ? rbase[2] : rbase[3];
        out_xy[2 * o] = (int32_t)hdr->ext_x[q];
        out_xy[2 * o + 1] = (int32_t)hdr->ext_y[q];
        out_idx[o] = (int32_t)hdr->ext_idx[q];
    }

    // ---- pass 2: the kept points ----
    uint32_t done = 0;  // kept points of the earlier runs
    for (uint32_t c0 = 0; c0 < nseg; c0 += kBatchBlock) {
        const uint32_t sg = c0 + tid;
        uint32_t c[4] = {0, 0, 0, 0};
        if (sg < nseg) {
#pragma unroll
            for (int q = 0; q < 4; ++q) c[q] = segcnt[4 * sg + q];
        }
        uint32_t all;
        const uint32_t ex = block_excl_sum<kBatchWaves>(c[0] + c[1] + c[2] + c[3], scratch, all);
        s_pre[tid] = ex;
        s_sg[tid] = sg;
        s_cum[tid][0] = c[0];
        s_cum[tid][1] = c[0] + c[1];
        s_cum[tid][2] = c[0] + c[1] + c[2];
        s_cum[tid][3] = c[0] + c[1] + c[2] + c[3];
        __syncthreads();
        const uint32_t nrun = min((uint32_t)kBatchBlock, nseg - c0);
        for (uint32_t p = tid; p < all; p += kBatchBlock) {
            // the last segment of the run with pre <= p holds p (an empty
            // segment shares its pre with the next one)
            uint32_t lo = 0, hi = nrun;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) / 2;
                if (s_pre[mid] <= p) lo = mid;
                else hi = mid;
            }
            const uint32_t j = p - s_pre[lo];
            const uint32_t q = j < s_cum[lo][0] ? 0u : j < s_cum[lo][1] ? 1u : j < s_cum[lo][2] ? 2u : 3u;
            const PolyRec r = kept[s_sg[lo] * kSeg + j];
            const uint32_t o = done + p + q + 1;
            out_xy[2 * o] = r.x;
            out_xy[2 * o + 1] = r.y;
            out_idx[o] = r.idx;
        }
        done += all;
        __syncthreads();
    }
    if (tid == 0) {
        for (int q = 0; q < 4; ++q) host_hdr->fin_w2[q] = s_reg[q];
        host_hdr->gat_count = npoly;
    }
}

// ---------------------------------------------------------------------------
// SPA in subsets (Section 2.2.2; the limitation of Section 4.3): the
// divide-and-conquer variant that the paper implements, kept for the
// discard-effectiveness experiments (the path itself runs the exact rule).
// Thread t checks subset t, `chunk` consecutive points of a region's sorted
// k2 sequence, with the rule of Figure 2: subset 0 starts from the region's
// first point (sigma), a later subset from its own first point, which it
// keeps.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_spa_chunked(const uint32_t* __restrict__ k2, uint32_t m, uint32_t sigma,
                                                        uint32_t chunk, uint8_t* __restrict__ keep)
{
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t s0 = t * chunk;
    if (s0 >= m) return;
    const uint32_t e = (uint32_t)min((uint64_t)m, s0 + chunk);
    u64 thr = t == 0 ? (u64)sigma : ~0ull;
    for (uint32_t i = (uint32_t)s0; i < e; ++i) {
        const uint32_t v = k2[i];
        const bool k = (u64)v < thr;
        keep[i] = k ? 1 : 0;
        if (k) thr = v;
    }
}

// The finished hull, from pinned host memory into the caller's buffers.  The
// host rewrites that memory between calls, so it is read with system-scope
// loads, which no stale cache line can serve.
// p[0 .. n) = v.
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, uint32_t n)
{
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_put_result(const int32_t* host_hull, int32_t h,
                                                       int32_t* __restrict__ out_idx, int32_t* __restrict__ out_count)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < h) out_idx[i] = __hip_atomic_load(host_hull + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (i == 0) *out_count = h;
}

// ---------------------------------------------------------------------------
// Host side: workspaces, the pipeline and the C ABI
// ---------------------------------------------------------------------------

namespace {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr size_t kHostChainDefault = 1u << 20;  // pinned chain records at first
constexpr size_t kHostChainMax = 1u << 24;      // the most it grows to

struct Workspace {
    std::mutex mu;
    int device = 0;
    hipStream_t stream = nullptr;
    size_t cap = 0;  // points
    char* dbuf = nullptr;
    DevHeader* hdr = nullptr;
    ExtPartial* part = nullptr;
    uint32_t* stab = nullptr;       // the sample table (zero between calls)
    uint32_t* open_idx = nullptr;   // k_stream's per-workgroup lists
    u64* open_xym = nullptr;
    uint32_t* wgcount = nullptr;
    uint32_t* rowoff = nullptr;     // k_cand's rows of the bucket table: first position per bucket
    uint32_t* rowmin = nullptr;     // and smallest k2 per bucket
    uint32_t* key[2] = {nullptr, nullptr};  // k_cand's parts: records in chunk order, by bucket
    u64* val[2] = {nullptr, nullptr};
    Buckets bk = {};
    PolyRec* dev_chain = nullptr;
    DevHeader* h_hdr = nullptr;     // pinned, device-visible: written by k_chain
    DevHeader* h_hdr_dev = nullptr; // its device address
    PolyRec* h_chain = nullptr;     // pinned, device-visible
    PolyRec* h_chain_dev = nullptr; // its device address
    size_t h_chain_cap = 0;
    size_t h_chain_want = kHostChainDefault;  // raised by a call whose chain spilled
    int32_t* h_out = nullptr;       // pinned, device-visible: count, then indices
    int32_t* h_out_dev = nullptr;   // its device address
    size_t h_out_cap = 0;
    int32_t* h_pxy = nullptr;       // pinned, device-visible: k_gather's polygon,
    int32_t* h_pidx = nullptr;      // (x, y) pairs and indices
    int32_t* h_pxy_dev = nullptr;
    int32_t* h_pidx_dev = nullptr;
    size_t h_poly_cap = 0;          // vertices
    std::vector<int32_t> xy, idx;   // finish input
    std::vector<PolyRec> spill;     // chain records beyond the pinned buffer
    PolyRec* dev_spill = nullptr;   // device: chain records beyond the pinned buffer
    PolyRec* dev_kept = nullptr;    // device copies of the kept chain points and
    uint32_t* dev_segcnt = nullptr; // their per-segment counts (the device finish)
    u64* states = nullptr;          // k_finish_wide's look-back states (zeroed at allocation)
    uint32_t* h_segcnt = nullptr;   // pinned, device-visible: kept points per segment and region
    uint32_t* h_segcnt_dev = nullptr;
    size_t h_segcnt_cap = 0;        // segments
    int64_t s2[4] = {}, w2[4] = {}, chain = 0;  // counts of the last call
    // batched calls: set offsets and launch order (device), staging (pinned)
    int64_t* b_offsets = nullptr;
    int32_t* b_order = nullptr;
    size_t b_cap = 0;  // sets
    int64_t* h_b_offsets = nullptr;
    int32_t* h_b_order = nullptr;
    int32_t* h_b_counts = nullptr;
    hipEvent_t ev[8] = {};
    bool events = false;
    bool no_events = false;  // hull2d_noalloc's view: never creates or records events
    bool captured = false;   // a HIP graph captured a call on this workspace: it must not move
};

// Launch shape of k_stream for n points whose first `head` (0 or 1) points
// precede the 16-byte aligned part: grid, and the points one workgroup can
// visit (its region in the open lists).
struct StreamShape {
    uint32_t n4, grid, per, region;
};

// ---- launch shapes (ch_tuning), per size class ----
constexpr ch_tuning kDefaultTuning = {1024, 4, 2048, 1024, 1024, 2, 0, 1 << 18, 1 << 15, kBatchList / 2};
constexpr int kTuningClasses = 16;
std::mutex g_tune_mu;
int g_tune_count = 0;
int64_t g_tune_nmax[kTuningClasses];
ch_tuning g_tune[kTuningClasses];

bool tuning_valid(const ch_tuning& t)
{
    const bool grid = t.stream_grid == 128 || t.stream_grid == 256 || t.stream_grid == 512 || t.stream_grid == 1024;
    return grid && (t.stream_unroll == 2 || t.stream_unroll == 4) && t.cand_per_row >= 1024 &&
           t.cand_per_row <= (1 << 20) && t.chain_grid >= 64 && t.chain_grid <= 4096 &&
           t.wide_grid >= 64 && t.wide_grid <= 4096 && (t.batch_unroll == 1 || t.batch_unroll == 2) &&
           (t.batch_order == 0 || t.batch_order == 1) && t.serve_batch_max >= 0 && t.serve_batch_max <= (1 << 22) &&
           t.fused_max >= 0 && t.fused_max <= (1 << 22) && t.list_max >= 0 && t.list_max <= kBatchList;
}

// The shapes of a call with n points: the class with the smallest n_max >= n.
ch_tuning tuning_for(int64_t n)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int best = -1;
    for (int k = 0; k < g_tune_count; ++k)
        if (n >= 0 && g_tune_nmax[k] >= n && (best < 0 || g_tune_nmax[k] < g_tune_nmax[best])) best = k;
    return best >= 0 ? g_tune[best] : kDefaultTuning;
}

// k_stream's shape for n points whose first `head` (0 or 1) points precede
// the 16-byte aligned part: grid (at most grid_max), and the float4s one
// workgroup streams (a whole number of rounds of kBlock * unroll) and the
// points it can visit (its region in the open lists).
StreamShape stream_shape(size_t n, uint32_t head, uint32_t grid_max, uint32_t unroll)
{
    StreamShape sh;
    sh.n4 = (uint32_t)((n - head) / 2);
    const size_t round = (size_t)kBlock * unroll;
    sh.grid = (uint32_t)std::max<size_t>(1, std::min<size_t>(grid_max, (sh.n4 + round - 1) / round));
    const size_t per = std::max<size_t>(1, (sh.n4 + sh.grid - 1) / sh.grid);
    sh.per = (uint32_t)((per + round - 1) / round * round);
    sh.grid = (uint32_t)std::max<size_t>(1, (sh.n4 + sh.per - 1) / sh.per);  // no empty workgroup
    sh.region = 2 * sh.per + 2;  // points one workgroup can visit (+ head and tail)
    return sh;
}

// Records the per-workgroup regions need for any call with up to cap
// points, whatever its launch shape: k_stream's lists take grid regions,
// and k_cand's parts tile the same regions; both grid and the region grow
// with n, so the largest call of each shape bounds the rest.
size_t region_cap(size_t cap)
{
    size_t best = 0;
    for (uint32_t g : {128u, 256u, 512u, 1024u})
        for (uint32_t u : {2u, 4u})
            for (uint32_t head : {0u, 1u}) {
                const StreamShape sh = stream_shape(std::max<size_t>(cap, 2), head, g, u);
                best = std::max(best, (size_t)sh.grid * sh.region);
            }
    return best;
}

// The device workspace for calls with up to cap points: its size, and, when
// w is given, every array's place in it from base.
size_t layout(Workspace* w, char* base, size_t cap)
{
    const size_t rc = region_cap(cap);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* r = base ? base + o : nullptr;
        o += align_up(bytes, 256);
        return r;
    };
    Workspace tmp;
    Workspace& W = w ? *w : tmp;
    // zeroed at allocation: the header, the look-back states, the sample table
    W.hdr = reinterpret_cast<DevHeader*>(take(sizeof(DevHeader)));
    W.states = reinterpret_cast<u64*>(take(sizeof(u64) * (cap / kSeg + 16)));
    W.stab = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kStabWords));
    W.part = reinterpret_cast<ExtPartial*>(take(sizeof(ExtPartial) * kStreamGrid));
    W.bk.cnt = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kBuckets));
    W.bk.off = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kBuckets));
    W.bk.surv = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kBuckets));
    W.bk.lstart = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kBuckets));
    W.bk.lthr = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kBuckets));
    W.bk.bmin = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kBuckets));
    W.bk.wtot = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kScanGrid));
    W.bk.wmin = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kScanGrid));
    W.rowoff = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kCandMaxRows * (kBuckets + 1)));
    W.rowmin = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kCandMaxRows * kBuckets));
    W.wgcount = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kStreamGrid));
    W.open_idx = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * rc));
    W.open_xym = reinterpret_cast<u64*>(take(sizeof(u64) * rc));
    for (int i = 0; i < 2; ++i) W.key[i] = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * rc));
    for (int i = 0; i < 2; ++i) W.val[i] = reinterpret_cast<u64*>(take(sizeof(u64) * rc));
    W.dev_chain = reinterpret_cast<PolyRec*>(take(sizeof(PolyRec) * cap));
    W.dev_spill = reinterpret_cast<PolyRec*>(take(sizeof(PolyRec) * cap));
    W.dev_kept = reinterpret_cast<PolyRec*>(take(sizeof(PolyRec) * cap));
    W.dev_segcnt = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 4 * (cap / kSeg + 1)));
    return o;
}

size_t device_bytes(size_t cap) { return layout(nullptr, nullptr, cap); }

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;
std::atomic<int> g_timing{0};  // 0 off, 1 every stage, 2 steps 1-6 and the finish only
thread_local ch_stats t_stats;
thread_local ch_batch_stats t_bstats;

int hip_status(hipError_t e)
{
    if (e == hipSuccess) return CH_OK;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? CH_ENOMEM : CH_EHIP;
}

inline int hip_status(int rc) { return rc; }  // already a ch_status

#define CH_TRY(expr)                      \
    do {                                  \
        const int rc_ = hip_status(expr); \
        if (rc_ != CH_OK) return rc_;     \
    } while (0)

#define CH_LAUNCH(...)                                 \
    do {                                               \
        __VA_ARGS__;                                   \
        const int rc_ = hip_status(hipGetLastError()); \
        if (rc_ != CH_OK) return rc_;                  \
    } while (0)

int ensure_device(Workspace& w, size_t n)
{
    if (w.dbuf && w.cap >= n) return CH_OK;
    // a captured graph holds the workspace's addresses: it stays until the
    // caller releases the stream
    if (w.captured) return CH_EINVAL;
    size_t cap = std::max<size_t>(n, 1u << 16);
    if (w.cap) cap = std::max(cap, w.cap + w.cap / 2);
    if (w.dbuf) {
        CH_TRY(hipStreamSynchronize(w.stream));
        CH_TRY(hipFree(w.dbuf));
        w.dbuf = nullptr;
        w.cap = 0;
    }
    char* p = nullptr;
    CH_TRY(hipMalloc(&p, device_bytes(cap)));
    w.dbuf = p;
    w.cap = cap;
    layout(&w, p, cap);
    // the header's call counter, the look-back states and the sample table
    // start at zero (they sit together at the start of the layout)
    CH_TRY(hipMemsetAsync(w.hdr, 0, reinterpret_cast<char*>(w.part) - reinterpret_cast<char*>(w.hdr), w.stream));
    return CH_OK;
}

// Pinned buffers: the header, the result (out vertices) and, for the host
// polygon of chainhull_polygon (chain), the chain records and segment counts.
int ensure_host(Workspace& w, size_t out, bool chain)
{
    if (!w.h_hdr) {
        CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_hdr), sizeof(DevHeader), hipHostMallocMapped));
        CH_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&w.h_hdr_dev), w.h_hdr, 0));
    }
    if (chain && w.h_chain && w.h_chain_cap < w.h_chain_want) {  // no kernel of this workspace runs here
        CH_TRY(hipHostFree(w.h_chain));
        w.h_chain = nullptr;
        w.h_chain_cap = 0;
    }
    if (chain && !w.h_chain) {
        CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_chain), sizeof(PolyRec) * w.h_chain_want,
                             hipHostMallocMapped));
        CH_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&w.h_chain_dev), w.h_chain, 0));
        w.h_chain_cap = w.h_chain_want;
    }
    const size_t nseg = w.cap / kSeg + 1;
    if (chain && w.h_segcnt_cap < nseg) {
        if (w.h_segcnt) CH_TRY(hipHostFree(w.h_segcnt));
        w.h_segcnt = nullptr;
        CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_segcnt), sizeof(uint32_t) * 4 * nseg, hipHostMallocMapped));
        CH_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&w.h_segcnt_dev), w.h_segcnt, 0));
        w.h_segcnt_cap = nseg;
    }
    if (w.h_out_cap < out + 1) {
        if (w.h_out) CH_TRY(hipHostFree(w.h_out));
        w.h_out = nullptr;
        const size_t cap = std::max<size_t>(out + 1, 4096);
        CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_out), sizeof(int32_t) * cap, hipHostMallocMapped));
        CH_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&w.h_out_dev), w.h_out, 0));
        w.h_out_cap = cap;
    }
    return CH_OK;
}

Workspace* workspace_for(hipStream_t stream, int* rc)
{
    int dev = 0;
    *rc = hip_status(hipGetDevice(&dev));
    if (*rc != CH_OK) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) return it->second;
    Workspace* w = new Workspace();
    w->device = dev;
    w->stream = stream;
    g_ws[key] = w;
    return w;
}

void free_workspace(Workspace* w)
{
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(w->device);
    (void)hipStreamSynchronize(w->stream);
    if (w->dbuf) (void)hipFree(w->dbuf);
    if (w->h_hdr) (void)hipHostFree(w->h_hdr);
    if (w->h_chain) (void)hipHostFree(w->h_chain);
    if (w->h_out) (void)hipHostFree(w->h_out);
    if (w->h_segcnt) (void)hipHostFree(w->h_segcnt);
    if (w->h_pxy) (void)hipHostFree(w->h_pxy);
    if (w->h_pidx) (void)hipHostFree(w->h_pidx);
    if (w->b_offsets) (void)hipFree(w->b_offsets);
    if (w->b_order) (void)hipFree(w->b_order);
    if (w->h_b_offsets) (void)hipHostFree(w->h_b_offsets);
    if (w->h_b_order) (void)hipHostFree(w->h_b_order);
    if (w->h_b_counts) (void)hipHostFree(w->h_b_counts);
    if (w->events) {
        for (auto& e : w->ev) (void)hipEventDestroy(e);
    }
    (void)hipSetDevice(cur);
    delete w;
}

int record(Workspace& w, int k)
{
    const int mode = g_timing;
    if (!mode || w.no_events) return CH_OK;
    if (mode == 2 && k != 0 && k != 5 && k != 6) return CH_OK;
    if (!w.events) {
        for (auto& e : w.ev) CH_TRY(hipEventCreate(&e));
        w.events = true;
    }
    return hip_status(hipEventRecord(w.ev[k], w.stream));
}

// Steps 1-6 on the device; the counts end in w.h_hdr.  Without fin_idx the
// chains end in w.h_chain (and w.spill).  With fin_idx, k_finish_wide then
// finishes the hull on the device into fin_idx / fin_count
// (h_hdr->fin_done); only if they gave up does gather_polygon fetch the
// polygon for the host finish.  Timing events: 0 | k_sample | 1 | k_stream |
// 2 | k_cand (+ k_count_regions) | 3 | k_scan | 4 | k_bucket_spa, k_chain |
// 5 | k_finish_wide | 6.
// Set for good once a call failed after k_sample and before k_cand (which
// clears the sample table): from then on every call clears its table first.
std::atomic<bool> g_stab_dirty{false};

// Which launches of a call: all of them, the head (through k_stream and
// the list mode, when it runs; then *listed says whether it did), or the
// tail (from k_cand on, after a head whose list mode left the input).
enum class Part { kAll, kHead, kTail };

int launch_preprocess(Workspace& w, const float* pts, uint32_t n, bool stats, int32_t* fin_idx,
                      int32_t* fin_count, bool fused = false, Part part = Part::kAll, bool* listed = nullptr)
{
    hipStream_t s = w.stream;
    const ch_tuning tu = tuning_for(n);
    const uint32_t head = (reinterpret_cast<uintptr_t>(pts) & 15u) ? 1u : 0u;
    const StreamShape sh = stream_shape(n, head, (uint32_t)tu.stream_grid, (uint32_t)tu.stream_unroll);
    // from k_sample until k_cand is queued, a failure leaves the sample
    // table filled
    struct StabGuard {
        bool armed = false;
        ~StabGuard()
        {
            if (armed) g_stab_dirty.store(true, std::memory_order_relaxed);
        }
    } guard;
    const int32_t* gate = nullptr;
    if (part != Part::kTail) {
        CH_TRY(record(w, 0));
        // small inputs (fused, with a device finish): every step in one
        // workgroup of the batched kernel; the kernels below do their work only
        // if it leaves kBatchRedo in the count (gate)
        if (fused && fin_idx) {
            const uint32_t pts_odd = (uint32_t)((reinterpret_cast<uintptr_t>(pts) >> 3) & 1u);
            auto kern = tu.batch_unroll == 1 ? k_batch_hull<1> : k_batch_hull<2>;
            CH_LAUNCH(hipLaunchKernelGGL(kern, dim3(1), dim3(kBatchBlock), 0, s, pts, nullptr, nullptr, fin_idx, fin_count,
                                         pts_odd, 1, (int64_t)n, ListSrc{}));
            gate = fin_count;
        }
        if (g_stab_dirty.load(std::memory_order_relaxed)) {
            // a call failed between k_sample and k_cand somewhere: clear this
            // workspace's sample table before it is used (a fill kernel, not a
            // memset, so that a capture records a kernel node)
            CH_LAUNCH(hipLaunchKernelGGL(k_fill_u32, dim3(kStabWords / kBlock), dim3(kBlock), 0, s, w.stab, 0u,
                                         (uint32_t)kStabWords));
        }
        guard.armed = true;
        // a small input: each k_stream workgroup samples it itself
        const bool own = n > 0 && n <= kSelfSampleMax;
        if (!own) {
            // one run of kBlock * kSamplePerThread points per 8 such runs of
            // the input, from 8 to kSampleBlocks runs
            const uint32_t sblocks = (uint32_t)std::min<uint64_t>(
                kSampleBlocks, std::max<uint64_t>(8, (uint64_t)n / (8ull * kBlock * kSamplePerThread)));
            const uint64_t total = (uint64_t)sblocks * kBlock * kSamplePerThread;
            const uint32_t runs = n >= total ? 1u : 0u;
            const uint32_t step =
                runs && sblocks > 1 ? (uint32_t)((n - (uint64_t)kBlock * kSamplePerThread) / (sblocks - 1)) : 0u;
            const uint64_t mul = runs ? 0ull : ((uint64_t)n << 32) / total;
            CH_LAUNCH(hipLaunchKernelGGL(k_sample, dim3(sblocks), dim3(kBlock), 0, s, pts, n, runs, step, mul, w.stab,
                                         gate));
        }
        CH_TRY(record(w, 1));
        const uint64_t smul = own && n > (uint32_t)kBlock ? ((uint64_t)(n - kBlock) << 32) / (kSamplePerThread - 1) : 0ull;
        auto kstream = tu.stream_unroll == 2 ? (own ? k_stream<2, true> : k_stream<2, false>)
                                             : (own ? k_stream<4, true> : k_stream<4, false>);
        CH_LAUNCH(hipLaunchKernelGGL(kstream, dim3(sh.grid), dim3(kBlock), 0, s, pts, n, head, w.stab, w.part,
                                     w.open_idx, w.open_xym, sh.per, sh.region, w.wgcount, smul, gate));
        CH_TRY(record(w, 2));
        if (fin_idx && !gate && tu.list_max > 0) {
            // few open points: every later step in one workgroup (the batched
            // kernel's list mode, which also clears the sample table); the
            // kernels below run only if it leaves the input (gate)
            const uint32_t pts_odd = (uint32_t)((reinterpret_cast<uintptr_t>(pts) >> 3) & 1u);
            auto kern = tu.batch_unroll == 1 ? k_batch_hull<1, true> : k_batch_hull<2, true>;
            CH_LAUNCH(hipLaunchKernelGGL(kern, dim3(1), dim3(kBatchBlock), 0, s, pts, nullptr, nullptr, fin_idx, fin_count,
                                         pts_odd, 1, (int64_t)n,
                                         ListSrc{w.open_idx, w.open_xym, w.wgcount, w.part, w.h_hdr_dev, w.stab, sh.region, sh.grid,
                                                 (uint32_t)tu.list_max}));
            gate = fin_count;
            if (part == Part::kHead) {
                // the caller waits for its count and queues the tail only if it
                // left the input (the tail's k_cand then clears the table)
                guard.armed = false;
                if (listed) *listed = true;
                for (int k = 3; k <= 6; ++k) CH_TRY(record(w, k));
                return CH_OK;
            }
        }
        if (listed) *listed = false;
    } else {
        guard.armed = true;  // (the head's list mode may not have cleared the table)
    }
    // the rows of the bucket table follow the open count (k_stream's, on the
    // device): up to one k_cand workgroup per cand_per_row open points
    const uint32_t gc = std::min<uint32_t>(kCandMaxRows, sh.grid);
    const uint32_t per_row = (uint32_t)tu.cand_per_row;
    CH_LAUNCH(hipLaunchKernelGGL(k_cand, dim3(gc), dim3(kCandBlock), 0, s, w.hdr, w.stab, w.part, w.open_idx, w.open_xym, sh.region,
                                 w.wgcount, sh.grid, per_row, w.key[0], w.val[0], w.key[1], w.val[1], w.rowoff,
                                 w.rowmin, gate));
    guard.armed = false;
    if (stats) {
        const uint32_t gr = std::max<uint32_t>(1u, std::min<uint32_t>(256u, (n + kBlock * 8 - 1) / (kBlock * 8)));
        CH_LAUNCH(hipLaunchKernelGGL(k_count_regions, dim3(gr), dim3(kBlock), 0, s, pts, n, w.hdr));
    }
    CH_TRY(record(w, 3));
    // the bucket table's columns -> bucket sizes, starts and thresholds;
    // then SPA per bucket, its records gathered from the rows' parts
    CH_LAUNCH(hipLaunchKernelGGL(k_scan, dim3(kScanGrid), dim3(kBlock), 0, s, w.hdr, w.rowoff, w.rowmin, sh.grid,
                                 per_row, w.bk, gate));
    CH_TRY(record(w, 4));
    CH_LAUNCH(hipLaunchKernelGGL(k_bucket_spa, dim3(kBuckets / kBucketsPerSpa), dim3(kBlock), 0, s, w.key[1],
                                 w.val[1], sh.region, sh.grid, per_row, w.rowoff, w.hdr, w.bk, w.dev_chain, gate));
    // hull2d (fin_idx) leaves the host chain buffer alone: its host finish
    // reads k_gather's polygon
    const uint32_t gch = (uint32_t)std::min<size_t>((size_t)tu.chain_grid, (n + kSeg - 1) / kSeg);
    CH_LAUNCH(hipLaunchKernelGGL(k_chain, dim3(gch), dim3(kBlock), 0, s, w.dev_chain, w.hdr, w.bk,
                                 fin_idx ? nullptr : w.h_chain_dev, (uint32_t)w.h_chain_cap, w.dev_spill,
                                 fin_idx ? nullptr : w.h_segcnt_dev, w.h_hdr_dev, stats ? 0 : 1, w.dev_kept,
                                 w.dev_segcnt, gate));
    CH_TRY(record(w, 5));
    if (fin_idx) {
        // items: four extreme points and at most one piece per segment and
        // region (each region adds at most one segment boundary)
        const size_t items = 7 + ((size_t)n + kSeg - 1) / kSeg;
        const uint32_t gw = (uint32_t)std::min<size_t>((size_t)tu.wide_grid, items);
        CH_LAUNCH(hipLaunchKernelGGL(k_finish_wide, dim3(gw), dim3(kWideBlock), 0, s, w.hdr, w.dev_segcnt,
                                     w.dev_kept, w.states, fin_idx, fin_count, w.h_hdr_dev, gate));
    }
    CH_TRY(record(w, 6));
    return CH_OK;
}

constexpr int64_t kWaitListMax = 1 << 20;

// hull2d's head: the launches through k_stream and the list mode, waited
// for; *count receives the list mode's count (kBatchRedo: the tail must
// run).  *listed is false when the list mode is off.
int run_listed(Workspace& w, const float* pts, uint32_t n, int32_t* out_idx, int32_t* out_count, bool* listed,
               int32_t* count)
{
    *listed = false;
    CH_TRY(launch_preprocess(w, pts, n, false, out_idx, out_count, false, Part::kHead, listed));
    if (!*listed) return CH_OK;  // (everything was queued: the caller waits as usual)
    CH_TRY(hipMemcpyAsync(&w.h_hdr->list_count, out_count, sizeof(int32_t), hipMemcpyDeviceToHost, w.stream));
    CH_TRY(hipStreamSynchronize(w.stream));
    *count = w.h_hdr->list_count;
    return CH_OK;
}

// The small-input path of hull2d: the batched kernel on the one set,
// waited for; *count receives its count (the hull size, a negative status,
// or kBatchRedo for a set it leaves to the single-hull path).  Timing
// events 0 and 5 bracket it (the whole hull), 6 follows at once.
int run_fused(Workspace& w, const float* pts, uint32_t n, int32_t* out_idx, int32_t* out_count, int32_t* count)
{
    const ch_tuning tu = tuning_for(n);
    CH_TRY(record(w, 0));
    const uint32_t pts_odd = (uint32_t)((reinterpret_cast<uintptr_t>(pts) >> 3) & 1u);
    auto kern = tu.batch_unroll == 1 ? k_batch_hull<1> : k_batch_hull<2>;
    CH_LAUNCH(hipLaunchKernelGGL(kern, dim3(1), dim3(kBatchBlock), 0, w.stream, pts, nullptr, nullptr, out_idx,
                                 out_count, pts_odd, 1, (int64_t)n, ListSrc{}));
    CH_TRY(record(w, 5));
    CH_TRY(record(w, 6));
    CH_TRY(hipMemcpyAsync(&w.h_hdr->fin_hull, out_count, sizeof(int32_t), hipMemcpyDeviceToHost, w.stream));
    CH_TRY(hipStreamSynchronize(w.stream));
    *count = w.h_hdr->fin_hull;
    return CH_OK;
}

// Statistics of a hull the small-input path computed: the stage counts are
// not kept (-1), the timing spans are the batched kernel's.
void fill_fused_stats(const Workspace& w, int64_t n, int32_t hull, ch_stats* st)
{
    std::memset(st, 0, sizeof(*st));
    st->n = n;
    for (int e = 0; e < 4; ++e) {
        st->ext_idx[e] = -1;
        st->s1[e] = -1;
        st->s2[e] = -1;
    }
    st->open = -1;
    st->candidates = -1;
    st->polygon = -1;
    st->hull = hull;
    st->device_finish = 1;
    st->fused = 1;
    if (g_timing && w.events) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, w.ev[0], w.ev[5]) == hipSuccess) st->ms_pre = ms;
    }
}

int run_preprocess(Workspace& w, const float* pts, uint32_t n, bool stats, int32_t* fin_idx = nullptr,
                   int32_t* fin_count = nullptr, Part part = Part::kAll)
{
    CH_TRY(launch_preprocess(w, pts, n, stats, fin_idx, fin_count, false, part));
    CH_TRY(hipStreamSynchronize(w.stream));
    if (w.h_hdr->err & kErrDomain) return CH_EDOMAIN;
    if (w.h_hdr->err) return CH_EHIP;
    if (fin_idx) return CH_OK;  // the hull is written, or k_gather's turn
    // kept chain points sit below the chain length
    const size_t m = w.h_hdr->chain;
    w.spill.clear();
    if (m > w.h_chain_cap) {
        w.spill.resize(m - w.h_chain_cap);
        CH_TRY(hipMemcpy(w.spill.data(), w.dev_spill, sizeof(PolyRec) * w.spill.size(), hipMemcpyDeviceToHost));
        // the next call's chain of this size lands in pinned memory whole
        size_t want = w.h_chain_cap;
        while (want < m && want < kHostChainMax) want *= 2;
        w.h_chain_want = want;
    }
    return CH_OK;
}

inline const PolyRec& chain_at(const Workspace& w, size_t i)
{
    return i < w.h_chain_cap ? w.h_chain[i] : w.spill[i - w.h_chain_cap];
}

// The simple polygon [P_minx, R1, P_miny, R2, P_maxx, R3, P_maxy, R4] with
// consecutive coincident vertices dropped (cyclically), into w.xy / w.idx:
// each region's chain is its buckets' survivors in bucket order.
void build_polygon(Workspace& w)
{
    const DevHeader& h = *w.h_hdr;
    w.xy.clear();
    w.idx.clear();
    auto push = [&](int32_t idx, int32_t x, int32_t y) {
        const size_t k = w.idx.size();
        if (k && w.xy[2 * k - 2] == x && w.xy[2 * k - 1] == y) return;
        w.idx.push_back(idx);
        w.xy.push_back(x);
        w.xy.push_back(y);
    };
    int cur = -1;  // regions whose extreme point is in
    auto enter = [&](int q) {
        while (cur < q) {
            ++cur;
            push((int32_t)h.ext_idx[cur], (int32_t)h.ext_x[cur], (int32_t)h.ext_y[cur]);
        }
    };
    for (int q = 0; q < 4; ++q) w.w2[q] = 0;
    const size_t nseg = ((size_t)h.chain + kSeg - 1) / kSeg;
    for (size_t sg = 0; sg < nseg; ++sg) {
        size_t at = sg * kSeg;
        for (int q = 0; q < 4; ++q) {
            const uint32_t c = w.h_segcnt[4 * sg + q];
            if (!c) continue;
            enter(q);
            for (uint32_t r = 0; r < c; ++r, ++at) {
                const PolyRec& rec = chain_at(w, at);
                push(rec.idx, rec.x, rec.y);
            }
            w.w2[q] += c;
        }
    }
    enter(3);
    for (int q = 0; q < 4; ++q) w.s2[q] = h.s2[q];
    w.chain = h.chain;
    while (w.idx.size() > 1 && w.xy[2 * w.idx.size() - 2] == w.xy[0] && w.xy[2 * w.idx.size() - 1] == w.xy[1]) {
        w.idx.pop_back();
        w.xy.pop_back();
        w.xy.pop_back();
    }
}

void fill_stats(const Workspace& w, int64_t n, ch_stats* st, bool stats)
{
    std::memset(st, 0, sizeof(*st));
    st->n = n;
    if (n == 0) return;
    const DevHeader& h = *w.h_hdr;
    for (int e = 0; e < 4; ++e) {
        st->ext_idx[e] = (int32_t)h.ext_idx[e];
        st->ext_xy[2 * e] = (int32_t)h.ext_x[e];
        st->ext_xy[2 * e + 1] = (int32_t)h.ext_y[e];
        st->s1[e] = stats ? (int64_t)h.s1[e] : -1;
        st->s2[e] = w.s2[e];
    }
    st->open = h.open;
    st->candidates = h.cand;
    st->polygon = w.w2[0] + w.w2[1] + w.w2[2] + w.w2[3] + 4;
    if (g_timing && w.events) {
        // stage slots: 0 sample + staircases, 1 k_stream, 2 k_cand, 3 sort,
        // 4 SPA + chains, 5 device finish (6 and 7, the host finish, are
        // wall-clock times set by the caller); steps 1-6 and the finish as
        // single spans in either mode
        if (g_timing == 1) {
            for (int k = 0; k < 6; ++k) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, w.ev[k], w.ev[k + 1]) == hipSuccess) st->ms[k] = ms;
            }
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, w.ev[0], w.ev[5]) == hipSuccess) st->ms_pre = ms;
        if (hipEventElapsedTime(&ms, w.ev[5], w.ev[6]) == hipSuccess) st->ms_finish = ms;
    }
}

// After run_preprocess with fin_idx left the finish to the host: the
// polygon, gathered on the device into pinned memory (w.h_pxy, w.h_pidx;
// its size returned in *m), and the per-region counts for the statistics.
int gather_polygon(Workspace& w, size_t* m)
{
    const size_t need = (size_t)w.h_hdr->chain + 4;  // at least the polygon
    if (w.h_poly_cap < need) {
        if (w.h_pxy) CH_TRY(hipHostFree(w.h_pxy));
        if (w.h_pidx) CH_TRY(hipHostFree(w.h_pidx));
        w.h_pxy = w.h_pidx = nullptr;
        w.h_poly_cap = 0;
        size_t cap = 4096;
        while (cap < need) cap *= 2;
        CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_pxy), sizeof(int32_t) * 2 * cap, hipHostMallocMapped));
        CH_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&w.h_pxy_dev), w.h_pxy, 0));
        CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_pidx), sizeof(int32_t) * cap, hipHostMallocMapped));
        CH_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&w.h_pidx_dev), w.h_pidx, 0));
        w.h_poly_cap = cap;
    }
    const uint32_t cap32 = (uint32_t)std::min<size_t>(w.h_poly_cap, UINT32_MAX);
    CH_LAUNCH(hipLaunchKernelGGL(k_gather, dim3(1), dim3(kBatchBlock), 0, w.stream, w.hdr, w.dev_segcnt,
                                 w.dev_kept, w.h_pxy_dev, w.h_pidx_dev, cap32, w.h_hdr_dev));
    CH_TRY(hipStreamSynchronize(w.stream));
    const DevHeader& h = *w.h_hdr;
    if (h.gat_count < 4 || h.gat_count > w.h_poly_cap) return CH_EHIP;
    for (int q = 0; q < 4; ++q) {
        w.w2[q] = h.fin_w2[q];
        w.s2[q] = h.s2[q];
    }
    w.chain = h.chain;
    *m = h.gat_count;
    return CH_OK;
}

int hull_one(const float* points, int64_t n, int32_t* out_idx, int32_t* out_count, hipStream_t stream)
{
    ch_stats& st = t_stats;
    std::memset(&st, 0, sizeof(st));
    st.n = n;
    if (n < 0 || n > INT32_MAX || !out_count || (n > 0 && (!points || !out_idx))) return CH_EINVAL;
    if (reinterpret_cast<uintptr_t>(points) & 7u) return CH_EINVAL;
    int rc = CH_OK;
    Workspace* w = workspace_for(stream, &rc);
    if (!w) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    if (n == 0) {
        // no host buffer: a copy from an earlier call may still read it
        CH_TRY(hipMemsetAsync(out_count, 0, sizeof(int32_t), stream));
        return CH_OK;
    }
    CH_TRY(ensure_device(*w, (size_t)n));
    CH_TRY(ensure_host(*w, 0, false));
    if (n <= (int64_t)tuning_for(n).fused_max) {
        // small input: every step in one workgroup of the batched kernel;
        // only a set it leaves (kBatchRedo) takes the single-hull path below
        int32_t c = 0;
        CH_TRY(run_fused(*w, points, (uint32_t)n, out_idx, out_count, &c));
        if (c != kBatchRedo) {
            if (c < 0) {
                (void)hipMemsetAsync(out_count, 0, sizeof(int32_t), stream);
                return c == CH_EDOMAIN ? CH_EDOMAIN : CH_EHIP;
            }
            fill_fused_stats(*w, n, c, &st);
            return CH_OK;
        }
    }
    // up to kWaitListMax points: the head, waited for, then (only if the
    // list mode left the input) the tail, so that a call with few open
    // points queues no tail kernels; larger inputs, which seldom leave few
    // open points, queue everything at once (the tail gated on the device)
    bool listed = false;
    int32_t lc = 0;
    if (n <= kWaitListMax) {
        CH_TRY(run_listed(*w, points, (uint32_t)n, out_idx, out_count, &listed, &lc));
    } else {
        CH_TRY(launch_preprocess(*w, points, (uint32_t)n, false, out_idx, out_count));
    }
    if (listed && lc != kBatchRedo) {
        if (lc < 0) {
            (void)hipMemsetAsync(out_count, 0, sizeof(int32_t), stream);
            return lc == CH_EDOMAIN ? CH_EDOMAIN : CH_EHIP;
        }
        // the list mode published the header's counts
        for (int q = 0; q < 4; ++q) {
            w->w2[q] = w->h_hdr->fin_w2[q];
            w->s2[q] = w->h_hdr->s2[q];
        }
        w->chain = w->h_hdr->chain;
        fill_stats(*w, n, &st, false);
        st.hull = lc;
        st.device_finish = 1;
        return CH_OK;
    }
    if (listed) {
        rc = run_preprocess(*w, points, (uint32_t)n, false, out_idx, out_count, Part::kTail);
    } else {
        CH_TRY(hipStreamSynchronize(stream));  // (the head queued every kernel)
        rc = w->h_hdr->err & kErrDomain ? CH_EDOMAIN : w->h_hdr->err ? CH_EHIP : CH_OK;
    }
    if (rc == CH_OK && w->h_hdr->fin_done && !w->h_hdr->fin_fail) {
        // finished on the device: the hull is in out_idx / out_count
        for (int q = 0; q < 4; ++q) {
            w->w2[q] = w->h_hdr->fin_w2[q];
            w->s2[q] = w->h_hdr->s2[q];
        }
        w->chain = w->h_hdr->chain;
        fill_stats(*w, n, &st, false);
        st.hull = w->h_hdr->fin_hull;
        st.device_finish = 1;
        return CH_OK;
    }
    int64_t h = 0;
    if (rc == CH_OK) {
        const auto t0 = std::chrono::steady_clock::now();
        size_t m = 0;
        rc = gather_polygon(*w, &m);
        const auto t1 = std::chrono::steady_clock::now();
        if (rc == CH_OK) {
            fill_stats(*w, n, &st, false);
            rc = ensure_host(*w, m, false);
        }
        if (rc == CH_OK) {
            rc = melkman_finish(w->h_pxy, w->h_pidx, (int64_t)m, w->h_out + 1, &h) == 0 ? CH_OK : CH_EHIP;
        }
        const auto t2 = std::chrono::steady_clock::now();
        st.ms[6] = std::chrono::duration<float, std::milli>(t1 - t0).count();
        st.ms[7] = std::chrono::duration<float, std::milli>(t2 - t1).count();
        st.hull = h;
    }
    if (rc != CH_OK) {
        // the call may have failed before its mid-call synchronisation
        (void)hipStreamSynchronize(stream);
        (void)hipMemsetAsync(out_count, 0, sizeof(int32_t), stream);
        return rc;
    }
    // Stream-ordered results: the pinned buffer is rewritten only after the
    // next call's synchronisation on this stream, which follows these copies.
    w->h_out[0] = (int32_t)h;
    const uint32_t g = (uint32_t)std::max<int64_t>(1, (h + kBlock - 1) / kBlock);
    CH_LAUNCH(hipLaunchKernelGGL(k_put_result, dim3(g), dim3(kBlock), 0, stream, w->h_out_dev + 1, (int32_t)h,
                                 out_idx, out_count));
    return CH_OK;
}


// hull2d_noalloc: the device address of the fixed buffer, looked up once per
// device with that device current.
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_base[kNoAllocDevices] = {};

int noalloc_base(int dev, char** base)
{
    if (dev < 0 || dev >= kNoAllocDevices) return CH_EHIP;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_base[dev]) {
        void* p = nullptr;
        CH_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch)));
        if (!p) return CH_EHIP;
        g_noalloc_base[dev] = static_cast<char*>(p);
    }
    *base = g_noalloc_base[dev];
    return CH_OK;
}

// What hull2d_noalloc needs of the buffer for n points: the workspace
// layout for n, then a device-side stand-in for the pinned header (k_chain
// and k_finish write it; nobody reads it).
size_t noalloc_bytes(size_t n) { return device_bytes(n) + align_up(sizeof(DevHeader), 256); }

}  // namespace
}  // namespace chainhull

using namespace chainhull;

extern "C" {

int hull2d(const float* points, int64_t n, int32_t* out_idx, int32_t* out_count, void* stream)
{
    return hull_one(points, n, out_idx, out_count, reinterpret_cast<hipStream_t>(stream));
}

int hull2d_async(const float* points, int64_t n, int32_t* out_idx, int32_t* out_count, void* stream)
{
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (n < 0 || n > INT32_MAX || !out_count || (n > 0 && (!points || !out_idx))) return CH_EINVAL;
    if (reinterpret_cast<uintptr_t>(points) & 7u) return CH_EINVAL;
    if (n == 0) {  // a kernel, not a memset: the call may be captured in a graph
        CH_LAUNCH(hipLaunchKernelGGL(k_put_result, dim3(1), dim3(kBlock), 0, s, nullptr, 0, out_idx, out_count));
        return CH_OK;
    }
    int rc = CH_OK;
    Workspace* w = workspace_for(s, &rc);
    if (!w) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    CH_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone && (!w->dbuf || w->cap < (size_t)n)) return CH_EINVAL;  // no allocation under capture
    CH_TRY(ensure_device(*w, (size_t)n));
    CH_TRY(ensure_host(*w, 0, false));
    if (cs == hipStreamCaptureStatusActive) w->captured = true;
    const bool fused = n <= (int64_t)tuning_for(n).fused_max;
    return launch_preprocess(*w, points, (uint32_t)n, false, out_idx, out_count, fused);
}

int hull2d_noalloc(const float* points, int64_t n, int32_t* out_idx, int32_t* out_count, void* stream)
{
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (n < 0 || n > INT32_MAX || !out_count || (n > 0 && (!points || !out_idx))) return CH_EINVAL;
    if (reinterpret_cast<uintptr_t>(points) & 7u) return CH_EINVAL;
    if (n > (int64_t)CH_NOALLOC_MAX_POINTS) return CH_ECAPACITY;
    if (n == 0) {
        CH_LAUNCH(hipLaunchKernelGGL(k_put_result, dim3(1), dim3(kBlock), 0, s, nullptr, 0, out_idx, out_count));
        return CH_OK;
    }
    // the whole layout for the largest call must fit the buffer
    if (noalloc_bytes(CH_NOALLOC_MAX_POINTS) > CH_NOALLOC_SCRATCH_BYTES) return CH_EHIP;
    int dev = 0;
    CH_TRY(hipGetDevice(&dev));
    char* base = nullptr;
    CH_TRY(noalloc_base(dev, &base));
    // a view of the buffer (no allocation): the workspace layout, the
    // header stand-in after it
    Workspace w;
    w.device = dev;
    w.stream = s;
    w.no_events = true;
    w.cap = (size_t)CH_NOALLOC_MAX_POINTS;
    // (the layout of the largest call, so that every array, the look-back
    // states among them, sits at the same place in every call)
    const size_t used = layout(&w, base, (size_t)CH_NOALLOC_MAX_POINTS);
    w.h_hdr_dev = reinterpret_cast<DevHeader*>(base + used);
    const bool fused = n <= (int64_t)tuning_for(n).fused_max;
    return launch_preprocess(w, points, (uint32_t)n, false, out_idx, out_count, fused);
}

int hull2d_batched(const float* points, const int64_t* offsets, int32_t num_sets, int32_t* out_idx,
                   int32_t* out_counts, void* stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    ch_batch_stats& bs = t_bstats;
    std::memset(&bs, 0, sizeof(bs));
    bs.num_sets = num_sets;
    if (num_sets < 0 || (num_sets > 0 && (!offsets || !out_counts))) return CH_EINVAL;
    if (num_sets == 0) return CH_OK;
    if (offsets[0] != 0) return CH_EINVAL;
    for (int32_t s = 0; s < num_sets; ++s) {
        if (offsets[s + 1] < offsets[s] || offsets[s + 1] > INT32_MAX) return CH_EINVAL;
    }
    if (offsets[num_sets] > 0 && (!points || !out_idx)) return CH_EINVAL;
    if (reinterpret_cast<uintptr_t>(points) & 7u) return CH_EINVAL;
    bs.points = offsets[num_sets];
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int rc = CH_OK;
    Workspace* w = workspace_for(st, &rc);
    if (!w) return rc;
    std::vector<int32_t> redo;
    {
        std::lock_guard<std::mutex> lk(w->mu);
        const size_t ns = (size_t)num_sets;
        if (w->b_cap < ns) {
            CH_TRY(hipStreamSynchronize(st));
            if (w->b_offsets) CH_TRY(hipFree(w->b_offsets));
            if (w->b_order) CH_TRY(hipFree(w->b_order));
            if (w->h_b_offsets) CH_TRY(hipHostFree(w->h_b_offsets));
            if (w->h_b_order) CH_TRY(hipHostFree(w->h_b_order));
            if (w->h_b_counts) CH_TRY(hipHostFree(w->h_b_counts));
            w->b_offsets = nullptr;
            w->b_order = nullptr;
            w->h_b_offsets = nullptr;
            w->h_b_order = nullptr;
            w->h_b_counts = nullptr;
            w->b_cap = 0;
            const size_t cap = std::max<size_t>(ns, 1024);
            CH_TRY(hipMalloc(reinterpret_cast<void**>(&w->b_offsets), sizeof(int64_t) * (cap + 1)));
            CH_TRY(hipMalloc(reinterpret_cast<void**>(&w->b_order), sizeof(int32_t) * cap));
            CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->h_b_offsets), sizeof(int64_t) * (cap + 1),
                                 hipHostMallocDefault));
            CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->h_b_order), sizeof(int32_t) * cap, hipHostMallocDefault));
            CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w->h_b_counts), sizeof(int32_t) * cap,
                                 hipHostMallocDefault));
            w->b_cap = cap;
        }
        // the staging buffers may still feed an earlier call's copies
        CH_TRY(hipStreamSynchronize(st));
        std::memcpy(w->h_b_offsets, offsets, sizeof(int64_t) * (ns + 1));
        // the kernel takes the sets up to kBatchMaxSet points, larger ones
        // first so that the last workgroups to start are short
        int32_t nk = 0;
        for (int32_t s = 0; s < num_sets; ++s) {
            if (offsets[s + 1] - offsets[s] <= kBatchMaxSet) w->h_b_order[nk++] = s;
        }
        const ch_tuning tu = tuning_for(offsets[num_sets]);
        if (tu.batch_order == 0) {
            std::stable_sort(w->h_b_order, w->h_b_order + nk, [&](int32_t a, int32_t b) {
                return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
            });
        }
        bs.device_sets = nk;
        if (nk > 0) {
            CH_TRY(hipMemcpyAsync(w->b_offsets, w->h_b_offsets, sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice,
                                  st));
            CH_TRY(hipMemcpyAsync(w->b_order, w->h_b_order, sizeof(int32_t) * (size_t)nk, hipMemcpyHostToDevice, st));
            CH_TRY(record(*w, 0));
            const uint32_t pts_odd = (uint32_t)((reinterpret_cast<uintptr_t>(points) >> 3) & 1u);
            auto kern = tu.batch_unroll == 1 ? k_batch_hull<1> : k_batch_hull<2>;
            CH_LAUNCH(hipLaunchKernelGGL(kern, dim3((uint32_t)nk), dim3(kBatchBlock), 0, st, points,
                                         w->b_offsets, w->b_order, out_idx, out_counts, pts_odd, num_sets,
                                         (int64_t)0, ListSrc{}));
            CH_TRY(record(*w, 1));
            CH_TRY(hipMemcpyAsync(w->h_b_counts, out_counts, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
        }
        CH_TRY(hipStreamSynchronize(st));
        if (g_timing && w->events && nk > 0) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, w->ev[0], w->ev[1]) == hipSuccess) bs.ms_kernel = ms;
        }
        for (int32_t s = 0; s < num_sets; ++s) {
            if (offsets[s + 1] - offsets[s] > kBatchMaxSet) w->h_b_counts[s] = kBatchRedo;
            if (w->h_b_counts[s] == kBatchRedo) redo.push_back(s);
        }
    }
    int first_err = CH_OK;
    for (int32_t s = 0; s < num_sets; ++s) {
        const int32_t c = w->h_b_counts[s];
        if (c < 0 && c != kBatchRedo && first_err == CH_OK) first_err = c;
    }
    // sets beyond the kernel's limit or capacities: the single-hull path
    bs.redo_sets = (int32_t)redo.size();
    for (const int32_t s : redo) {
        const int64_t lo = offsets[s], m = offsets[s + 1] - lo;
        const int r = hull_one(points + 2 * lo, m, out_idx + lo, out_counts + s, st);
        if (r != CH_OK) {
            // hull_one leaves the stream usable and has set the count to 0;
            // the set's own status replaces it, in stream order
            int32_t* code = w->h_b_counts + s;
            *code = r;
            CH_TRY(hipMemcpyAsync(out_counts + s, code, sizeof(int32_t), hipMemcpyHostToDevice, st));
            CH_TRY(hipStreamSynchronize(st));
            if (first_err == CH_OK) first_err = r;
        }
    }
    bs.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return first_err;
}

int hull2d_batched_async(const float* points, const int64_t* offsets, const int32_t* order, int32_t num_sets,
                         int32_t* out_idx, int32_t* out_counts, void* stream)
{
    if (num_sets < 0 || (num_sets > 0 && (!offsets || !out_counts || !points || !out_idx))) return CH_EINVAL;
    if (reinterpret_cast<uintptr_t>(points) & 7u) return CH_EINVAL;
    if (num_sets == 0) return CH_OK;
    const uint32_t pts_odd = (uint32_t)((reinterpret_cast<uintptr_t>(points) >> 3) & 1u);
    const ch_tuning tu = tuning_for(INT64_MAX);
    auto kern = tu.batch_unroll == 1 ? k_batch_hull<1> : k_batch_hull<2>;
    CH_LAUNCH(hipLaunchKernelGGL(kern, dim3((uint32_t)num_sets), dim3(kBatchBlock), 0,
                                 reinterpret_cast<hipStream_t>(stream), points, offsets, order, out_idx, out_counts,
                                 pts_odd, num_sets, (int64_t)0, ListSrc{}));
    return CH_OK;
}

int chainhull_polygon(const float* points, int64_t n, int32_t* poly_idx, int64_t* poly_count, ch_stats* stats,
                      void* stream)
{
    ch_stats& st = t_stats;
    std::memset(&st, 0, sizeof(st));
    st.n = n;
    if (poly_count) *poly_count = 0;
    if (n < 0 || n > INT32_MAX || !poly_count || (n > 0 && (!points || !poly_idx))) return CH_EINVAL;
    if (reinterpret_cast<uintptr_t>(points) & 7u) return CH_EINVAL;
    if (n == 0) {
        if (stats) *stats = st;
        return CH_OK;
    }
    int rc = CH_OK;
    Workspace* w = workspace_for(reinterpret_cast<hipStream_t>(stream), &rc);
    if (!w) return rc;
    std::lock_guard<std::mutex> lk(w->mu);
    CH_TRY(ensure_device(*w, (size_t)n));
    CH_TRY(ensure_host(*w, 0, true));  // after the device part: sized by its capacity
    rc = run_preprocess(*w, points, (uint32_t)n, true);
    if (rc != CH_OK) return rc;
    build_polygon(*w);
    fill_stats(*w, n, &st, true);
    for (size_t i = 0; i < w->idx.size(); ++i) poly_idx[i] = w->idx[i];
    *poly_count = (int64_t)w->idx.size();
    if (stats) *stats = st;
    return CH_OK;
}

int chainhull_finish_host(const int32_t* poly_xy, const int32_t* poly_idx, int64_t m, int32_t* out_idx,
                          int64_t* out_count)
{
    if (out_count) *out_count = 0;
    if (m < 0 || !out_count || (m > 0 && (!poly_xy || !poly_idx || !out_idx))) return CH_EINVAL;
    return melkman_finish(poly_xy, poly_idx, m, out_idx, out_count) == 0 ? CH_OK : CH_EINVAL;
}

int chainhull_last_batch_stats(ch_batch_stats* out)
{
    if (!out) return CH_EINVAL;
    *out = t_bstats;
    return CH_OK;
}

int chainhull_last_stats(ch_stats* out)
{
    if (!out) return CH_EINVAL;
    *out = t_stats;
    return CH_OK;
}

void chainhull_set_timing(int enable) { g_timing = enable == 2 ? 2 : (enable != 0 ? 1 : 0); }

const char* chainhull_strerror(int status)
{
    switch (status) {
    case CH_OK: return "success";
    case CH_EINVAL: return "invalid argument";
    case CH_EDOMAIN: return "a coordinate is not an integer in [0, 2^23)";
    case CH_ENOMEM: return "out of memory";
    case CH_EHIP: return "HIP runtime error";
    case CH_EADMIT: return "request not admitted";
    case CH_ECAPACITY: return "more points than the fixed buffer of hull2d_noalloc holds";
    default: return "unknown status";
    }
}

void chainhull_release(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_ws) free_workspace(kv.second);
    g_ws.clear();
}

int chainhull_spa_chunked(const uint32_t* k2_sorted, int64_t m, uint32_t sigma, int64_t chunk, uint8_t* keep,
                          void* stream)
{
    if (m < 0 || m > INT32_MAX || chunk < 1 || (m > 0 && (!k2_sorted || !keep))) return CH_EINVAL;
    if (m == 0) return CH_OK;
    const int64_t subsets = (m + chunk - 1) / chunk;
    const uint32_t grid = (uint32_t)((subsets + kBlock - 1) / kBlock);
    const uint32_t c = (uint32_t)std::min<int64_t>(chunk, m);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CH_LAUNCH(hipLaunchKernelGGL(k_spa_chunked, dim3(grid), dim3(kBlock), 0, st, k2_sorted, (uint32_t)m, sigma, c,
                                 keep));
    return CH_OK;
}

int chainhull_release_stream(void* stream)
{
    int dev = 0;
    const int rc = hip_status(hipGetDevice(&dev));
    if (rc != CH_OK) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find(std::make_pair(dev, reinterpret_cast<hipStream_t>(stream)));
    if (it != g_ws.end()) {
        free_workspace(it->second);
        g_ws.erase(it);
    }
    return CH_OK;
}

int chainhull_set_tuning(int64_t n_max, const ch_tuning* t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (n_max < 0) {
        g_tune_count = 0;
        return CH_OK;
    }
    if (!t || !tuning_valid(*t)) return CH_EINVAL;
    for (int k = 0; k < g_tune_count; ++k) {
        if (g_tune_nmax[k] == n_max) {
            g_tune[k] = *t;
            return CH_OK;
        }
    }
    if (g_tune_count >= kTuningClasses) return CH_EINVAL;
    g_tune_nmax[g_tune_count] = n_max;
    g_tune[g_tune_count] = *t;
    ++g_tune_count;
    return CH_OK;
}

int chainhull_get_tuning(int64_t n, ch_tuning* out)
{
    if (!out) return CH_EINVAL;
    *out = n < 0 ? kDefaultTuning : tuning_for(n);
    return CH_OK;
}

#ifdef CH_PHASE_TIMING
// Instrumented builds only (not declared in the public header): the batched
// kernel's phase sums (18 values), read and cleared.
int chainhull_phase_ticks(unsigned long long* out)
{
    if (!out) return CH_EINVAL;
    CH_TRY(hipDeviceSynchronize());
    CH_TRY(hipMemcpyFromSymbol(out, HIP_SYMBOL(chainhull::g_phase_ticks), sizeof(unsigned long long) * 18));
    static const unsigned long long zero[18] = {};
    CH_TRY(hipMemcpyToSymbol(HIP_SYMBOL(chainhull::g_phase_ticks), zero, sizeof(zero)));
    return CH_OK;
}
#endif

size_t chainhull_workspace_bytes(int64_t n)
{
    if (n < 0) return 0;
    return device_bytes(std::max<size_t>((size_t)n, 1u << 16));
}

}  // extern "C"
