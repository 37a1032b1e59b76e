// chainhull: the CudaChain preprocessing path (Section 2.1, steps 1-6) as
// hand-written gfx950 kernels, the pipeline around them and the C ABI.
//
// Data layout in HBM (one workspace per device and stream):
//   points           caller's n x float32[2], read twice (steps 1 and 2)
//   ExtPartial[G1]   per-workgroup lexicographic extreme keys (step 1)
//   DevHeader        extreme points, quadrilateral edges, region frames and
//                    every counter of the call
//   key[2][cap]      u32 sort key  q << 23 | k1       (double buffer)
//   val[2][cap]      u64 payload   k2 << 32 | index   (double buffer)
//   hist[512 * G]    per-chunk digit counts of the region sort
//   spa_part/cnt[4G] per-chunk SPA minima and survivor counts
//   poly[cap + 4]    the simple polygon as (index, x, y) int32 triples
// After the sort the data sits in buffer 1; the SPA survivors are written,
// chunk-local, into buffer 0.
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
// with M = 2^23 - 1.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "chainhull.h"
#include "finish.h"

namespace chainhull {

constexpr uint32_t kM = (1u << 23) - 1;
constexpr int kBlock = 256;        // threads per workgroup (4 waves of 64)
constexpr int kWaves = kBlock / 64;
constexpr int kExtBlocks = 2048;   // workgroups of the extreme-point pass
constexpr int kExtUnroll = 4;      // float4 loads in flight per thread
constexpr int kTilePts = 4096;     // points per classify workgroup
constexpr int kPtsPerThread = kTilePts / kBlock;  // 16
constexpr int kSlotBits = 9;
constexpr int kSlots = 1 << kSlotBits;            // k1 slots per region and tile
constexpr int kSortBlocks = 512;   // chunks of the region sort and of SPA
constexpr int kSortIpt = 8;        // records per thread per sort sub-tile
constexpr int kSortTile = kBlock * kSortIpt;
constexpr int kMaxBins = 512;
constexpr int kSpaIpt = 4;
constexpr int kSpaTile = kBlock * kSpaIpt;

typedef float v2f __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned long long u64;

struct DevHeader {
    double ec[4];        // ex*E_q.y - ey*E_q.x for the edge E_q -> E_{q+1}
    int32_t ex[4], ey[4];
    uint32_t ext_x[4], ext_y[4], ext_idx[4];  // P_minx, P_miny, P_maxx, P_maxy
    uint32_t k1lo[4], k1shift[4], sigma[4];   // per-region frame data
    uint32_t err;        // nonzero: a coordinate is outside the domain
    uint32_t s1[4];      // round-1 survivors per region
    uint32_t cand;       // records written by the tile filter
    uint32_t s2[4];      // SPA survivors per region
    uint32_t poly;       // polygon vertices, the four extreme points included
    uint32_t pad[7];
};

struct ExtPartial {
    u64 key[4];
    uint32_t idx[4];
    uint32_t err;
    uint32_t pad[3];
};

struct PolyRec {
    int32_t idx, x, y;
};

// ---------------------------------------------------------------------------
// Wave and workgroup helpers (wave64)
// ---------------------------------------------------------------------------

__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint32_t sel4(uint32_t q, uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3)
{
    return q == 0 ? a0 : q == 1 ? a1 : q == 2 ? a2 : a3;
}

// Region frame: (k1, k2) of integer point (X, Y) in region q.
__device__ inline uint32_t frame_k1(uint32_t q, uint32_t X, uint32_t Y) { return sel4(q, X, Y, kM - X, kM - Y); }
__device__ inline uint32_t frame_k2(uint32_t q, uint32_t X, uint32_t Y) { return sel4(q, Y, kM - X, kM - Y, X); }

__device__ inline void lexmin_pair(u64& k, uint32_t& i, u64 ok, uint32_t oi)
{
    if (ok < k || (ok == k && oi < i)) {
        k = ok;
        i = oi;
    }
}

__device__ inline void wave_lexmin(u64& k, uint32_t& i)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const u64 ok = __shfl_xor(k, off);
        const uint32_t oi = __shfl_xor(i, off);
        lexmin_pair(k, i, ok, oi);
    }
}

__device__ inline uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ inline uint32_t wave_min(uint32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor(v, off));
    return v;
}

__device__ inline uint32_t wave_incl_sum(uint32_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(v, off);
        if (lane >= (uint32_t)off) v += o;
    }
    return v;
}

__device__ inline uint32_t wave_incl_min(uint32_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(v, off);
        if (lane >= (uint32_t)off) v = min(v, o);
    }
    return v;
}

// Exclusive workgroup sum of one value per thread; `total` gets the sum.
__device__ inline uint32_t block_excl_sum(uint32_t v, uint32_t* scratch, uint32_t& total)
{
    const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
    const uint32_t incl = wave_incl_sum(v);
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t s = scratch[w];
        before += (w < (int)wave) ? s : 0u;
        all += s;
    }
    __syncthreads();
    total = all;
    return before + incl - v;
}

// Exclusive workgroup minimum (identity ~0u); `total` gets the minimum.
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
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t s = scratch[w];
        if (w < (int)wave) before = min(before, s);
        all = min(all, s);
    }
    __syncthreads();
    total = all;
    return min(before, excl);
}

__device__ inline void chunk_range(uint32_t count, uint32_t b, uint32_t nb, uint32_t& lo, uint32_t& hi)
{
    const uint32_t per = (count + nb - 1) / nb;
    lo = min(count, b * per);
    hi = min(count, lo + per);
}

// ---------------------------------------------------------------------------
// Step 1 (Section 2.1 step 1; Section 2.2.1): the four extreme points by a
// parallel reduction, fused with domain validation.  Each extreme minimises
// a 46-bit lexicographic key, then the point index:
//   P_minx  (x, M - y)      P_miny  (y, x)
//   P_maxx  (M - x, y)      P_maxy  (M - y, M - x)
// ---------------------------------------------------------------------------

__device__ inline bool coord_ok(float v) { return v >= 0.0f && v < 8388608.0f && truncf(v) == v; }

struct ExtAcc {
    u64 k[4];
    uint32_t i[4];
    uint32_t bad;
};

__device__ inline void ext_init(ExtAcc& a)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        a.k[e] = ~0ull;
        a.i[e] = ~0u;
    }
    a.bad = 0;
}

// A thread visits its points in increasing index order, so on equal keys the
// first point seen (the smallest index) stays.
__device__ inline void ext_visit(ExtAcc& a, float fx, float fy, uint32_t idx)
{
    const bool ok = coord_ok(fx) && coord_ok(fy);
    a.bad |= ok ? 0u : 1u;
    const uint32_t X = ok ? (uint32_t)fx : 0u;
    const uint32_t Y = ok ? (uint32_t)fy : 0u;
    const u64 k0 = ((u64)X << 23) | (kM - Y);
    const u64 k1 = ((u64)Y << 23) | X;
    const u64 k2 = ((u64)(kM - X) << 23) | Y;
    const u64 k3 = ((u64)(kM - Y) << 23) | (kM - X);
    if (k0 < a.k[0]) { a.k[0] = k0; a.i[0] = idx; }
    if (k1 < a.k[1]) { a.k[1] = k1; a.i[1] = idx; }
    if (k2 < a.k[2]) { a.k[2] = k2; a.i[2] = idx; }
    if (k3 < a.k[3]) { a.k[3] = k3; a.i[3] = idx; }
}

__device__ inline void ext_block_reduce(ExtAcc& a, u64 (*sk)[4], uint32_t (*si)[4], uint32_t* sbad)
{
    const uint32_t wave = threadIdx.x / 64;
#pragma unroll
    for (int e = 0; e < 4; ++e) wave_lexmin(a.k[e], a.i[e]);
    const uint32_t bad = __ballot(a.bad) != 0ull ? 1u : 0u;
    if (lane_id() == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            sk[wave][e] = a.k[e];
            si[wave][e] = a.i[e];
        }
        sbad[wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int e = 0; e < 4; ++e) {
            for (int w = 1; w < kWaves; ++w) lexmin_pair(sk[0][e], si[0][e], sk[w][e], si[w][e]);
        }
        for (int w = 1; w < kWaves; ++w) sbad[0] |= sbad[w];
    }
    __syncthreads();
}

// `head` leading points (0 or 1) are visited singly so that the rest of the
// array is 16-byte aligned for float4 loads; an odd last point likewise.
__global__ __launch_bounds__(kBlock) void k_extremes(const float* __restrict__ pts, uint32_t n, uint32_t head,
                                                     ExtPartial* __restrict__ part)
{
    __shared__ u64 sk[kWaves][4];
    __shared__ uint32_t si[kWaves][4];
    __shared__ uint32_t sbad[kWaves];
    ExtAcc a;
    ext_init(a);
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0 && head) ext_visit(a, pts[0], pts[1], 0);

    const v4f* p4 = reinterpret_cast<const v4f*>(pts + 2 * head);
    const uint32_t n4 = (n - head) / 2;
    const uint32_t stride = gridDim.x * kBlock;
    uint32_t f = blockIdx.x * kBlock + tid;
    for (; f + (kExtUnroll - 1) * stride < n4; f += kExtUnroll * stride) {
        v4f v[kExtUnroll];
#pragma unroll
        for (int u = 0; u < kExtUnroll; ++u) v[u] = p4[f + u * stride];
#pragma unroll
        for (int u = 0; u < kExtUnroll; ++u) {
            const uint32_t i = head + 2 * (f + u * stride);
            ext_visit(a, v[u].x, v[u].y, i);
            ext_visit(a, v[u].z, v[u].w, i + 1);
        }
    }
    for (; f < n4; f += stride) {
        const v4f v = p4[f];
        const uint32_t i = head + 2 * f;
        ext_visit(a, v.x, v.y, i);
        ext_visit(a, v.z, v.w, i + 1);
    }
    if (blockIdx.x == 0 && tid == 1 && ((n - head) & 1u)) ext_visit(a, pts[2 * (n - 1)], pts[2 * (n - 1) + 1], n - 1);

    ext_block_reduce(a, sk, si, sbad);
    if (tid < 4) {
        part[blockIdx.x].key[tid] = sk[0][tid];
        part[blockIdx.x].idx[tid] = si[0][tid];
    }
    if (tid == 0) part[blockIdx.x].err = sbad[0];
}

// One workgroup: reduce the partials, derive the quadrilateral's edges and the
// region frames, and zero the call's counters.
__global__ __launch_bounds__(kBlock) void k_extremes_final(const ExtPartial* __restrict__ part, int nparts,
                                                           DevHeader* __restrict__ hdr)
{
    __shared__ u64 sk[kWaves][4];
    __shared__ uint32_t si[kWaves][4];
    __shared__ uint32_t sbad[kWaves];
    ExtAcc a;
    ext_init(a);
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
#pragma unroll
        for (int e = 0; e < 4; ++e) lexmin_pair(a.k[e], a.i[e], part[b].key[e], part[b].idx[e]);
        a.bad |= part[b].err;
    }
    ext_block_reduce(a, sk, si, sbad);
    if (threadIdx.x != 0) return;

    uint32_t X[4], Y[4];
    const u64* k = sk[0];
    X[0] = (uint32_t)(k[0] >> 23);      Y[0] = kM - (uint32_t)(k[0] & kM);  // P_minx
    Y[1] = (uint32_t)(k[1] >> 23);      X[1] = (uint32_t)(k[1] & kM);       // P_miny
    X[2] = kM - (uint32_t)(k[2] >> 23); Y[2] = (uint32_t)(k[2] & kM);       // P_maxx
    Y[3] = kM - (uint32_t)(k[3] >> 23); X[3] = kM - (uint32_t)(k[3] & kM);  // P_maxy
    for (int e = 0; e < 4; ++e) {
        hdr->ext_x[e] = X[e];
        hdr->ext_y[e] = Y[e];
        hdr->ext_idx[e] = si[0][e];
    }
    // Edge q runs from E_q to E_{q+1}, E = (P_minx, P_miny, P_maxx, P_maxy);
    // region q is strictly right of it: ex*(y - E_q.y) - ey*(x - E_q.x) < 0.
    for (int q = 0; q < 4; ++q) {
        const int r = (q + 1) & 3;
        const int32_t ex = (int32_t)X[r] - (int32_t)X[q];
        const int32_t ey = (int32_t)Y[r] - (int32_t)Y[q];
        hdr->ex[q] = ex;
        hdr->ey[q] = ey;
        hdr->ec[q] = (double)ex * (double)Y[q] - (double)ey * (double)X[q];
    }
    // Frames: the k1 range of each region and its first point's k2 (sigma).
    uint32_t lo[4], hi[4], sig[4];
    lo[0] = X[0];      hi[0] = X[1];      sig[0] = Y[0];       // R1: P_minx .. P_miny
    lo[1] = Y[1];      hi[1] = Y[2];      sig[1] = kM - X[1];  // R2: P_miny .. P_maxx
    lo[2] = kM - X[2]; hi[2] = kM - X[3]; sig[2] = kM - Y[2];  // R3: P_maxx .. P_maxy
    lo[3] = kM - Y[3]; hi[3] = kM - Y[0]; sig[3] = X[3];       // R4: P_maxy .. P_minx
    for (int q = 0; q < 4; ++q) {
        const uint32_t span = hi[q] >= lo[q] ? hi[q] - lo[q] : 0u;
        uint32_t sh = 0;
        while ((span >> sh) >= (uint32_t)kSlots) ++sh;
        hdr->k1lo[q] = lo[q];
        hdr->k1shift[q] = sh;
        hdr->sigma[q] = sig[q];
        hdr->s1[q] = 0;
        hdr->s2[q] = 0;
    }
    hdr->cand = 0;
    hdr->poly = 0;
    hdr->err = sbad[0];
}

// ---------------------------------------------------------------------------
// Step 2 (Section 2.1.1): exact region test against the quadrilateral (the
// first discard), fused with a tile-level use of the SPA dominance rule, so
// that only the tile's possible chain points reach HBM.
//
// A point p of region q is dominated by another point p' of the region when
// k1' <= k1 and k2' <= k2 and p' precedes p in (k1, k2, index) order; then p
// lies in the triangle (first point, p', last point) and is not a hull vertex
// (the argument of Figure 3).  Domination inside a tile is domination in the
// whole set, so dropping tile-dominated points leaves the result of the
// region sort and SPA unchanged.
//
// Per tile and region, k1 is cut into kSlots slots.  A point is dropped when
//   * the region's first point or a point of an earlier slot has k2 <= its k2,
//   * the slot's smallest-(k2, k1) point precedes it with k1 <= its k1, or
//   * it repeats that point's coordinates with a larger index.
// ---------------------------------------------------------------------------

template <bool kVec4>
__global__ __launch_bounds__(kBlock) void k_classify(const float* __restrict__ pts, uint32_t n,
                                                     DevHeader* __restrict__ hdr, uint32_t* __restrict__ out_key,
                                                     u64* __restrict__ out_val)
{
    __shared__ u64 smin[4][kSlots];
    __shared__ uint32_t sidx[4][kSlots];
    __shared__ uint32_t sexc[4][kSlots];
    __shared__ uint32_t scratch[kWaves];
    __shared__ uint32_t s1cnt[kWaves][4];
    __shared__ uint32_t sbase;

    if (hdr->err) return;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / 64;
    const uint32_t tile = blockIdx.x * kTilePts;

    const double ec0 = hdr->ec[0], ec1 = hdr->ec[1], ec2 = hdr->ec[2], ec3 = hdr->ec[3];
    const double ex0 = hdr->ex[0], ex1 = hdr->ex[1], ex2 = hdr->ex[2], ex3 = hdr->ex[3];
    const double ey0 = hdr->ey[0], ey1 = hdr->ey[1], ey2 = hdr->ey[2], ey3 = hdr->ey[3];
    const uint32_t lo0 = hdr->k1lo[0], lo1 = hdr->k1lo[1], lo2 = hdr->k1lo[2], lo3 = hdr->k1lo[3];
    const uint32_t sh0 = hdr->k1shift[0], sh1 = hdr->k1shift[1], sh2 = hdr->k1shift[2], sh3 = hdr->k1shift[3];
    auto slot_of = [&](uint32_t q, uint32_t k1) -> uint32_t {
        const uint32_t d = (k1 - sel4(q, lo0, lo1, lo2, lo3)) >> sel4(q, sh0, sh1, sh2, sh3);
        return min(d, (uint32_t)(kSlots - 1));
    };

    for (int s = tid; s < 4 * kSlots; s += kBlock) {
        (&smin[0][0])[s] = ~0ull;
        (&sidx[0][0])[s] = ~0u;
    }

    // Point j of this thread: with float4 loads it is tile + 2*(k*256+tid) + h
    // for j = 2k + h; otherwise tile + j*256 + tid.
    float px[kPtsPerThread], py[kPtsPerThread];
    if (kVec4) {
        const v4f* p4 = reinterpret_cast<const v4f*>(pts) + tile / 2;
#pragma unroll
        for (int k = 0; k < kPtsPerThread / 2; ++k) {
            const uint32_t i = tile + 2 * (k * kBlock + tid);
            v4f v = {0.f, 0.f, 0.f, 0.f};
            if (i + 1 < n) {
                v = __builtin_nontemporal_load(p4 + k * kBlock + tid);
            } else if (i < n) {
                v.x = pts[2 * i];
                v.y = pts[2 * i + 1];
            }
            px[2 * k] = v.x;
            py[2 * k] = v.y;
            px[2 * k + 1] = v.z;
            py[2 * k + 1] = v.w;
        }
    } else {
        const v2f* p2 = reinterpret_cast<const v2f*>(pts);
#pragma unroll
        for (int k = 0; k < kPtsPerThread; ++k) {
            const uint32_t i = tile + k * kBlock + tid;
            v2f v = {0.f, 0.f};
            if (i < n) v = __builtin_nontemporal_load(p2 + i);
            px[k] = v.x;
            py[k] = v.y;
        }
    }
    auto index_of = [&](int j) -> uint32_t {
        return kVec4 ? tile + 2 * ((uint32_t)(j >> 1) * kBlock + tid) + (uint32_t)(j & 1)
                     : tile + (uint32_t)j * kBlock + tid;
    };

    __syncthreads();

    // Phase 1: region of every point and the per-slot minimum of (k2, k1).
    u64 reg = 0;  // 3 bits per point: region code, 4 = interior
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
#pragma unroll
    for (int j = 0; j < kPtsPerThread; ++j) {
        uint32_t q = 4;
        if (index_of(j) < n) {
            const double fx = (double)px[j], fy = (double)py[j];
            // exact: every product is below 2^46 and every sum below 2^47
            if (fma(ex3, fy, -(ey3 * fx)) < ec3) q = 3;
            if (fma(ex2, fy, -(ey2 * fx)) < ec2) q = 2;
            if (fma(ex1, fy, -(ey1 * fx)) < ec1) q = 1;
            if (fma(ex0, fy, -(ey0 * fx)) < ec0) q = 0;
        }
        reg |= (u64)q << (3 * j);
        c0 += q == 0;
        c1 += q == 1;
        c2 += q == 2;
        c3 += q == 3;
        if (q < 4) {
            const uint32_t X = (uint32_t)px[j], Y = (uint32_t)py[j];
            const uint32_t k1 = frame_k1(q, X, Y), k2 = frame_k2(q, X, Y);
            atomicMin(&smin[q][slot_of(q, k1)], ((u64)k2 << 23) | k1);
        }
    }
    {
        const uint32_t w0 = wave_sum(c0), w1 = wave_sum(c1), w2 = wave_sum(c2), w3 = wave_sum(c3);
        if (lane_id() == 0) {
            s1cnt[wave][0] = w0;
            s1cnt[wave][1] = w1;
            s1cnt[wave][2] = w2;
            s1cnt[wave][3] = w3;
        }
    }
    __syncthreads();

    // Phase 2: wave w scans region w's slots; sexc[w][s] becomes the smallest
    // k2 over earlier slots and the region's first point.
    {
        const uint32_t q = wave;
        const uint32_t sigma = hdr->sigma[q];
        constexpr int per = kSlots / 64;
        uint32_t v[per];
        uint32_t run = ~0u;
#pragma unroll
        for (int s = 0; s < per; ++s) {
            const u64 m = smin[q][lane_id() * per + s];
            v[s] = m == ~0ull ? ~0u : (uint32_t)(m >> 23);
            run = min(run, v[s]);
        }
        const uint32_t incl = wave_incl_min(run);
        uint32_t before = __shfl_up(incl, 1);
        if (lane_id() == 0) before = ~0u;
        before = min(before, sigma);
#pragma unroll
        for (int s = 0; s < per; ++s) {
            sexc[q][lane_id() * per + s] = before;
            before = min(before, v[s]);
        }
    }
    if (tid < 4) {
        uint32_t tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += s1cnt[w][tid];
        if (tot) atomicAdd(&hdr->s1[tid], tot);
    }
    __syncthreads();

    // Phase 3: dominance tests.
    uint32_t keep = 0, dupc = 0;
#pragma unroll
    for (int j = 0; j < kPtsPerThread; ++j) {
        const uint32_t q = (uint32_t)(reg >> (3 * j)) & 7u;
        if (q < 4) {
            const uint32_t X = (uint32_t)px[j], Y = (uint32_t)py[j];
            const uint32_t k1 = frame_k1(q, X, Y), k2 = frame_k2(q, X, Y);
            const uint32_t slot = slot_of(q, k1);
            const u64 me = ((u64)k2 << 23) | k1;
            const u64 best = smin[q][slot];
            bool k = k2 < sexc[q][slot];
            if (k && best < me && (uint32_t)(best & kM) <= k1) k = false;
            if (k && best == me) {
                atomicMin(&sidx[q][slot], index_of(j));
                dupc |= 1u << j;
            }
            keep |= (k ? 1u : 0u) << j;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPtsPerThread; ++j) {
        if ((dupc >> j) & 1u) {
            const uint32_t q = (uint32_t)(reg >> (3 * j)) & 7u;
            const uint32_t X = (uint32_t)px[j], Y = (uint32_t)py[j];
            if (sidx[q][slot_of(q, frame_k1(q, X, Y))] != index_of(j)) keep &= ~(1u << j);
        }
    }

    // Phase 4: compact the tile's kept records (one global atomic per tile).
    uint32_t total;
    const uint32_t off = block_excl_sum(__popc(keep), scratch, total);
    if (tid == 0) sbase = total ? atomicAdd(&hdr->cand, total) : 0u;
    __syncthreads();
    uint32_t pos = sbase + off;
#pragma unroll
    for (int j = 0; j < kPtsPerThread; ++j) {
        if ((keep >> j) & 1u) {
            const uint32_t q = (uint32_t)(reg >> (3 * j)) & 7u;
            const uint32_t X = (uint32_t)px[j], Y = (uint32_t)py[j];
            out_key[pos] = (q << 23) | frame_k1(q, X, Y);
            out_val[pos] = ((u64)frame_k2(q, X, Y) << 32) | index_of(j);
            ++pos;
        }
    }
}

// ---------------------------------------------------------------------------
// Steps 3-4 (Section 2.1; Table 1): sort the surviving records of all four
// regions at once by the 25-bit key q << 23 | k1, least significant digit
// first (8, 8, 9 bits), stably, so each region lands contiguously and in
// Table 1's order.  A pass = per-chunk digit counts, one scan over all
// counts, then a stable scatter whose in-wave ranks come from ballot
// matching.  The record count lives in device memory; kSortBlocks chunks
// split it.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_sort_hist(const uint32_t* __restrict__ key,
                                                      const DevHeader* __restrict__ hdr, int shift, int bits,
                                                      uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[kMaxBins];
    const uint32_t bins = 1u << bits, mask = bins - 1;
    for (uint32_t d = threadIdx.x; d < bins; d += kBlock) h[d] = 0;
    __syncthreads();
    uint32_t lo, hi;
    chunk_range(hdr->err ? 0u : hdr->cand, blockIdx.x, gridDim.x, lo, hi);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kBlock) atomicAdd(&h[(key[i] >> shift) & mask], 1u);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < bins; d += kBlock) hist[d * gridDim.x + blockIdx.x] = h[d];
}

// One workgroup of 1024 threads: exclusive prefix sum of `len` counts in
// place (digit-major, so the result is each chunk's first slot per digit).
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* __restrict__ hist, uint32_t len)
{
    __shared__ uint32_t wsum[16];
    const uint32_t tid = threadIdx.x, per = (len + 1023) / 1024;
    const uint32_t lo = min(len, tid * per), hi = min(len, lo + per);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i) s += hist[i];
    const uint32_t incl = wave_incl_sum(s);
    if (lane_id() == 63) wsum[tid / 64] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t w = 0; w < tid / 64; ++w) before += wsum[w];
    uint32_t run = before + incl - s;
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t c = hist[i];
        hist[i] = run;
        run += c;
    }
}

template <int kBits>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(const uint32_t* __restrict__ key_in,
                                                         const u64* __restrict__ val_in,
                                                         uint32_t* __restrict__ key_out, u64* __restrict__ val_out,
                                                         const DevHeader* __restrict__ hdr, int shift,
                                                         const uint32_t* __restrict__ offs)
{
    constexpr uint32_t kBins = 1u << kBits, kMask = kBins - 1;
    __shared__ uint32_t cursor[kBins];
    __shared__ uint32_t wcnt[kWaves][kBins];
    const uint32_t tid = threadIdx.x, wave = tid / 64, lane = lane_id();
    for (uint32_t d = tid; d < kBins; d += kBlock) {
        cursor[d] = offs[d * gridDim.x + blockIdx.x];
#pragma unroll
        for (int w = 0; w < kWaves; ++w) wcnt[w][d] = 0;
    }
    __syncthreads();
    const uint32_t count = hdr->err ? 0u : hdr->cand;
    uint32_t lo, hi;
    chunk_range(count, blockIdx.x, gridDim.x, lo, hi);
    const u64 lt = (1ull << lane) - 1ull;
    for (uint32_t base = lo; base < hi; base += kSortTile) {
        // Wave w owns records [base + w*64*IPT, +64*IPT); record j of lane l
        // sits at +j*64 + l, so (j, l) is the order of the wave's records.
        uint32_t k[kSortIpt], d[kSortIpt], r[kSortIpt];
        u64 v[kSortIpt];
        const uint32_t wbase = base + wave * 64 * kSortIpt;
#pragma unroll
        for (int j = 0; j < kSortIpt; ++j) {
            const uint32_t i = wbase + j * 64 + lane;
            const bool ok = i < hi;
            k[j] = ok ? key_in[i] : 0u;
            v[j] = ok ? val_in[i] : 0ull;
            d[j] = (k[j] >> shift) & kMask;
            u64 peers = __ballot(ok);
#pragma unroll
            for (int b = 0; b < kBits; ++b) {
                const u64 bal = __ballot((d[j] >> b) & 1u);
                peers &= ((d[j] >> b) & 1u) ? bal : ~bal;
            }
            const uint32_t below = (uint32_t)__popcll(peers & lt);
            const uint32_t cur = ok ? wcnt[wave][d[j]] : 0u;
            r[j] = cur + below;
            if (ok && below == 0) wcnt[wave][d[j]] = cur + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // wcnt[w][d] becomes the output slot of wave w's first digit-d record.
        for (uint32_t dd = tid; dd < kBins; dd += kBlock) {
            uint32_t run = cursor[dd];
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wcnt[w][dd];
                wcnt[w][dd] = run;
                run += c;
            }
            cursor[dd] = run;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSortIpt; ++j) {
            const uint32_t i = wbase + j * 64 + lane;
            const uint32_t dst = wcnt[wave][d[j]] + r[j];
            if (i < hi && dst < count) {
                key_out[dst] = k[j];
                val_out[dst] = v[j];
            }
        }
        __syncthreads();
        for (uint32_t dd = tid; dd < kBins; dd += kBlock) {
#pragma unroll
            for (int w = 0; w < kWaves; ++w) wcnt[w][dd] = 0;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Step 5 (Figure 2): SPA over the sorted records as a segmented exclusive
// prefix minimum.  In each region a record is kept iff its k2 is below the
// region's first point's k2 and below every earlier record's k2; Figure 2's
// threshold t is exactly that running minimum, since a discarded record
// never lowers it.  Records with equal key (q, k1) form a group; only the
// group's smallest (k2, index) can survive, and it does so iff its k2 is
// below the minimum over the records before the group.
//
// The prefix minimum runs over tagged values ((3 - q) << 23 | k2): records of
// earlier regions carry larger tags, so a prefix minimum with this region's
// tag is this region's running minimum.  Chunks get their seed from the
// per-chunk minima of the chunks before them.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_spa_part(const uint32_t* __restrict__ key, const u64* __restrict__ val,
                                                     const DevHeader* __restrict__ hdr, uint32_t* __restrict__ part)
{
    __shared__ uint32_t sm[kWaves][4];
    uint32_t lo, hi;
    chunk_range(hdr->err ? 0u : hdr->cand, blockIdx.x, gridDim.x, lo, hi);
    uint32_t m0 = ~0u, m1 = ~0u, m2 = ~0u, m3 = ~0u;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        const uint32_t q = key[i] >> 23, k2 = (uint32_t)(val[i] >> 32);
        if (q == 0) m0 = min(m0, k2);
        if (q == 1) m1 = min(m1, k2);
        if (q == 2) m2 = min(m2, k2);
        if (q == 3) m3 = min(m3, k2);
    }
    m0 = wave_min(m0);
    m1 = wave_min(m1);
    m2 = wave_min(m2);
    m3 = wave_min(m3);
    const uint32_t wave = threadIdx.x / 64;
    if (lane_id() == 0) {
        sm[wave][0] = m0;
        sm[wave][1] = m1;
        sm[wave][2] = m2;
        sm[wave][3] = m3;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        uint32_t m = ~0u;
        for (int w = 0; w < kWaves; ++w) m = min(m, sm[w][threadIdx.x]);
        part[blockIdx.x * 4 + threadIdx.x] = m;
    }
}

__global__ __launch_bounds__(kBlock) void k_spa_keep(const uint32_t* __restrict__ key, const u64* __restrict__ val,
                                                     const DevHeader* __restrict__ hdr,
                                                     const uint32_t* __restrict__ part, uint32_t* __restrict__ kept_key,
                                                     u64* __restrict__ kept_val, uint32_t* __restrict__ cnt)
{
    __shared__ uint32_t seed[4];
    __shared__ uint32_t red[kWaves][4];
    __shared__ uint32_t scratch[kWaves];
    __shared__ uint32_t kcnt[4];
    const uint32_t tid = threadIdx.x, wave = tid / 64, b = blockIdx.x;
    const uint32_t count = hdr->err ? 0u : hdr->cand;

    // Seed per region: the first point's k2 and the minima of earlier chunks.
    {
        uint32_t m[4] = {~0u, ~0u, ~0u, ~0u};
        for (uint32_t c = tid; c < b; c += kBlock) {
#pragma unroll
            for (int q = 0; q < 4; ++q) m[q] = min(m[q], part[c * 4 + q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            m[q] = wave_min(m[q]);
            if (lane_id() == 0) red[wave][q] = m[q];
        }
        if (tid < 4) kcnt[tid] = 0;
        __syncthreads();
        if (tid < 4) {
            uint32_t s = hdr->sigma[tid];
            for (int w = 0; w < kWaves; ++w) s = min(s, red[w][tid]);
            seed[tid] = s;
        }
        __syncthreads();
    }

    uint32_t lo, hi;
    chunk_range(count, b, gridDim.x, lo, hi);
    uint32_t carry = ~0u;   // tagged minimum over this chunk's earlier sub-tiles
    uint32_t written = 0;   // survivors written so far by this chunk
    for (uint32_t base = lo; base < hi; base += kSpaTile) {
        // Thread t holds records base + t*IPT + j (consecutive per thread).
        uint32_t kk[kSpaIpt], tag[kSpaIpt], pre[kSpaIpt];
        u64 vv[kSpaIpt];
        uint32_t run = ~0u;
#pragma unroll
        for (int j = 0; j < kSpaIpt; ++j) {
            const uint32_t i = base + tid * kSpaIpt + j;
            const bool ok = i < hi;
            kk[j] = ok ? key[i] : 0u;
            vv[j] = ok ? val[i] : 0ull;
            tag[j] = ok ? ((3u - (kk[j] >> 23)) << 23) | (uint32_t)(vv[j] >> 32) : ~0u;
            pre[j] = run;
            run = min(run, tag[j]);
        }
        uint32_t tile_min;
        const uint32_t before = min(carry, block_excl_min(run, scratch, tile_min));
        uint32_t keep = 0;
        u64 gmin[kSpaIpt];
#pragma unroll
        for (int j = 0; j < kSpaIpt; ++j) {
            const uint32_t i = base + tid * kSpaIpt + j;
            gmin[j] = vv[j];
            if (i < hi) {
                const uint32_t q = kk[j] >> 23;
                const uint32_t pm = min(before, pre[j]);
                uint32_t thr = seed[q];
                if ((pm >> 23) == 3u - q) thr = min(thr, pm & kM);
                const bool head = (i == 0) || key[i - 1] != kk[j];
                if (head) {
                    u64 g = vv[j];
                    for (uint32_t m = i + 1; m < count && key[m] == kk[j]; ++m) g = min(g, val[m]);
                    gmin[j] = g;
                    if ((uint32_t)(g >> 32) < thr) keep |= 1u << j;
                }
            }
        }
        uint32_t total;
        uint32_t pos = block_excl_sum(__popc(keep), scratch, total);
#pragma unroll
        for (int j = 0; j < kSpaIpt; ++j) {
            if ((keep >> j) & 1u) {
                kept_key[lo + written + pos] = kk[j];
                kept_val[lo + written + pos] = gmin[j];
                atomicAdd(&kcnt[kk[j] >> 23], 1u);
                ++pos;
            }
        }
        written += total;
        carry = min(carry, tile_min);
    }
    __syncthreads();
    if (tid < 4) cnt[b * 4 + tid] = kcnt[tid];
}

// ---------------------------------------------------------------------------
// Step 6 (Section 2.1; Section 2.2.2): join the chains into the simple polygon
// [P_minx, R1, P_miny, R2, P_maxx, R3, P_maxy, R4] with coordinates rebuilt
// from the frames.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_chain(const uint32_t* __restrict__ kept_key,
                                                  const u64* __restrict__ kept_val, const uint32_t* __restrict__ cnt,
                                                  DevHeader* __restrict__ hdr, PolyRec* __restrict__ poly)
{
    __shared__ uint32_t tot[kWaves][4], pre[kWaves][4];
    __shared__ uint32_t T[4], P[4], mine[4];
    const uint32_t tid = threadIdx.x, wave = tid / 64, b = blockIdx.x, nb = gridDim.x;
    {
        uint32_t t[4] = {0, 0, 0, 0}, p[4] = {0, 0, 0, 0};
        for (uint32_t c = tid; c < nb; c += kBlock) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t v = cnt[c * 4 + q];
                t[q] += v;
                p[q] += c < b ? v : 0u;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            t[q] = wave_sum(t[q]);
            p[q] = wave_sum(p[q]);
            if (lane_id() == 0) {
                tot[wave][q] = t[q];
                pre[wave][q] = p[q];
            }
        }
        __syncthreads();
        if (tid < 4) {
            uint32_t a = 0, c = 0;
            for (int w = 0; w < kWaves; ++w) {
                a += tot[w][tid];
                c += pre[w][tid];
            }
            T[tid] = a;
            P[tid] = c;
            mine[tid] = cnt[b * 4 + tid];
        }
        __syncthreads();
    }
    const uint32_t count = hdr->err ? 0u : hdr->cand;
    if (b == 0 && tid < 4) {
        uint32_t at = tid;
        for (uint32_t q = 0; q < tid; ++q) at += T[q];
        poly[at] = PolyRec{(int32_t)hdr->ext_idx[tid], (int32_t)hdr->ext_x[tid], (int32_t)hdr->ext_y[tid]};
        hdr->s2[tid] = T[tid];
        if (tid == 0) hdr->poly = 4 + T[0] + T[1] + T[2] + T[3];
    }
    uint32_t lo, hi;
    chunk_range(count, b, nb, lo, hi);
    const uint32_t n_here = mine[0] + mine[1] + mine[2] + mine[3];
    for (uint32_t k = tid; k < n_here; k += kBlock) {
        const uint32_t kk = kept_key[lo + k];
        const u64 vv = kept_val[lo + k];
        const uint32_t q = kk >> 23, k1 = kk & kM, k2 = (uint32_t)(vv >> 32);
        uint32_t start = q + 1, rank = k;
        for (uint32_t r = 0; r < q; ++r) {
            start += T[r];
            rank -= mine[r];
        }
        const uint32_t X = sel4(q, k1, kM - k2, kM - k1, k2);
        const uint32_t Y = sel4(q, k2, k1, kM - k2, kM - k1);
        poly[start + P[q] + rank] = PolyRec{(int32_t)(uint32_t)vv, (int32_t)X, (int32_t)Y};
    }
}

// ---------------------------------------------------------------------------
// Host side: workspaces, the pipeline and the C ABI
// ---------------------------------------------------------------------------

namespace {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Workspace {
    std::mutex mu;
    int device = 0;
    hipStream_t stream = nullptr;
    size_t cap = 0;  // points
    char* dbuf = nullptr;
    DevHeader* hdr = nullptr;
    ExtPartial* part = nullptr;
    uint32_t* key[2] = {nullptr, nullptr};
    u64* val[2] = {nullptr, nullptr};
    uint32_t* hist = nullptr;
    uint32_t* spa_part = nullptr;
    uint32_t* spa_cnt = nullptr;
    PolyRec* poly = nullptr;
    DevHeader* h_hdr = nullptr;     // pinned
    PolyRec* h_poly = nullptr;      // pinned
    size_t h_poly_cap = 0;
    int32_t* h_out = nullptr;       // pinned: count, then indices
    size_t h_out_cap = 0;
    std::vector<int32_t> xy, idx;   // finish input
    hipEvent_t ev[8] = {};
    bool events = false;
};

size_t device_bytes(size_t cap)
{
    size_t b = 0;
    b += align_up(sizeof(DevHeader), 256);
    b += align_up(sizeof(ExtPartial) * kExtBlocks, 256);
    b += 2 * align_up(sizeof(uint32_t) * cap, 256);
    b += 2 * align_up(sizeof(u64) * cap, 256);
    b += align_up(sizeof(uint32_t) * kMaxBins * kSortBlocks, 256);
    b += 2 * align_up(sizeof(uint32_t) * 4 * kSortBlocks, 256);
    b += align_up(sizeof(PolyRec) * (cap + 4), 256);
    return b;
}

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;
bool g_timing = false;
thread_local ch_stats t_stats;

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

int ensure_device(Workspace& w, size_t n)
{
    if (w.dbuf && w.cap >= n) return CH_OK;
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
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* r = p + o;
        o += align_up(bytes, 256);
        return r;
    };
    w.hdr = reinterpret_cast<DevHeader*>(take(sizeof(DevHeader)));
    w.part = reinterpret_cast<ExtPartial*>(take(sizeof(ExtPartial) * kExtBlocks));
    for (int i = 0; i < 2; ++i) w.key[i] = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * cap));
    for (int i = 0; i < 2; ++i) w.val[i] = reinterpret_cast<u64*>(take(sizeof(u64) * cap));
    w.hist = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kMaxBins * kSortBlocks));
    w.spa_part = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 4 * kSortBlocks));
    w.spa_cnt = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 4 * kSortBlocks));
    w.poly = reinterpret_cast<PolyRec*>(take(sizeof(PolyRec) * (cap + 4)));
    return CH_OK;
}

int ensure_host(Workspace& w, size_t poly, size_t out)
{
    if (!w.h_hdr) CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_hdr), sizeof(DevHeader), hipHostMallocDefault));
    if (w.h_poly_cap < poly) {
        if (w.h_poly) CH_TRY(hipHostFree(w.h_poly));
        w.h_poly = nullptr;
        const size_t cap = std::max<size_t>(poly, 4096);
        CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_poly), sizeof(PolyRec) * cap, hipHostMallocDefault));
        w.h_poly_cap = cap;
    }
    if (w.h_out_cap < out + 1) {
        if (w.h_out) CH_TRY(hipHostFree(w.h_out));
        w.h_out = nullptr;
        const size_t cap = std::max<size_t>(out + 1, 4096);
        CH_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_out), sizeof(int32_t) * cap, hipHostMallocDefault));
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
    if (w->dbuf) (void)hipFree(w->dbuf);
    if (w->h_hdr) (void)hipHostFree(w->h_hdr);
    if (w->h_poly) (void)hipHostFree(w->h_poly);
    if (w->h_out) (void)hipHostFree(w->h_out);
    if (w->events) {
        for (auto& e : w->ev) (void)hipEventDestroy(e);
    }
    (void)hipSetDevice(cur);
    delete w;
}

int record(Workspace& w, int k)
{
    if (!g_timing) return CH_OK;
    if (!w.events) {
        for (auto& e : w.ev) CH_TRY(hipEventCreate(&e));
        w.events = true;
    }
    return hip_status(hipEventRecord(w.ev[k], w.stream));
}

#define CH_LAUNCH(...)                                   \
    do {                                                 \
        __VA_ARGS__;                                     \
        const int rc_ = hip_status(hipGetLastError());   \
        if (rc_ != CH_OK) return rc_;                    \
    } while (0)

// Steps 1-6 on the device; leaves the polygon in w.poly and the counts in
// w.hdr, then copies both to pinned host memory and waits.
int run_preprocess(Workspace& w, const float* pts, uint32_t n)
{
    hipStream_t s = w.stream;
    CH_TRY(record(w, 0));
    const uint32_t head = (reinterpret_cast<uintptr_t>(pts) & 15u) ? 1u : 0u;
    const uint32_t n4 = (n - head) / 2;
    const int gext = (int)std::max<uint32_t>(1u, std::min<uint32_t>(kExtBlocks, (n4 + kBlock * kExtUnroll - 1) /
                                                                                   (kBlock * kExtUnroll)));
    CH_LAUNCH(hipLaunchKernelGGL(k_extremes, dim3(gext), dim3(kBlock), 0, s, pts, n, head, w.part));
    CH_TRY(record(w, 1));
    CH_LAUNCH(hipLaunchKernelGGL(k_extremes_final, dim3(1), dim3(kBlock), 0, s, w.part, gext, w.hdr));
    CH_TRY(record(w, 2));
    const uint32_t tiles = (n + kTilePts - 1) / kTilePts;
    if (head == 0) {
        CH_LAUNCH(hipLaunchKernelGGL(k_classify<true>, dim3(tiles), dim3(kBlock), 0, s, pts, n, w.hdr, w.key[0],
                                     w.val[0]));
    } else {
        CH_LAUNCH(hipLaunchKernelGGL(k_classify<false>, dim3(tiles), dim3(kBlock), 0, s, pts, n, w.hdr, w.key[0],
                                     w.val[0]));
    }
    CH_TRY(record(w, 3));
    // region sort: digits [0,8), [8,16), [16,25)
    const int shifts[3] = {0, 8, 16}, bits[3] = {8, 8, 9};
    for (int p = 0; p < 3; ++p) {
        const int src = p & 1, dst = src ^ 1;
        CH_LAUNCH(hipLaunchKernelGGL(k_sort_hist, dim3(kSortBlocks), dim3(kBlock), 0, s, w.key[src], w.hdr, shifts[p],
                                     bits[p], w.hist));
        CH_LAUNCH(hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, w.hist,
                                     (uint32_t)((1u << bits[p]) * kSortBlocks)));
        if (bits[p] == 8) {
            CH_LAUNCH(hipLaunchKernelGGL(k_sort_scatter<8>, dim3(kSortBlocks), dim3(kBlock), 0, s, w.key[src],
                                         w.val[src], w.key[dst], w.val[dst], w.hdr, shifts[p], w.hist));
        } else {
            CH_LAUNCH(hipLaunchKernelGGL(k_sort_scatter<9>, dim3(kSortBlocks), dim3(kBlock), 0, s, w.key[src],
                                         w.val[src], w.key[dst], w.val[dst], w.hdr, shifts[p], w.hist));
        }
    }
    CH_TRY(record(w, 4));
    CH_LAUNCH(hipLaunchKernelGGL(k_spa_part, dim3(kSortBlocks), dim3(kBlock), 0, s, w.key[1], w.val[1], w.hdr,
                                 w.spa_part));
    CH_LAUNCH(hipLaunchKernelGGL(k_spa_keep, dim3(kSortBlocks), dim3(kBlock), 0, s, w.key[1], w.val[1], w.hdr,
                                 w.spa_part, w.key[0], w.val[0], w.spa_cnt));
    CH_TRY(record(w, 5));
    CH_LAUNCH(hipLaunchKernelGGL(k_chain, dim3(kSortBlocks), dim3(kBlock), 0, s, w.key[0], w.val[0], w.spa_cnt, w.hdr,
                                 w.poly));
    CH_TRY(record(w, 6));
    CH_TRY(hipMemcpyAsync(w.h_hdr, w.hdr, sizeof(DevHeader), hipMemcpyDeviceToHost, s));
    CH_TRY(hipStreamSynchronize(s));
    if (w.h_hdr->err) return CH_EDOMAIN;
    const size_t m = w.h_hdr->poly;
    CH_TRY(ensure_host(w, m, 0));
    if (m) CH_TRY(hipMemcpyAsync(w.h_poly, w.poly, sizeof(PolyRec) * m, hipMemcpyDeviceToHost, s));
    CH_TRY(record(w, 7));
    CH_TRY(hipStreamSynchronize(s));
    return CH_OK;
}

void fill_stats(const Workspace& w, int64_t n, ch_stats* st)
{
    std::memset(st, 0, sizeof(*st));
    st->n = n;
    if (n == 0) return;
    const DevHeader& h = *w.h_hdr;
    for (int e = 0; e < 4; ++e) {
        st->ext_idx[e] = (int32_t)h.ext_idx[e];
        st->ext_xy[2 * e] = (int32_t)h.ext_x[e];
        st->ext_xy[2 * e + 1] = (int32_t)h.ext_y[e];
        st->s1[e] = h.s1[e];
        st->s2[e] = h.s2[e];
    }
    st->candidates = h.cand;
    st->polygon = h.poly;
    if (g_timing && w.events) {
        for (int k = 0; k < 7; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, w.ev[k], w.ev[k + 1]) == hipSuccess) st->ms[k] = ms;
        }
    }
}

// Finish on the host: Melkman on the polygon copied out by run_preprocess.
int finish(Workspace& w, int32_t* out, int64_t* h)
{
    const size_t m = w.h_hdr->poly;
    w.xy.resize(2 * m);
    w.idx.resize(m);
    for (size_t i = 0; i < m; ++i) {
        w.idx[i] = w.h_poly[i].idx;
        w.xy[2 * i] = w.h_poly[i].x;
        w.xy[2 * i + 1] = w.h_poly[i].y;
    }
    return melkman_finish(w.xy.data(), w.idx.data(), (int64_t)m, out, h) == 0 ? CH_OK : CH_EHIP;
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
    CH_TRY(ensure_host(*w, 0, 0));
    if (n == 0) {
        w->h_out[0] = 0;
        CH_TRY(hipMemcpyAsync(out_count, w->h_out, sizeof(int32_t), hipMemcpyHostToDevice, stream));
        CH_TRY(hipStreamSynchronize(stream));
        return CH_OK;
    }
    CH_TRY(ensure_device(*w, (size_t)n));
    rc = run_preprocess(*w, points, (uint32_t)n);
    if (rc == CH_OK) {
        fill_stats(*w, n, &st);
        rc = ensure_host(*w, 0, (size_t)w->h_hdr->poly);
    }
    int64_t h = 0;
    if (rc == CH_OK) {
        const auto t0 = std::chrono::steady_clock::now();
        rc = finish(*w, w->h_out + 1, &h);
        const auto t1 = std::chrono::steady_clock::now();
        st.ms[7] = std::chrono::duration<float, std::milli>(t1 - t0).count();
        st.hull = h;
    }
    if (rc != CH_OK) h = 0;
    w->h_out[0] = (int32_t)h;
    CH_TRY(hipMemcpyAsync(out_count, w->h_out, sizeof(int32_t), hipMemcpyHostToDevice, stream));
    if (h) CH_TRY(hipMemcpyAsync(out_idx, w->h_out + 1, sizeof(int32_t) * (size_t)h, hipMemcpyHostToDevice, stream));
    CH_TRY(hipStreamSynchronize(stream));
    return rc;
}

}  // namespace
}  // namespace chainhull

using namespace chainhull;

extern "C" {

int hull2d(const float* points, int64_t n, int32_t* out_idx, int32_t* out_count, void* stream)
{
    return hull_one(points, n, out_idx, out_count, reinterpret_cast<hipStream_t>(stream));
}

int hull2d_batched(const float* points, const int64_t* offsets, int32_t num_sets, int32_t* out_idx,
                   int32_t* out_counts, void* stream)
{
    if (num_sets < 0 || (num_sets > 0 && (!offsets || !out_counts))) return CH_EINVAL;
    if (num_sets == 0) return CH_OK;
    if (offsets[0] != 0) return CH_EINVAL;
    for (int32_t s = 0; s < num_sets; ++s) {
        if (offsets[s + 1] < offsets[s] || offsets[s + 1] > INT32_MAX) return CH_EINVAL;
    }
    if (offsets[num_sets] > 0 && (!points || !out_idx)) return CH_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int first_err = CH_OK;
    for (int32_t s = 0; s < num_sets; ++s) {
        const int64_t lo = offsets[s], m = offsets[s + 1] - lo;
        const int rc = hull_one(points + 2 * lo, m, out_idx + lo, out_counts + s, st);
        if (rc != CH_OK) {
            int32_t code = rc;
            (void)hipMemcpy(out_counts + s, &code, sizeof(code), hipMemcpyHostToDevice);
            if (first_err == CH_OK) first_err = rc;
        }
    }
    return first_err;
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
    CH_TRY(ensure_host(*w, 0, 0));
    CH_TRY(ensure_device(*w, (size_t)n));
    rc = run_preprocess(*w, points, (uint32_t)n);
    if (rc != CH_OK) return rc;
    fill_stats(*w, n, &st);
    // drop consecutive coincident vertices (cyclically), as the finish does
    const size_t m = w->h_hdr->poly;
    int64_t k = 0;
    int32_t lx = -1, ly = -1;
    for (size_t i = 0; i < m; ++i) {
        const PolyRec& r = w->h_poly[i];
        if (k > 0 && r.x == lx && r.y == ly) continue;
        poly_idx[k++] = r.idx;
        lx = r.x;
        ly = r.y;
    }
    if (m) {
        const int32_t fx = w->h_poly[0].x, fy = w->h_poly[0].y;
        // the first vertex is kept; trailing copies of it close the cycle
        while (k > 1 && lx == fx && ly == fy) {
            --k;
            // coordinates of the new last kept vertex
            for (size_t i = m; i-- > 0;) {
                if (w->h_poly[i].idx == poly_idx[k - 1]) {
                    lx = w->h_poly[i].x;
                    ly = w->h_poly[i].y;
                    break;
                }
            }
        }
    }
    *poly_count = k;
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

int chainhull_last_stats(ch_stats* out)
{
    if (!out) return CH_EINVAL;
    *out = t_stats;
    return CH_OK;
}

void chainhull_set_timing(int enable) { g_timing = enable != 0; }

const char* chainhull_strerror(int status)
{
    switch (status) {
    case CH_OK: return "success";
    case CH_EINVAL: return "invalid argument";
    case CH_EDOMAIN: return "a coordinate is not an integer in [0, 2^23)";
    case CH_ENOMEM: return "out of memory";
    case CH_EHIP: return "HIP runtime error";
    case CH_EADMIT: return "request not admitted";
    default: return "unknown status";
    }
}

void chainhull_release(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_ws) free_workspace(kv.second);
    g_ws.clear();
}

size_t chainhull_workspace_bytes(int64_t n)
{
    if (n < 0) return 0;
    return device_bytes(std::max<size_t>((size_t)n, 1u << 16));
}

}  // extern "C"
