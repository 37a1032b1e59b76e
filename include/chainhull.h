/*
 * chainhull: the data-parallel hot path of the CudaChain planar convex hull
 * method (G. Mei, "CudaChain: A Practical GPU-accelerated 2D Convex Hull
 * Algorithm", arXiv 1508.05488) on AMD Instinct MI355X (gfx950).
 *
 * The method (Section 2.1, steps 1-7): find the four extreme points; discard
 * the points inside their quadrilateral and distribute the rest into four
 * corner regions (Section 2.1.1); sort each region (Table 1); discard again
 * with the Sorting-based Preprocessing Approach, SPA (Figure 2); join the
 * per-region chains into a simple polygon; finish with Melkman's convex hull
 * of a simple polygon (Section 2.1.3).
 *
 * Domain.  Points are interleaved float32 (x, y) pairs whose values are
 * integers in [0, 2^23); -0.0 counts as 0.  Every predicate is exact.  Any
 * other value (NaN, +-Inf, a fraction, a negative value, >= 2^23) is rejected
 * with CH_EDOMAIN.
 *
 * Output convention.  The hull is the list of its strict vertices (collinear
 * boundary points are excluded), each reported by the smallest index among
 * its exact duplicates, counter-clockwise (y axis up), starting at the vertex
 * with the smallest y and, among those, the smallest x.  One distinct point
 * gives [its smallest index]; an all-collinear set gives its two end points,
 * the lowest-then-leftmost first; n == 0 gives an empty hull.
 *
 * Ownership.  Every pointer is owned by the caller; the library never frees
 * or keeps one past the call.  The library owns a workspace per (device,
 * stream) that grows on demand and is freed by chainhull_release().
 * Concurrency.  Calls on different streams may run concurrently; calls on
 * one stream must not overlap (the caller serialises them).
 * Errors.  Every entry point returns a ch_status.  On failure the hull count
 * is 0 and the output indices are unspecified.  HIP failures return CH_EHIP
 * and leave the stream usable.
 */
#ifndef CHAINHULL_H
#define CHAINHULL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CH_OK = 0,
    CH_EINVAL = -1,  /* bad argument: n out of range, null pointer, bad offsets */
    CH_EDOMAIN = -2, /* a coordinate is not an integer in [0, 2^23) */
    CH_ENOMEM = -3,  /* device or pinned host allocation failed */
    CH_EHIP = -4,    /* a HIP runtime call failed */
    CH_EADMIT = -5,  /* a serving request that alone exceeds the server's memory budget */
    CH_ECAPACITY = -6 /* hull2d_noalloc: more points than its fixed device buffer holds */
} ch_status;

/* Counts and timings of the most recent call on the calling thread. */
typedef struct {
    int64_t n;            /* input points */
    int32_t ext_idx[4];   /* P_minx, P_miny, P_maxx, P_maxy (Section 2.1 step 1) */
    int32_t ext_xy[8];    /* their (x, y) */
    int64_t s1[4];        /* round-1 survivors in R1..R4 (Section 2.1.1); counted
                             by chainhull_polygon only, -1 after hull2d */
    int64_t open;         /* points that pass the sampled-staircase dominance test
                             in the single pass over the input */
    int64_t candidates;   /* records the dominance filters pass to the region sort */
    int64_t s2[4];        /* SPA survivors in R1..R4 (Figure 2) */
    int64_t polygon;      /* vertices of the polygon handed to the finish, the
                             four extreme points included, before de-duplication
                             (after the pre-hull in hull2d) */
    int64_t hull;         /* hull vertices */
    /* Milliseconds per stage when timing is on (chainhull_set_timing), from
     * HIP events on the call's stream: 0 sampled staircases, 1 the pass over
     * the points (validation, staircase test, extreme points reduced),
     * 2 quadrilateral discard + region distribution + chunk dominance filter
     * + each workgroup's records sorted by bucket (and, in chainhull_polygon,
     * the round-1 counts), 3 the bucket table's columns (bucket sizes,
     * starts, thresholds), 4 region sort, second level + SPA + chain
     * concatenation (+ pre-hull in hull2d), 5 the device finish of hull2d;
     * the host finish of
     * hull2d in wall-clock time, 0 when the device finished (it runs only if
     * the device finish gives up): 6 the polygon gathered on the device into
     * pinned memory and waited for, 7 Melkman's algorithm on it. */
    float ms[8];
    int32_t device_finish;  /* 1 when hull2d finished step 7 on the device */
    int32_t fused;          /* 1 when the small-input path (one workgroup of the
                               batched kernel) computed the hull: the stage counts
                               are then -1 and ms_pre spans that kernel */
    float ms_pre;         /* steps 1-6 on the device (stages 0-4) as one HIP event
                             span, when timing is on */
    float ms_finish;      /* the device finish (stage 5) as one span */
} ch_stats;

/*
 * hull2d: exact convex hull of one point set (Section 2.1, steps 1-7).
 *   points     device memory, n interleaved float32 (x, y) pairs, 8-byte
 *              aligned, values integers in [0, 2^23).
 *   n          0 <= n <= 2^31 - 1.
 *   out_idx    device memory, room for n int32 (a hull never has more
 *              vertices than points); receives the hull vertex indices.
 *   out_count  device memory, one int32; receives the number of vertices.
 *   stream     a hipStream_t (NULL for the default stream); all device work
 *              is ordered on it.
 * Synchrony: returns after the hull is known on the host; the copies into
 * out_idx and out_count are queued on `stream`, so later work on that
 * stream sees them (synchronise the stream before reading them on the host).
 * On failure out_count is set to 0 the same way.
 * Returns CH_OK, CH_EINVAL, CH_EDOMAIN, CH_ENOMEM or CH_EHIP.
 */
int hull2d(const float* points, int64_t n, int32_t* out_idx, int32_t* out_count, void* stream);
/* (Step 7 runs on the device, across workgroups, for every polygon that
 * steps 1-6 and the pre-hull leave.  Melkman on the host remains as a
 * fallback for a polygon the device finish gives up on, which is not
 * expected; the result is the same.) */

/*
 * hull2d_async: hull2d with every step on the device and nothing
 * synchronised (Section 2.1, steps 1-7), for callers that queue several
 * hulls back to back or capture the call in a HIP graph.
 *   points, n, out_idx, stream  as in hull2d.
 *   out_count  device memory, one int32; receives, in stream order, the
 *              number of hull vertices, or CH_EDOMAIN (a coordinate out of
 *              the domain), or CH_EHIP (a failed step, or a device finish
 *              that gave up on the polygon: not expected, and hull2d
 *              computes such an input on the host).  CH_BATCH_REDO stands
 *              there only while the finish runs.
 * Returns after queueing the kernels: CH_OK, CH_EINVAL (bad argument, before
 * any work), CH_ENOMEM or CH_EHIP.  The stream's workspace (shared with
 * hull2d on that stream) is allocated or grown only when n exceeds what it
 * holds; a graph captures the call allocation-free after a first call with
 * at least as many points (under capture, a call that would allocate
 * returns CH_EINVAL).  A captured graph keeps using the workspace's
 * addresses: from the capture on, a call on that stream that would grow the
 * workspace returns CH_EINVAL, until chainhull_release_stream (or
 * chainhull_release) frees it; the graph must not be replayed after that.
 * Calls on one stream run one after another; the statistics of
 * chainhull_last_stats are not filled.
 */
int hull2d_async(const float* points, int64_t n, int32_t* out_idx, int32_t* out_count, void* stream);

/* The fixed device buffer of hull2d_noalloc: its size, and the most points a
 * call may have. */
#define CH_NOALLOC_MAX_POINTS 1048576
#define CH_NOALLOC_SCRATCH_BYTES (96u << 20)

/*
 * hull2d_noalloc: hull2d_async for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same kernels and result as hull2d_async, with
 * every intermediate array in one fixed buffer of CH_NOALLOC_SCRATCH_BYTES
 * of device memory that the library holds per device (a static device
 * array, present from the library's load on a device until the process
 * ends) instead of a per-stream workspace.  Nothing is allocated, on the
 * device or in pinned host memory, and no timing events are recorded.
 *   points, out_idx, out_count, stream  as in hull2d_async; out_count
 *              receives, in stream order, the hull size, CH_EDOMAIN or
 *              CH_EHIP as there.
 *   n          0 <= n <= CH_NOALLOC_MAX_POINTS; a larger n returns
 *              CH_ECAPACITY before any device work.
 * Every call on a device uses that device's one buffer: calls that overlap
 * on one device (on different streams, or from different threads) race and
 * corrupt each other's results; the caller serialises them.  The buffer
 * keeps the last call's contents; each call clears what it needs first.
 * The first call on a device looks up the buffer's device address (no
 * allocation).  Returns after queueing the kernels: CH_OK, CH_EINVAL (bad
 * argument), CH_ECAPACITY or CH_EHIP.
 */
int hull2d_noalloc(const float* points, int64_t n, int32_t* out_idx, int32_t* out_count, void* stream);

/*
 * hull2d_batched: num_sets independent hulls (Section 2.1 applied per set).
 *   points      device memory, the sets' points concatenated as in hull2d.
 *   offsets     host memory, num_sets + 1 non-decreasing int64 with
 *               offsets[0] == 0 and offsets[num_sets] <= 2^31 - 1; set s is
 *               points[offsets[s] .. offsets[s+1]).
 *   num_sets    >= 0.
 *   out_idx     device memory, room for offsets[num_sets] int32; set s
 *               writes its hull at out_idx + offsets[s], with indices local
 *               to the set, in the output convention above.
 *   out_counts  device memory, num_sets int32: the hull size of each set, or
 *               that set's negative ch_status if it failed (CH_EDOMAIN for a
 *               set with an out-of-domain coordinate; the other sets are
 *               still computed).
 *   stream      as in hull2d.
 * One kernel launch computes every set of at most 2^22 points, one
 * workgroup per set, all seven steps on the device.  A set beyond that
 * size, or one whose open points, sort records or chain exceed the
 * workgroup's on-chip capacities (for instance many points on the hull),
 * is then computed by the single-hull path, with the same result.
 * Blocking: returns after every count is known; the results are ordered on
 * `stream` as in hull2d.
 * Returns CH_OK if every set succeeded, else the first failing status
 * (CH_EINVAL for bad arguments, before any work).
 */
int hull2d_batched(const float* points, const int64_t* offsets, int32_t num_sets,
                   int32_t* out_idx, int32_t* out_counts, void* stream);

/* The count hull2d_batched_async reports for a set it leaves to the caller
 * (more than 2^22 points, or beyond the kernel's on-chip capacities): such a
 * set is computed with hull2d. */
#define CH_BATCH_REDO (-2147483647 - 1)

/*
 * hull2d_batched_async: the batched kernel alone, stream-ordered and
 * allocation-free, so that it can be captured in a HIP graph (Section 2.1
 * per set, every step on the device).
 *   points, out_idx  as in hull2d_batched.
 *   offsets     device memory, num_sets + 1 int64 as in hull2d_batched (they
 *               must describe `points`; a set with offsets[s+1] < offsets[s]
 *               or a negative offset gets CH_EINVAL in its count).
 *   order       device memory, num_sets int32, a permutation of the sets: the
 *               launch order (larger sets first is fastest); NULL for 0, 1, ..
 *   out_counts  device memory, num_sets int32: each set's hull size, its
 *               negative ch_status, or CH_BATCH_REDO for a set left to hull2d.
 * Returns after queueing one kernel on `stream` (nothing is synchronised or
 * allocated): CH_OK, CH_EINVAL (bad pointer or num_sets) or CH_EHIP.
 */
int hull2d_batched_async(const float* points, const int64_t* offsets, const int32_t* order, int32_t num_sets,
                         int32_t* out_idx, int32_t* out_counts, void* stream);

/* Counts and timings of the calling thread's last hull2d_batched call. */
typedef struct {
    int32_t num_sets;     /* sets in the call */
    int32_t device_sets;  /* sets given to the one-launch kernel */
    int32_t redo_sets;    /* sets computed by the single-hull path */
    int64_t points;       /* points over all sets */
    float ms_kernel;      /* the one-launch kernel, from HIP events on the call's
                             stream when timing is on (chainhull_set_timing) */
    float ms_total;       /* wall clock of the whole call */
} ch_batch_stats;

/* Copy the calling thread's last hull2d_batched counts into *out.  Returns
 * CH_OK, or CH_EINVAL for a null pointer. */
int chainhull_last_batch_stats(ch_batch_stats* out);

/*
 * chainhull_polygon: steps 1-6 only (Section 2.1): the simple polygon
 * [P_minx, R1 chain, P_miny, R2 chain, P_maxx, R3 chain, P_maxy, R4 chain]
 * (Table 1 order; consecutive coincident extreme points are dropped) that
 * step 7 takes as input.
 *   points, n, stream  as in hull2d.
 *   poly_idx    host memory, room for n + 4 int32; receives the vertices'
 *               point indices.
 *   poly_count  host memory; receives the number of polygon vertices.
 *   stats       host memory or NULL; receives the call's counts.
 * Blocking.  Returns as hull2d.
 */
int chainhull_polygon(const float* points, int64_t n, int32_t* poly_idx, int64_t* poly_count,
                      ch_stats* stats, void* stream);

/*
 * chainhull_finish_host: step 7 alone (Section 2.1.3), Melkman's convex hull
 * of a simple polygon, on the host.  Needs no GPU.
 *   poly_xy     host memory, m interleaved int32 (x, y) vertices of a simple
 *               polygon in counter-clockwise order, coordinates in [0, 2^23).
 *   poly_idx    host memory, m int32: the point index of each vertex.
 *   m           number of vertices, >= 0.
 *   out_idx     host memory, room for m int32; receives the hull in the
 *               output convention above.
 *   out_count   host memory; receives the hull size.
 * Returns CH_OK or CH_EINVAL (null pointer, m < 0, coordinate out of range,
 * or a polygon that is not simple enough for the deque to stay valid).
 */
int chainhull_finish_host(const int32_t* poly_xy, const int32_t* poly_idx, int64_t m,
                          int32_t* out_idx, int64_t* out_count);

/* Copy the counts of the calling thread's last hull2d or chainhull_polygon
 * call into *out.  Returns CH_OK, or CH_EINVAL for a null pointer. */
int chainhull_last_stats(ch_stats* out);

/* HIP event timing of later calls: 0 off, 1 every stage (ms[0..5]), 2 only
 * steps 1-6 and the device finish as two spans (ms_pre, ms_finish: fewer
 * event records in the stream); any other nonzero value means 1.  Timing
 * adds event records to the stream; it does not change results. */
void chainhull_set_timing(int enable);

/* A static description of a ch_status value. */
const char* chainhull_strerror(int status);

/* Free every cached workspace (device and pinned host memory).  Must not be
 * called while another call is running. */
void chainhull_release(void);

/*
 * chainhull_spa_chunked: the divide-and-conquer SPA that the paper
 * implements (Section 2.2.2; its limitation, Section 4.3), for
 * discard-effectiveness experiments; the hull path runs the exact rule.
 *   k2_sorted  device memory, m uint32: one region's k2 values in its sorted
 *              order (Table 1, in the region's frame).
 *   sigma      k2 of the region's first point.
 *   chunk      subset length, >= 1: subset j is points [j*chunk, (j+1)*chunk).
 *   keep       device memory, m bytes: 1 where the point survives.
 * Each subset applies the rule of Figure 2 on its own (a point survives iff
 * its k2 is below the subset's running threshold); subset 0 starts from
 * sigma, a later subset keeps its first point and starts from it.  With
 * chunk >= m this is the exact SPA.  Stream-ordered, no synchronisation.
 * Returns CH_OK, CH_EINVAL or CH_EHIP.
 */
int chainhull_spa_chunked(const uint32_t* k2_sorted, int64_t m, uint32_t sigma, int64_t chunk, uint8_t* keep,
                          void* stream);

/* Free the cached workspace of one stream on the current device (device and
 * pinned host memory).  No call on that stream may be running, and no graph
 * that captured a call on it may be replayed afterwards (this also lifts
 * the capture's hold on the workspace's size).  Returns CH_OK (also when
 * the stream has no workspace). */
int chainhull_release_stream(void* stream);

/*
 * Launch shapes (the autotuner's knobs).  The paper fixes its block size by
 * the GPU generation and leaves the best work per thread open (Sections
 * 2.2.2, 4.3); here every shape that no LDS layout fixes is a run-time
 * choice, picked per size class by the project's autotuner
 * (paper_1508_05488_amd/autotune.py), which times the candidates on the
 * device, checks that each gives the same hulls, and stores the fastest
 * (the defaults unless a candidate is at least 2 % faster).
 * Every field must hold one of the values listed; results never depend on
 * the shape.
 */
typedef struct {
    int32_t stream_grid;     /* k_stream workgroups at most: 128, 256, 512 or 1024 */
    int32_t stream_unroll;   /* float4 loads in flight per k_stream thread: 2 or 4 */
    int32_t cand_per_row;    /* open points per k_cand workgroup (one row of the bucket
                                table each, at most 256): 1024 .. 2^20; the count of
                                open points is known on the device only, so the rows
                                follow it there */
    int32_t chain_grid;      /* k_chain workgroups at most: 64 .. 4096 */
    int32_t wide_grid;       /* k_finish_wide workgroups: 64 .. 4096 */
    int32_t batch_unroll;    /* float4 loads per thread and round in the batched kernel: 1 or 2 */
    int32_t batch_order;     /* batched launch order: 0 larger sets first, 1 as given */
    int32_t serve_batch_max; /* serving: requests of at most this many points are
                                batched (0 .. 2^22); read when a server is created */
    int32_t fused_max;       /* hull2d, hull2d_async, hull2d_noalloc: inputs of at
                                most this many points run every step in one
                                workgroup of the batched kernel first (0 .. 2^22;
                                0: never); the single-hull kernels then run only
                                for an input it leaves (queued behind it and
                                returning at once otherwise) */
    int32_t list_max;        /* hull2d, hull2d_async, hull2d_noalloc: when the pass
                                over the points leaves at most this many open
                                points (0 .. 8192; 0: never), one workgroup of the
                                batched kernel takes every later step from its
                                lists; the later single-hull kernels then return at
                                once (decided on the device) */
} ch_tuning;

/* Use *t for calls whose point count (for hull2d_batched: total points) is
 * at most n_max.  The table holds up to 16 such classes; a call takes the
 * class with the smallest n_max >= its n, else the defaults.  n_max < 0
 * clears the table (t may then be NULL).  Must not run while another call
 * is being set up.  Returns CH_OK or CH_EINVAL (a field out of range, or the
 * table is full). */
int chainhull_set_tuning(int64_t n_max, const ch_tuning* t);

/* The shapes a call with n points would use; n < 0: the defaults.  Returns
 * CH_OK or CH_EINVAL for a null pointer. */
int chainhull_get_tuning(int64_t n, ch_tuning* out);

/* Upper bound on the device workspace bytes a call with n points needs. */
size_t chainhull_workspace_bytes(int64_t n);

/*
 * Serving: hull requests of mixed sizes that arrive over time, computed with
 * continuous batching on the device that is current at creation (Section
 * 2.1 per request; the result of a request is exactly hull2d's for it
 * alone, whatever else is in flight).
 *
 * Worker threads, each with its own stream, take the oldest pending work
 * when free: a request of more than serve_batch_max points (the tuned launch
 * shape in force when the server is created; 2^18 by default) alone through
 * the single-hull path, or every pending smaller request together (gathered
 * into the worker's staging buffer and computed by one hull2d_batched
 * launch).  Requests that arrive while others run join the next batch; the
 * workers' streams overlap on the device.
 *
 * Admission: a request holds part of mem_budget from submission until it
 * completes (12 bytes per point when it is batched, the single-hull
 * workspace bound otherwise); requests are admitted first come, first
 * served, as budget frees up.  The device memory a worker keeps between
 * requests (its stream's workspace, its staging buffers) counts against
 * the same budget: a worker releases it after a request when the requests
 * in flight and the workers' memory would otherwise exceed the budget.
 */
typedef struct ch_server ch_server;

typedef struct {
    int64_t completed;         /* requests finished */
    int64_t batches;           /* batched launches */
    int64_t batched_requests;  /* requests computed in batched launches */
    int64_t single_requests;   /* requests computed alone */
    int64_t points;            /* points of the finished requests */
    int64_t pending;           /* requests submitted and not started */
    int32_t max_inflight;      /* most requests running at once */
    int32_t reserved0;
    uint64_t reserved_bytes;   /* budget held by admitted requests now */
} ch_server_stats;

/* Create a server with `workers` (1..16) worker threads and streams and a
 * memory budget in bytes (> 0).  *out receives it.  Returns CH_OK,
 * CH_EINVAL or CH_EHIP. */
int chainhull_server_create(int32_t workers, size_t mem_budget, ch_server** out);

/* Submit one request.  points: device memory, n float32 (x, y) pairs as in
 * hull2d, 8-byte aligned, written completely before the call (the workers'
 * streams are not ordered after any stream of the caller's) and unchanged
 * until the request completes; out_idx
 * (room for n int32) and out_count (one int32): device memory that receives
 * the hull as hull2d writes it.  *ticket receives the request's ticket.
 * Returns at once: CH_OK, CH_EINVAL (bad argument, or the server is being
 * destroyed), or CH_EADMIT (the request alone exceeds the budget). */
int chainhull_server_submit(ch_server* s, const float* points, int64_t n, int32_t* out_idx, int32_t* out_count,
                            uint64_t* ticket);

/* Block until the request completes; its outputs are then written.  *hull
 * (if not NULL) receives the hull size, *latency_ms (if not NULL) the time
 * from submission to completion.  A ticket can be waited for once (by one
 * thread).  Returns the request's ch_status, or CH_EINVAL for an unknown
 * ticket or one that another thread is waiting for.  submit, wait and stats
 * may be called from any threads concurrently. */
int chainhull_server_wait(ch_server* s, uint64_t ticket, int32_t* hull, double* latency_ms);

/* Copy the server's counters into *out.  Returns CH_OK or CH_EINVAL. */
int chainhull_server_stats(ch_server* s, ch_server_stats* out);

/* Finish every submitted request, stop the workers and free the server.
 * Requests not yet waited for are discarded (their outputs are written).  No
 * other call on the server may run during or after it.  Returns CH_OK or
 * CH_EINVAL. */
int chainhull_server_destroy(ch_server* s);

#ifdef __cplusplus
}
#endif

#endif /* CHAINHULL_H */
