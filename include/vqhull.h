/*
 * vqhull.h -- C ABI of the MI355X (gfx950) planar Quickhull library.
 *
 * The library computes the vertices of the convex hull of planar point sets,
 * in clockwise order, by the recursive partition of Quickhull (VQhull paper,
 * Section 2.1, Algorithm 1): the leftmost point p and rightmost point q split
 * the points into those left of p->q and those left of q->p; each subset
 * keeps only the points outside the triangle formed with its farthest point,
 * recursively.  The pass that dominates the run time -- classify every point of
 * every live subproblem against two edges, find the farthest point of each
 * side, and extract the two subsets (Section 3 "Subset Extraction", Section 4
 * "Bandwidth considerations") -- runs as one fused HIP kernel per level over
 * all live subproblems.
 *
 * Results (what is computed, exactly):
 *   - orient(a,b,c) = (a.x-c.x)*(b.y-c.y) - (a.y-c.y)*(b.x-c.x), each operation
 *     rounded to nearest binary64, never fused; "u left of a->b" is
 *     orient(a,b,u) > 0 (Section 2.1, the left-of inequality).
 *   - the farthest point of a subset is the maximum of the key orient(a,b,u)
 *     for its edge a->b; ties go to the smaller x, then the smaller y, then
 *     the lower index (Section 2.1, the farther-than comparison, read as this
 *     total order).
 *   - p = lexicographic minimum of (x, y, index); q = lexicographic maximum of
 *     (x, y), lowest index among equal points.
 *   - a point left of both p->r and r->q (possible only under rounding) goes to
 *     the first subset; points on an edge are dropped.
 *   - output: [p] ++ Hull(S1,p,r1,q) ++ [q] ++ Hull(S2,q,r2,p) with
 *     Hull(P,a,r,b) = Hull(S1,a,r1,r) ++ [r] ++ Hull(S2,r,r2,b): clockwise from
 *     p with y pointing up.  Only the vertices Algorithm 1 emits are listed,
 *     each once, as 0-based indices into the request's own arrays.
 *   - n = 0 gives 0 vertices; all points equal gives [p]; all points on one
 *     line gives [p, q].
 *   The output depends only on the multiset of (x, y, index) triples, not on
 *   the order of work inside the GPU, so it is identical from run to run and
 *   identical for a request alone or inside a batch.
 *
 * Conventions:
 *   - Array arguments are DEVICE pointers on the current HIP device unless
 *     stated otherwise.  x and y are read-only and must stay unmodified until
 *     the call's stream work has completed.
 *   - Calls are stream-ordered.  The hull calls synchronize the given stream
 *     internally between levels (they read small level counters back to the
 *     host), so they return after the result has been written; the results are
 *     then visible to later work on the same stream.  The exception is
 *     vqhull_hull_batched_async, which enqueues a fixed budget of levels and
 *     returns at once.
 *   - vqhull_hull, vqhull_hull_batched and the _xy calls use the library's own
 *     device workspace (about 40 bytes per input point plus small tables), one
 *     cache per device, grown on demand and guarded by a mutex: concurrent
 *     calls from several host threads are serialized per device.
 *     vqhull_release_workspace() frees it.  The _ws, _inplace and _async calls
 *     take the caller's workspace instead (and run concurrently on different
 *     streams); vqhull_hull_noalloc uses a static array of the library.
 *   - Errors detectable on the host return at once with a status and enqueue
 *     no work.  A NaN or infinity in a request's input is detected on the
 *     device: that request's count is set to -VQHULL_ERR_NONFINITE and its
 *     index list is unspecified; the call itself returns VQHULL_OK.
 */
#ifndef VQHULL_H
#define VQHULL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VQHULL_OK = 0,
  VQHULL_ERR_INVALID_ARGUMENT = 1, /* null pointer, negative size, bad offsets, n >= 2^31 */
  VQHULL_ERR_OUT_OF_MEMORY = 2,    /* device workspace could not be allocated */
  VQHULL_ERR_NONFINITE = 3,        /* a NaN or infinity in the input (reported per request) */
  VQHULL_ERR_HIP = 4,              /* a HIP runtime call failed; see vqhull_last_error() */
  VQHULL_ERR_TIMEOUT = 5,          /* vqhull_server_wait_timeout: the request was not done in time */
  VQHULL_ERR_INCOMPLETE = 6        /* vqhull_hull_batched_async: the level budget ended before the
                                      recursion did (reported per request) */
} vqhull_status;

/* Stream handle: a hipStream_t passed as an opaque pointer (NULL = the default
 * stream), so that this header does not need the HIP headers. */
typedef void* vqhull_stream_t;

/*
 * Hull of one point set (Algorithm 1 on x[0..n), y[0..n)).
 *   x, y       device arrays of n binary64 coordinates (structure of arrays).
 *   n          number of points, 0 <= n < 2^31.
 *   out_idx    device int64 array with room for n entries (1 if n = 0); on
 *              return out_idx[0..h) holds the hull vertices, clockwise from p.
 *   out_count  device int64 scalar: h >= 0, or -VQHULL_ERR_NONFINITE.
 *   stream     HIP stream the work is ordered on.
 * Returns VQHULL_OK, or an error status with nothing enqueued.
 */
int vqhull_hull(const double* x, const double* y, int64_t n, int64_t* out_idx, int64_t* out_count,
                vqhull_stream_t stream);

/*
 * Hulls of nreq independent point sets in one pass (the batched form of
 * Algorithm 1: every level of every request is processed by the same kernel
 * launches).
 *   x, y       device arrays holding all requests back to back.
 *   offsets    HOST array of nreq+1 non-decreasing int64 values, offsets[0] = 0;
 *              request i owns x[offsets[i] .. offsets[i+1]).  The total
 *              offsets[nreq] must be below 2^31.
 *   nreq       number of requests, >= 0.
 *   out_idx    device int64 array of offsets[nreq] entries (at least 1);
 *              request i writes its vertex list to out_idx[offsets[i] ..), as
 *              indices local to the request (0 .. n_i-1).
 *   out_counts device int64 array of nreq entries: h_i, or -VQHULL_ERR_NONFINITE.
 * The result of each request equals that of vqhull_hull on its points alone.
 */
int vqhull_hull_batched(const double* x, const double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
                        int64_t* out_counts, vqhull_stream_t stream);

/*
 * The same two calls for interleaved input, the array-of-structures layout
 * (x0, y0, x1, y1, ...) of the paper's benchmark inputs (Section 5.2).
 *   xy         device array of 2n binary64 values, 16-byte aligned (one
 *              double2 per point); x_i = xy[2i], y_i = xy[2i+1].
 * Every other argument, the result and the errors are those of vqhull_hull /
 * vqhull_hull_batched on the same points (the same index lists).  The points
 * are deinterleaved once into the library's workspace (8 n + 8 n bytes): a
 * plain copy of x and y, or with the octagon prefilter on, the filter pass
 * itself (which writes only the points it keeps); every later kernel reads
 * the workspace.  VQHULL_ERR_INVALID_ARGUMENT also for a misaligned xy.
 */
int vqhull_hull_xy(const double* xy, int64_t n, int64_t* out_idx, int64_t* out_count, vqhull_stream_t stream);
int vqhull_hull_batched_xy(const double* xy, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
                           int64_t* out_counts, vqhull_stream_t stream);

/*
 * Caller-owned workspace (so that every byte of device memory a hull needs can
 * come from the caller's allocator, e.g. a torch tensor).  The problem is the
 * one of Algorithm 1 (Section 2.1: given a planar point set, the vertices of
 * its convex hull in clockwise order); these calls compute exactly what
 * vqhull_hull / vqhull_hull_batched compute, with the same kernels.
 *
 * vqhull_workspace_bytes(n_total, nreq): the bytes of device workspace a
 *   _ws call with n_total points in nreq requests needs under the current
 *   configuration (vqhull_set_config may change it: query again after a
 *   change).  About 72 bytes per point: two ping-pong point buffers (x, y,
 *   index: 40 bytes per point), a node table with one 32-byte node per point
 *   (the most vertices the recursion can emit), and tables per tile, segment
 *   and request.  Returns 0 for n_total or nreq outside [0, 2^31).
 *
 * vqhull_hull_ws / vqhull_hull_batched_ws: arguments, results and errors of
 *   vqhull_hull / vqhull_hull_batched, plus
 *     workspace        device pointer, 256-byte aligned, of workspace_bytes
 *                      bytes, owned by the caller.  Its contents on entry
 *                      do not matter; on return they are unspecified.  The
 *                      library keeps no pointer into it after the call.
 *     workspace_bytes  at least vqhull_workspace_bytes(n_total, nreq) for the
 *                      call's sizes, else VQHULL_ERR_INVALID_ARGUMENT (also
 *                      for a null or misaligned workspace) with nothing
 *                      enqueued.
 *   The library allocates no device memory in these calls (host-side pinned
 *   staging and events are created once per concurrent caller and reused).
 *   Calls on different streams with different workspaces may run
 *   concurrently; one workspace must not be used by two calls at once.  Like
 *   vqhull_hull, a call returns after its result has been written.
 */
size_t vqhull_workspace_bytes(int64_t n_total, int64_t nreq);
int vqhull_hull_ws(const double* x, const double* y, int64_t n, int64_t* out_idx, int64_t* out_count,
                   void* workspace, size_t workspace_bytes, vqhull_stream_t stream);
int vqhull_hull_batched_ws(const double* x, const double* y, const int64_t* offsets, int64_t nreq,
                           int64_t* out_idx, int64_t* out_counts, void* workspace, size_t workspace_bytes,
                           vqhull_stream_t stream);

/*
 * Stream-ordered batched call: the hulls of Algorithm 1 (Section 2.1) for the
 * requests of vqhull_hull_batched_ws, enqueued on the stream with no host
 * wait; the call returns once its work is enqueued.  The recursion runs a
 * fixed budget of `levels` breadth-first levels (the top level counts as
 * two: its argmax pass and its fused pass), whose kernels read their work
 * counts from the device; levels past the end of the recursion do no work.
 *   levels     the level budget, 1 <= levels <= 4096; a disk or square of
 *              10^8 points needs about 8, a circle of 5 10^7 about 16, the
 *              worst case (points on a convex curve of growing curvature)
 *              up to the number of points.
 *   workspace, workspace_bytes  as for vqhull_hull_batched_ws (the same
 *              vqhull_workspace_bytes); the workspace and out_idx must stay
 *              untouched until the stream has finished the call's work.
 * Every other argument is that of vqhull_hull_batched_ws.  On the device,
 * out_counts[i] receives h_i, or -VQHULL_ERR_NONFINITE for a request with a
 * NaN or infinity, or -VQHULL_ERR_INCOMPLETE for every request of the call
 * when the recursion had work left after the last level of the budget (its
 * lists are then not written: run the call again with a larger budget or
 * with vqhull_hull_batched_ws, whose level loop is not bounded).  The index
 * lists of a completed call equal those of vqhull_hull_batched.
 * Returns VQHULL_OK once enqueued, VQHULL_ERR_INVALID_ARGUMENT (bad sizes,
 * offsets, level budget or workspace) with nothing enqueued, or
 * VQHULL_ERR_HIP.  The request table is staged in pinned host memory of the
 * library, which a later call reuses only once the stream has copied it
 * (with more than 32 calls on a device still waiting for their copies, a
 * call waits for the oldest one).
 * The call writes no status to the host: vqhull_last_level_stats and
 * vqhull_last_kernel_times do not cover it.
 */
int vqhull_hull_batched_async(const double* x, const double* y, const int64_t* offsets, int64_t nreq,
                              int64_t* out_idx, int64_t* out_counts, int32_t levels, void* workspace,
                              size_t workspace_bytes, vqhull_stream_t stream);

/*
 * In-place mode (the paper keeps no second copy of the points: its extraction
 * permutes them inside the input array, Section 3.1): the caller's x and y
 * are writable and serve as one of the two ping-pong point buffers, so the
 * library's point buffers take 24 bytes per point instead of 40.
 *   x, y       DEVICE arrays, overwritten: their contents after the call are
 *              unspecified (they hold intermediate subsets).  The result is
 *              the hull of the points they held on entry.
 *   workspace, workspace_bytes  as for vqhull_hull_ws, with
 *              vqhull_workspace_bytes_inplace(n_total, nreq) bytes at least.
 * Every other argument, the result and the errors are those of
 * vqhull_hull_ws / vqhull_hull_batched_ws.
 */
size_t vqhull_workspace_bytes_inplace(int64_t n_total, int64_t nreq);
int vqhull_hull_inplace(double* x, double* y, int64_t n, int64_t* out_idx, int64_t* out_count, void* workspace,
                        size_t workspace_bytes, vqhull_stream_t stream);
int vqhull_hull_batched_inplace(double* x, double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
                                int64_t* out_counts, void* workspace, size_t workspace_bytes,
                                vqhull_stream_t stream);

/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): vqhull_hull with every device table in a
 * static device array of the library, VQHULL_NOALLOC_MAX_POINTS points at
 * most (84 MiB, one copy per GPU the library runs on, held until the process
 * ends).  Arguments, result and errors are those of vqhull_hull, plus
 * VQHULL_ERR_INVALID_ARGUMENT for n > VQHULL_NOALLOC_MAX_POINTS.  The call
 * makes no hipMalloc, hipFree, pinned-memory or event allocation: levels are
 * enqueued in chunks whose kernels read their work counts from the device,
 * and the host waits on the stream once per chunk.  Calls on one GPU share its
 * array: the library runs them one at a time (a mutex per GPU), each returning
 * after its result is written, so their contents never mix; the array keeps
 * the last call's contents, which no call reads before writing.  Not for use
 * inside stream capture (the call waits on the stream).  Level statistics
 * and kernel times (vqhull_last_level_stats, vqhull_last_kernel_times) are
 * not recorded for it.
 */
#define VQHULL_NOALLOC_MAX_POINTS 1048576
int vqhull_hull_noalloc(const double* x, const double* y, int64_t n, int64_t* out_idx, int64_t* out_count,
                        vqhull_stream_t stream);

/* Tuning knobs of the hull kernels (all values are rounded to supported ones).
 * Defaults: 256 x 16 sweep shape, LDS threshold 2048, persistent sweeps, no
 * reversed tiles, deeper levels in the sweep shape, no prefilter; an
 * unsupported sweep shape becomes 256 x 16. */
typedef struct {
  int sweep_block;  /* threads per workgroup of the partition sweep: 256, 512 or 1024 */
  int sweep_ppt;    /* points per thread of the partition sweep: 8, 16 or 32 */
  int lds_limit;    /* subproblems of at most this many points finish inside one workgroup: 256..2048 */
  int reverse_tiles;/* debug: process tiles in reverse order (the result must not change) */
  int sweep_persistent; /* 1: the sweep runs as many workgroups as fit on the GPU at once, each
                           looping over tiles; 0: one workgroup per tile */
  int level_block;  /* threads per workgroup of the sweeps of recursion levels >= 2, with the same
                       tile (sweep_block x sweep_ppt points); 0 or an unsupported shape: the
                       sweep shape */
  int prefilter;    /* 1: the octagon prefilter (Section 6, the Akl-Toussaint heuristic) runs
                       first on every request of more than lds_limit points: the points
                       strictly inside the octagon of eight directional extremes (minimum and
                       maximum of x, y, x-y and x+y), with a margin above the rounding error of
                       the edge test, are dropped and Algorithm 1 runs on the rest.  Dropped
                       points lie strictly inside the hull, so in exact arithmetic the result
                       is unchanged.  vqhull_hull, vqhull_hull_batched and their interleaved
                       forms only (the server's lanes and the served tuner run the plain
                       method).  0: off (default). */
} vqhull_config;

/* Read / replace the configuration used by later calls (host pointers). */
int vqhull_get_config(vqhull_config* cfg);
int vqhull_set_config(const vqhull_config* cfg);

/*
 * Autotuner: compute the hull of x[0..n) (device arrays, 1 <= n < 2^31) under
 * every supported configuration -- sweep shapes 256x16, 256x32, 512x8, 512x16,
 * 1024x8 (deeper levels with 256-thread workgroups where that shape exists);
 * LDS thresholds 512, 1024, 2048; persistent or one workgroup per tile -- timing `repeats` runs of each (median wall time, after one warm-up run)
 * and checking that each result equals the first configuration's.  *best
 * receives the fastest configuration whose result is equal; up to cap entries
 * (host array) receive the table and *count the number of configurations
 * tried.  The library's current configuration is not changed.  Allocates
 * 8 n + 8 bytes of device memory for the duration of the call.
 */
typedef struct {
  vqhull_config cfg;
  double ms;          /* median wall time of one hull call */
  int32_t same_result;/* 1 if the index list equals the first configuration's */
  int32_t reserved;
} vqhull_tune_entry;
int vqhull_autotune(const double* x, const double* y, int64_t n, int32_t repeats, vqhull_tune_entry* entries,
                    int64_t cap, int64_t* count, vqhull_config* best, vqhull_stream_t stream);

/* Per-level statistics of the last hull call on this device (vqhull_hull,
 * vqhull_hull_batched, their interleaved and _ws forms; host pointer,
 * up to cap entries of 4 int64: live subproblems, points swept, subproblems
 * finished in LDS, points finished in LDS).  Returns the number of levels. */
int64_t vqhull_last_level_stats(int64_t* out, int64_t cap);

/* How the partition sweep of each level of the last hull call on this device
 * read and wrote its points (the calls of vqhull_last_level_stats; host
 * pointer, up to cap entries; returns the number of levels):
 *   VQHULL_SWEEP_ARGMAX  read the level's points and wrote none: the sizes and
 *                        farthest points of the children only (level 0, and
 *                        the first level of a level pair);
 *   VQHULL_SWEEP_FUSED   read the points of the level before again and wrote
 *                        this level's children (level 1, and the second level
 *                        of a pair) and copies of the points of the level
 *                        before's small children;
 *   VQHULL_SWEEP_LEVEL   read the level's points and wrote its children. */
#define VQHULL_SWEEP_LEVEL 0
#define VQHULL_SWEEP_ARGMAX 1
#define VQHULL_SWEEP_FUSED 2
int64_t vqhull_last_level_kinds(int32_t* out, int64_t cap);

/* Level pairs of vqhull_hull, vqhull_hull_batched and their interleaved and
 * _ws forms (the top level's argmax and fused passes applied below the top;
 * Algorithm 1's partition and results unchanged): a level
 * swept without writing, then the next level read in place from it, one
 * write per point instead of two.  mode 0: never; 1 (default): from the
 * fourth level on, where the level before kept more than 3/4 of the points it
 * swept (at least 2^20 of them) and the levels left whose segments exceed the
 * LDS threshold (about log2 of the average segment over the threshold, at
 * least 2) come in a whole number of pairs; 2: from the third level on, back
 * to back.
 * The server's lanes and the stream-ordered call, whose level sequences are
 * fixed before any status is known, sweep level by level.  The result does
 * not depend on the mode.  Returns VQHULL_ERR_INVALID_ARGUMENT for any other
 * mode. */
int vqhull_set_level_pairs(int mode);

/* Kernel timing of the last hull call on this device (the same calls), for benchmarks: when
 * enabled, HIP events are recorded on the call's stream around every kernel
 * launch.  Kinds: */
enum {
  VQHULL_K_EXTREMES = 0, /* leftmost / rightmost points */
  VQHULL_K_PLAN0 = 1,    /* root planning */
  VQHULL_K_SWEEP = 2,    /* fused partition sweep of one level */
  VQHULL_K_PLAN = 3,     /* planning of one level, in one launch with the LDS finisher of that
                            level's small subproblems (workgroup 0 plans, the others finish) */
  VQHULL_K_FINISH = 4,   /* one launch doing a whole single request of at most the LDS threshold's
                            points (extremes and Algorithm 1 in one workgroup's LDS) */
  VQHULL_K_ASSEMBLE = 5, /* clockwise assembly (both kernels) */
  VQHULL_K_FILTER = 6,   /* octagon prefilter: edges, filter, prefix of the kept counts (with the
                            prefilter, VQHULL_K_EXTREMES times the eight-direction extremes pass) */
  VQHULL_K_COMPACT = 7,  /* octagon prefilter: kept points moved to the front of each request */
  VQHULL_K_INGEST = 8    /* interleaved input without the prefilter: x and y copied into the workspace */
};
typedef struct {
  int32_t kind;       /* VQHULL_K_* */
  int32_t level;      /* recursion level of the launch (0 for the root) */
  double ms;          /* elapsed time between the events around the launch */
  int64_t points_in;  /* points the launch reads */
  int64_t points_out; /* points the launch writes (sweep: |S1| + |S2| over all segments) */
} vqhull_kernel_time;

/* Kernel timing of later calls: 0 off, 1 every launch, 2 the partition
 * sweeps only, 3 the fused top-level pass only (the sweep of level 1: two
 * events per call, the fewest the stream carries).  Each timed launch adds
 * two timestamped events to the stream (a few microseconds of device time).
 * VQHULL_ERR_INVALID_ARGUMENT for other values. */
int vqhull_set_timing(int enable);

/* Copy up to cap records of the last call (host pointer); returns the count. */
int64_t vqhull_last_kernel_times(vqhull_kernel_time* out, int64_t cap);

/*
 * The orientation predicate of Section 2.1 as the kernels evaluate it, on n
 * triples (for checking it against a host evaluation bit for bit).
 *   abc   device array of 6n doubles: a.x, a.y, b.x, b.y, c.x, c.y per triple.
 *   out   device array of 2n doubles: out[2i] = orient(a, b, c) =
 *         fl(fl(fl(a.x-c.x)*fl(b.y-c.y)) - fl(fl(a.y-c.y)*fl(b.x-c.x))) as the
 *         finisher and planners call it, out[2i+1] the same value in the form
 *         the partition sweeps compute (differences to c formed first).
 * Stream-ordered; VQHULL_ERR_INVALID_ARGUMENT for n < 0 or null pointers.
 */
int vqhull_orient(const double* abc, int64_t n, double* out, vqhull_stream_t stream);

/*
 * HBM probe for the bandwidth context (the paper reports bandwidth as a share
 * of the STREAM "Scale" kernel, Section 5.1): out[i] = s * in[i] for
 * i < n, one read and one write of 8 bytes per element.
 *   in, out  device arrays of n doubles (must not overlap).
 * Returns VQHULL_OK or VQHULL_ERR_INVALID_ARGUMENT; stream-ordered, no sync.
 */
int vqhull_stream_scale(const double* in, double* out, int64_t n, double s, vqhull_stream_t stream);

/* Free the cached device workspace of the current device. */
int vqhull_release_workspace(void);

/* Human-readable text of a status code (static storage). */
const char* vqhull_status_string(int status);

/* Text of the last HIP error seen by this thread (static thread-local storage). */
const char* vqhull_last_error(void);

/*
 * Continuous-batching server: the served form of the batched hull.
 *
 * Requests are submitted one at a time, each with its own device arrays, and
 * queue in arrival order.  The server runs `lanes` batch lanes; each has its
 * own HIP stream, device workspace and batch buffers, allocated once at
 * creation, and a host thread that repeatedly takes the oldest pending
 * requests that fit the lane (at most lane_points points and lane_requests
 * requests; admission by the lane's device memory), gathers them into one
 * batch, runs the batched hull on it (vqhull_hull_batched semantics), and
 * writes every request's vertex list and count to that request's buffers.
 * Requests that arrive while batches are on the GPU are taken by the next lane
 * that frees up, so the work of different batches overlaps on the device.
 * Each request's result is identical to vqhull_hull on its points alone.
 *
 * Device memory per lane is about 64 + 40 bytes per lane point plus small
 * tables.  All functions are thread-safe.  Host pointers: cfg, out, ticket,
 * tickets, info, stats.  Times are seconds on the host's steady clock since
 * the server's creation.
 */
typedef struct vqhull_server vqhull_server; /* opaque */

typedef struct {
  int32_t lanes;         /* concurrent batches (1..8), one HIP stream each */
  int32_t graph_levels;  /* 0: plain launches; L in 1..64: each lane captures its whole batch step
                            (table copies, gather, extremes, L recursion levels, assembly, scatter)
                            once as a hipGraph and replays it for every batch; a batch whose
                            recursion is deeper than L is computed again with plain launches */
  int64_t lane_points;   /* points per batch (1 .. 2^31-1); also the largest request */
  int64_t lane_requests; /* requests per batch (1 .. 2^24) */
} vqhull_server_config;

typedef struct {
  int64_t n;        /* points of the request */
  int64_t batch;    /* batch that computed it (-1 while pending or running) */
  int32_t lane;     /* lane that took it (-1 while pending) */
  int32_t status;   /* VQHULL_OK or the request's error (meaningful once done) */
  int32_t done;     /* 1 once the results are in the caller's buffers */
  int32_t reserved;
  double t_submit;  /* when vqhull_server_submit accepted it */
  double t_start;   /* when a lane took it into a batch */
  double t_done;    /* when its batch finished (results written) */
} vqhull_ticket_info;

typedef struct {
  int64_t submitted, completed, failed, batches, points, pending;
  double busy_seconds; /* summed wall time of all batches over all lanes */
  double now;          /* the server clock when the statistics were taken */
  int64_t graph_batches; /* batches finished by one replay of a lane's graph */
  int64_t plain_batches; /* batches computed with plain launches */
} vqhull_server_counters;

/* Create a server on the current device; VQHULL_ERR_INVALID_ARGUMENT for a
 * configuration out of range, VQHULL_ERR_OUT_OF_MEMORY if the lanes do not fit. */
int vqhull_server_create(const vqhull_server_config* cfg, vqhull_server** out);

/*
 * Queue one request.  x, y: device arrays of n binary64 coordinates, 0 <= n <=
 * lane_points; out_idx: device int64 array with room for n entries (may be
 * NULL when n = 0); out_count: device int64 scalar, receives h or
 * -VQHULL_ERR_NONFINITE.  The caller keeps all four valid and x, y unmodified
 * until the request is done.  *ticket receives the request's id (0, 1, 2, ...
 * in submission order).  Returns at once; no HIP call is made.
 */
int vqhull_server_submit(vqhull_server* s, const double* x, const double* y, int64_t n, int64_t* out_idx,
                         int64_t* out_count, int64_t* ticket);

/*
 * Queue count requests at once, in array order (same rules as
 * vqhull_server_submit per request).  x, y, n, out_idx, out_count are HOST
 * arrays of count entries (x[i], y[i], out_idx[i], out_count[i] being device
 * pointers); the requests get tickets *first_ticket .. *first_ticket+count-1.
 * All requests are checked before any is queued.
 */
int vqhull_server_submit_batch(vqhull_server* s, int64_t count, const double* const* x, const double* const* y,
                               const int64_t* n, int64_t* const* out_idx, int64_t* const* out_count,
                               int64_t* first_ticket);

/* Block until the request is done; returns its status (VQHULL_OK,
 * VQHULL_ERR_NONFINITE, ...) or VQHULL_ERR_INVALID_ARGUMENT for an unknown ticket. */
int vqhull_server_wait(vqhull_server* s, int64_t ticket);

/* Watchdog form of vqhull_server_wait: wait at most `seconds` (0 = look once,
 * without blocking).  Returns the request's status once done, or
 * VQHULL_ERR_TIMEOUT if it is still queued or running at the deadline.  A
 * timed-out request is not cancelled: it still completes and writes out_idx
 * and out_count, so the caller keeps those buffers (and x, y) alive until a
 * later wait, poll or drain reports it done.  VQHULL_ERR_INVALID_ARGUMENT for
 * a null server, an unknown ticket, or seconds negative, NaN or above 10^6. */
int vqhull_server_wait_timeout(vqhull_server* s, int64_t ticket, double seconds);

/* Completed tickets not returned by an earlier poll, oldest first, up to cap;
 * returns how many were written (a negative status on bad arguments). */
int64_t vqhull_server_poll(vqhull_server* s, int64_t* tickets, int64_t cap);

/* Block until every submitted request is done. */
int vqhull_server_drain(vqhull_server* s);

/* Timing and placement of one request. */
int vqhull_server_ticket_info(vqhull_server* s, int64_t ticket, vqhull_ticket_info* info);

/* Server-wide counters. */
int vqhull_server_stats(vqhull_server* s, vqhull_server_counters* stats);

/* Finish the queued requests, stop the lanes and free the server. */
int vqhull_server_destroy(vqhull_server* s);

#ifdef __cplusplus
}
#endif

#endif /* VQHULL_H */
