// Internal types shared by the host engine and the gfx950 kernels.
//
// Data layout in HBM (all positions are "global positions": request i owns
// positions [off_i, off_i + n_i) of the caller's x/y arrays, of both workspace
// buffers and of out_idx):
//   - two ping-pong workspace buffers, each structure-of-arrays
//     {x: double[N], y: double[N], idx: uint32[N]} (20 bytes per point);
//     idx is the point's index local to its request;
//   - per level: a segment table (one row per live subproblem with more points
//     than the LDS finisher takes), a tile -> segment map, one packed 64-bit
//     counter per segment and one candidate record per tile;
//   - a node table (one node per emitted vertex outside the LDS finisher)
//     from which the clockwise order is assembled at the end.
#pragma once
#include <stdint.h>

namespace vqh {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int64_t kCountNonfinite = -3;  // the count of a request with a NaN or infinity (-VQHULL_ERR_NONFINITE)
constexpr int64_t kCountIncomplete = -6;  // a stream-ordered call's level budget ended first (-VQHULL_ERR_INCOMPLETE)

// Source of a finisher job's points.
enum : uint32_t { kSrcBufA = 0, kSrcBufB = 1, kSrcUser = 2 };

struct Req {
  uint32_t off;     // global position of the request's point 0
  uint32_t n;       // number of points
  uint32_t p, q;    // local indices of the lexicographic extremes
  int32_t root;     // root node (vertex q), -1 if none
  uint32_t err;     // set to 1 by a kernel that sees a non-finite coordinate
  uint32_t tile0;   // first extremes tile of this request
  uint32_t pad;
  // The request's own coordinate arrays: its point j is (x[j], y[j]).  The
  // kernels that read the caller's points take them from here, so requests
  // need not sit in one array (the server's lanes read them where they are).
  const double* x;
  const double* y;
};

// A live subproblem Hull(P, a, r, b): P is the point range [beg, beg + cnt) of
// the level's input buffer.  At level 0 the input is the caller's arrays and
// the index of a point is its position minus ibase.
struct Seg {
  double ax, ay, rx, ry, bx, by;
  uint32_t beg, cnt;
  uint32_t tile0;   // first tile of this segment in the level's tile map (and its first record slot)
  uint32_t req;
  int32_t node;     // node of r
  uint32_t ibase;
  uint32_t rtiles;  // tiles whose records hold this segment's candidates (0: ceil(cnt / tile))
  uint32_t rside;   // which record array (fused level: the side of the root it came from)
};

// The fused pass classifies every point of a root twice: against the root's
// triangle (p, q, p) and then against the triangle of the child it falls in.
// A child swept at the next level is "virtual": its points are never written;
// its own children (the root's grandchildren) are.  A child small enough for
// the LDS finisher is "pass-through": its points are copied into its range.
// A level pair does the same below the top: a segment (a, r, b) whose level
// was swept without writing is read again and classified against (a, r, b),
// then against its child (a, r1, r) or (r, r2, b).
enum : uint32_t { kFuseSkip = 0, kFuseSplit = 1, kFuseCopy = 2 };

struct FusedRoot {
  double px, py, qx, qy;  // the segment's a and r (a root's extreme points p and q)
  double bx, by;          // the segment's b (a root: p again)
  double rx[2], ry[2];    // farthest point of each child: child 0 = (a, r1, r) holds S1, child 1 = (r, r2, b) S2
  uint32_t beg[2], cnt[2];  // child ranges in the output buffer
  uint32_t kind[2];         // kFuse*
  uint32_t slot[2];         // kFuseSplit: next-level segment id; kFuseCopy: job id
  uint32_t off, n;          // the root's points in the caller's arrays
  uint32_t tile0, req;
};

// Farthest-point candidate: key = orient value for the edge, then (x, y, i)
// break ties.  i == kNone marks "no candidate".
struct Cand {
  double k, x, y;
  uint32_t i, pad;
};

struct TilePart {
  Cand c[2];
};

struct ExtPart {
  double minx, miny, maxx, maxy;
  uint32_t mini, maxi;  // local indices (kNone: empty)
  uint32_t pad[2];
};

// A subproblem small enough to finish inside one workgroup's LDS.
struct Job {
  double ax, ay, rx, ry, bx, by;
  uint32_t ri;      // local index of r
  uint32_t beg, cnt;
  uint32_t src;     // kSrcBufA / kSrcBufB / kSrcUser
  uint32_t req;
  int32_t node;     // node of r; receives the size and location of the finished list
  uint32_t ibase;   // kSrcUser: global position of local index 0
  uint32_t pad;
};

struct Node {
  uint32_t vertex;  // local index of the vertex
  int32_t c[2];     // child nodes for the S1 / S2 sides, -1 if none
  uint32_t size;    // vertices in the subtree
  uint32_t start;   // output position of the subtree's first vertex
  uint32_t req;
  uint32_t list;    // finished-in-LDS subtree: global position of its ordered list, else kNone
  uint32_t lbuf;    // which workspace idx array holds that list (0 = A, 1 = B)
};

// What a planning kernel produces for the level it creates.  The kernels of
// that level read their work counts from it on the device, so the host can
// enqueue a level before it knows them; the host reads it back one level later.
struct Status {
  uint32_t nseg;        // segments of the level
  uint32_t ntiles;      // sweep tiles of the level
  uint32_t njobs;       // finisher jobs created by the plan
  uint32_t nnodes;      // node count after the plan
  uint32_t swept;       // points in the level's segments
  uint32_t jobpts;      // points in the jobs created
  uint32_t survivors;   // points the previous sweep kept (|S1| + |S2| summed over its segments)
  uint32_t overflow;    // 1 if the node table was too small (nothing was created)
};

// A level planner works in rounds of one segment per thread; several
// planner workgroups take the rounds of a level in turn and find where each
// round's output goes by a decoupled look-back over the rounds before it: a
// round publishes its own totals (flag 1), then, once the totals of all
// earlier rounds are known, its inclusive totals (flag 2).  Counters:
// nodes, jobs, segments, tiles, swept points, job points, survivors.
constexpr int kPlanCounters = 7;
struct PlanRound {
  uint32_t flag;
  uint32_t agg[kPlanCounters];
  uint32_t incl[kPlanCounters];
  uint32_t pad;
};
constexpr uint32_t kPlanners = 8;        // planner workgroups of a level planner launch
constexpr uint32_t kPlanRoundMin = 256;  // the smallest round (segments per planner workgroup)

constexpr int kStatusRing = 4;

// The host's copy of a status record, written by the planner straight into
// pinned host memory: one 64-bit word per field, (tag << 32) | value, each a
// relaxed system-scope store.  The host knows the record is whole when every
// word carries the tag it gave that level, so the device needs no
// system-scope fence (which would write back the whole L2) and the stream no
// event between the levels.  Word order: the fields of Status in order.
constexpr int kStatusWords = 8;
// Segment and job counters (packed S1 | S2 << 32 reservations) sit one
// 128-byte line apart: the device-scope atomics of one line are serialised,
// and the two children of a segment take theirs from every tile.
constexpr size_t kCtrStride = 16;

// ----------------------------------------------------------------- launchers
// Host engine contexts (vqhull_engine.cpp): one hull computation at a time
// runs on a context (device workspace, pinned staging, status ring).  Status
// values are VQHULL_*; streams are hipStream_t.
struct Context;
int context_create(Context** out);  // on the current device
void context_destroy(Context* c);
// Allocate the workspace for batches of up to npoints points in nreq requests.
int context_reserve(Context* c, int64_t npoints, int64_t nreq, void* stream);
// vqhull_hull_batched on this context (arguments already validated).
int context_run(Context* c, const double* x, const double* y, const int64_t* offsets, int64_t nreq,
                int64_t* out_idx, int64_t* out_counts, void* stream);
const char* context_last_error();  // of the calling thread

// Fixed launch sequence for graph capture.  context_stage fills the
// context's pinned tables for a batch (host only), request i at offsets[i]
// with its own coordinate arrays xs[i], ys[i] (the kernels read the requests
// where they are; x and y passed to context_enqueue_fixed are not read for
// them); context_enqueue_fixed
// enqueues copies of those tables and `levels` recursion levels with grids
// sized for the reserved capacity (context_reserve with the same levels):
// no allocation, no host wait, the same launches for every batch.  Once the
// stream has finished, context_fixed_done says whether the recursion ended
// within `levels` levels without a table overflow; if not, the batch must be
// recomputed with context_run.
int context_reserve_fixed(Context* c, int64_t npoints, int64_t nreq, int levels, void* stream);
int context_stage(Context* c, const int64_t* offsets, int64_t nreq, const double* const* xs,
                  const double* const* ys);
int context_enqueue_fixed(Context* c, const double* x, const double* y, int64_t* out_idx, int64_t* out_counts,
                          int levels, void* stream);
bool context_fixed_done(Context* c, int levels);
// Changes whenever any context's workspace buffer is reallocated.
uint64_t allocation_generation();

// Counts that depend on the batch.  The kernels read them from device memory,
// so one launch sequence (grids sized for the largest batch) serves every
// batch; workgroups past a count exit at once.
struct BatchCounts {
  uint32_t nreq;       // requests
  uint32_t ext_tiles;  // tiles of the extremes pass
  uint32_t overflow;   // set by a planner whose node table was too small
  uint32_t pad;
};

struct ExtremesArgs {
  const double* x;
  const double* y;
  const uint32_t* tile_req;  // nullptr: single request 0
  Req* req;
  ExtPart* part;
  const BatchCounts* counts;
  uint32_t ntiles;  // grid (>= counts->ext_tiles)
};

// Sweep modes.  The *Ws forms are the top-level passes over the workspace
// copy the octagon prefilter leaves (buffer A, with an index array) instead of
// the caller's arrays.  The *Pair forms are a level pair below the top: the
// level's segments swept without writing (sizes and farthest points of their
// children), then swept again, writing their grandchildren.
enum : int {
  kSweepLevel = 0,
  kSweepArgmax = 1,
  kSweepFused = 2,
  kSweepArgmaxWs = 3,
  kSweepFusedWs = 4,
  kSweepArgmaxPair = 5,
  kSweepFusedPair = 6
};
constexpr int kSweepModes = 7;

// ------------------------------------------------------- octagon prefilter
// A variant of the method (Section 6's Akl-Toussaint heuristic): every
// request with more points than the LDS threshold first drops the points
// strictly inside the octagon of eight directional extremes (with a margin
// above the rounding error of the edge test); Algorithm 1 then runs unchanged
// on the points kept, which sit compacted at the front of the request's range
// of buffer A.
//
// Per extremes tile: minimum and maximum of y, fl(x - y) and fl(x + y), each
// with the lowest local index among equal values (kNone: empty).
struct OctPart {
  double mn[3], mx[3];
  uint32_t imn[3], imx[3];
};

// Per request: the origin o (= p) and the eight edges, edge i with direction
// (ex_i, ey_i) and threshold t_i; a point u is dropped iff
// fl(fl(ex_i * fl(u.y - o.y)) - fl(ey_i * fl(u.x - o.x))) > t_i for all eight.
// on = 0: the request does not go through the filter (it is read from the
// caller's arrays); keep_all = 1: it goes through but drops nothing (the
// filter writes every point straight to its place in buffer A).
struct OctEdges {
  double ox, oy;
  double ex[8], ey[8], t[8];
  uint32_t on, keep_all;
};

struct OctArgs {
  const double* x;
  const double* y;
  const double* xy;  // interleaved input (x0, y0, x1, y1, ...), or nullptr: x and y
  const uint32_t* tile_req;  // nullptr: single request 0
  Req* req;
  ExtPart* part;   // the lexicographic extremes, as the plain extremes pass writes them
  OctPart* opart;
  const BatchCounts* counts;
  uint32_t ntiles;  // grid (>= counts->ext_tiles)
};

struct FilterArgs {
  const double* x;
  const double* y;
  const double* xy;    // interleaved input, or nullptr
  const uint32_t* tile_req;
  const Req* req;
  const ExtPart* part;
  const OctPart* opart;
  OctEdges* oct;       // per request
  double* sx;          // staging (buffer B): each tile's kept points at the tile's own start
  double* sy;
  uint32_t* si;
  double* cx;          // compacted (buffer A): the request's kept points at its start
  double* cy;
  uint32_t* ci;
  uint32_t* tcount;    // kept points per extremes tile
  uint32_t* toff;      // exclusive prefix of tcount over all tiles (ext_tiles + 1 entries)
  const BatchCounts* counts;
  uint32_t ntiles;     // grid of the per-tile kernels (>= counts->ext_tiles)
  uint32_t min_points; // requests with more points go through the filter
  uint32_t drop_min;   // ... and may drop points if they have more than this many
};

struct SweepArgs {
  const double* ix;  // level input (caller arrays for the argmax and fused passes)
  const double* iy;
  const uint32_t* ii;  // level input indices (normal levels)
  double* ox;
  double* oy;
  uint32_t* oi;
  const Seg* seg;       // normal levels and the argmax pass
  const FusedRoot* fr;  // fused pass
  const uint32_t* tile_seg;
  unsigned long long* ctr;   // per segment (normal, argmax) or per next-level segment (fused)
  unsigned long long* jctr;  // fused pass: per pass-through job
  TilePart* part;   // records, at slot tile0 + (tile - tile0) % gridDim
  TilePart* part2;  // fused pass: records of the side-1 children
  Req* req;
  const Status* st;  // ntiles of this level
  uint32_t reverse;
};

struct Plan0Args {
  Req* req;
  BatchCounts* counts;
  uint32_t* level_nodes;  // node count after each level: [0] = 0, [1] = after the roots
  const ExtPart* epart;
  Seg* seg_out;
  unsigned long long* ctr_out;
  uint32_t* tile_seg_out;
  Job* jobs;
  Node* nodes;
  uint32_t node_cap;
  Status* st_out;
  uint64_t* st_host;  // tagged host words of *st_out (kStatusWords, pinned, device view), or null
  uint32_t st_tag;    // the tag of those words
  uint32_t tile;
  uint32_t lds_limit;
  uint32_t ext_tile;
  const uint32_t* toff;  // octagon prefilter: kept-point prefix per extremes tile (nullptr: off)
  uint32_t filter_min;   // requests with more points went through the filter
  PlanRound* rounds_next;  // look-back records of the level-0 planner, cleared here
  uint32_t rounds_cap;     // records per buffer
};

struct PlanArgs {
  const Seg* seg;
  const unsigned long long* ctr;
  const TilePart* part;
  const TilePart* part2;   // record array of segments with rside = 1
  uint32_t fuse;           // 1: plan the roots for the fused pass (children become virtual / pass-through)
  FusedRoot* fr_out;       // fused roots (fuse = 1)
  unsigned long long* jctr_out;  // pass-through job counters (fuse = 1)
  const Status* st_in;  // the level being planned (nseg, nnodes)
  uint32_t sweep_grid;  // workgroups of the sweep that produced `part`
  Seg* seg_out;
  unsigned long long* ctr_out;
  uint32_t* tile_seg_out;
  Job* jobs;
  Node* nodes;
  uint32_t node_cap;
  uint32_t out_buf;  // buffer the children were written to (0 = A, 1 = B)
  Status* st_out;
  uint64_t* st_host;  // tagged host words of *st_out (kStatusWords, pinned, device view), or null
  uint32_t st_tag;    // the tag of those words
  uint32_t tile;
  uint32_t lds_limit;
  uint32_t* level_nodes;  // [level + 2] = node count after this plan
  uint32_t level;
  BatchCounts* counts;    // overflow flag
  uint32_t planners;      // workgroups 0 .. planners-1 of the launch plan; the others finish jobs
  PlanRound* rounds;      // this planner's look-back records (cleared by the planner before it)
  PlanRound* rounds_next; // the next level planner's, cleared here
  uint32_t rounds_cap;    // records per buffer
};

struct FinishArgs {
  const Status* st;  // njobs
  const Job* jobs;
  const double* ux;  // caller arrays of root jobs, by global position (when req_arrays is 0)
  const double* uy;
  const double* bx[2];
  const double* by[2];
  uint32_t* bi[2];
  Node* nodes;
  Req* req;
  uint32_t req_arrays;  // 1: root jobs read the request's own arrays (Req::x, Req::y)
};

// One request of at most the LDS threshold's points, whole in one workgroup.
struct SmallArgs {
  const double* x;
  const double* y;
  uint32_t n;
  int64_t* out_idx;
  int64_t* out_count;
  uint32_t* list;  // n entries of workspace: the finisher's ordered list
  Node* node;      // one node of workspace
  Req* req;        // one request record of workspace
};

struct AssembleArgs {
  Node* nodes;
  const uint32_t* level_begin;  // node level boundaries, nlevels + 1 entries (device)
  uint32_t nlevels;
  Req* req;
  const BatchCounts* counts;
  const uint32_t* lists[2];
  int64_t* out_idx;
  int64_t* out_count;
  uint32_t max_nodes;  // bound on level_begin[nlevels] (sizes k_copy_lists' grid)
  // Stream-ordered calls: the status of the level after the last enqueued
  // one.  If it still has segments or jobs (or a table overflowed), every
  // request is marked incomplete and no list is written.  Null otherwise.
  const Status* last;
};

// Supported sweep shapes.
bool sweep_shape_supported(int block, int ppt);
int finish_tmax_for(int lds_limit);

// Launchers (return hipError_t as int).
int launch_extremes(const ExtremesArgs& a, void* stream);
int launch_sweep(const SweepArgs& a, int mode, int block, int ppt, uint32_t grid, void* stream);
uint32_t sweep_grid(int block, int ppt, int mode);  // persistent grid size for a sweep shape and mode
uint32_t finish_grid(int tmax);            // persistent grid size of the finisher
int launch_plan0(const Plan0Args& a, void* stream);
// The finisher of level k and the planner of level k in one launch.
int launch_finish_plan(const FinishArgs& a, const PlanArgs& p, int tmax, void* stream);
// A whole request of n <= tmax points in one workgroup (extremes, Algorithm 1
// in LDS, output in clockwise order).
int launch_small(const SmallArgs& a, int tmax, void* stream);
// Octagon prefilter: extremes in eight directions (instead of
// launch_extremes), the per-request edges, the per-tile filter into staging,
// the prefix of the kept counts, and the compaction into buffer A.
int launch_octagon(const OctArgs& a, void* stream);
int launch_oct_plan(const FilterArgs& a, uint32_t nreq, void* stream);
int launch_filter(const FilterArgs& a, void* stream);
int launch_filter_scan(const FilterArgs& a, void* stream);
int launch_compact(const FilterArgs& a, void* stream);
// Interleaved input without the prefilter: xy[0..2n) -> x[0..n), y[0..n)
// (k_ingest: per extremes tile, with the tile's lexicographic extremes
// record, in place of launch_extremes).
struct IngestArgs {
  const double* xy;
  double* x;
  double* y;
  const uint32_t* tile_req;
  Req* req;
  ExtPart* part;
  const BatchCounts* counts;
  uint32_t ntiles;
};
int launch_ingest(const IngestArgs& a, void* stream);
int launch_deinterleave(const double* xy, double* x, double* y, uint64_t n, void* stream);
int launch_assemble(const AssembleArgs& a, void* stream);
int launch_copy_lists(const AssembleArgs& a, void* stream);
int launch_stream_scale(const double* in, double* out, uint64_t n, double s, void* stream);
// The orientation predicate on n triples (abc: 6 doubles per triple; out: 2
// doubles per triple, the two forms the kernels evaluate).
int launch_orient(const double* abc, uint64_t n, double* out, void* stream);

// Batching server: a request as the caller handed it in, placed at batch
// offset off; a chunk is at most kServeChunk consecutive points of a request
// (every request with n > 0 has ceil(n / kServeChunk) chunks, n = 0 has one).
constexpr uint32_t kServeChunk = 4096;
struct ServedReq {
  const double* x;
  const double* y;
  int64_t* out_idx;
  int64_t* out_count;
  uint64_t off, n;
};
struct ServedChunk {
  uint32_t req, beg;
};
// grid workgroups, of which the first *nchunks (device) have a chunk.
int launch_gather(const ServedReq* reqs, const ServedChunk* chunks, const uint32_t* nchunks, uint32_t grid, double* dx,
                  double* dy, void* stream);
int launch_scatter(const ServedReq* reqs, const ServedChunk* chunks, const uint32_t* nchunks, uint32_t grid,
                   const int64_t* idx, const int64_t* counts, void* stream);

constexpr int kExtBlock = 256;
constexpr int kExtPPT = 16;
constexpr int kExtIter = 4;
constexpr uint32_t kExtTile = kExtBlock * kExtPPT * kExtIter;

}  // namespace vqh
