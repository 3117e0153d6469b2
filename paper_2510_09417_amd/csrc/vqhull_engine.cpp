// Host engine and C ABI of the gfx950 planar Quickhull.
//
// The recursion of Algorithm 1 runs breadth-first: each level is one sweep
// launch over every live segment of every request, followed by a one-workgroup
// planning kernel that lays out the next level and hands small subproblems to
// the LDS finisher.  The host reads the planner's small status record after
// each level to size the next launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/vqhull.h"
#include "vqhull_internal.h"

using namespace vqh;

static_assert(kCountNonfinite == -(int64_t)VQHULL_ERR_NONFINITE, "the kernels' count of a non-finite request");
static_assert(kCountIncomplete == -(int64_t)VQHULL_ERR_INCOMPLETE, "the kernels' count of an unfinished request");

namespace {

thread_local std::string g_last_error;

std::mutex g_cfg_mu;
vqhull_config g_cfg = {256, 16, 2048, 0, 1, 0, 0};

struct LevelStat {
  int64_t segs, swept, jobs, jobpts;
  int32_t kind;  // VQHULL_SWEEP_*: how the level's sweep read and wrote its points
};

std::atomic<int> g_timing{0};
std::atomic<int> g_pairs{1};  // level pairs: 0 off, 1 where levels keep most points, 2 from the first level sweep

struct TimedLaunch {
  int kind, level;
  int64_t in, out;
  int ev0, ev1;
};

// A device table: library-owned (grown on demand), or a fixed view into a
// caller's workspace (never reallocated or freed by the library).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  bool fixed = false;
};

}  // namespace

namespace vqh {

// One hull computation at a time runs on a context: device workspace, pinned
// staging, the status ring and timing records.  The public entry points use
// one context per device; the batching server owns one per lane.
struct Context {
  std::mutex mu;
  int device = -1;
  bool fixed = false;  // every device table is a view into a caller's workspace (the _ws calls)
  size_t cap_pts = 0;
  double* wx[2] = {nullptr, nullptr};
  double* wy[2] = {nullptr, nullptr};
  uint32_t* wi[2] = {nullptr, nullptr};
  DevBuf<Seg> seg[2];
  DevBuf<unsigned long long> ctr[2];
  DevBuf<uint32_t> tile_seg[2];
  DevBuf<TilePart> part, part2;
  DevBuf<FusedRoot> fr;
  DevBuf<PlanRound> rounds[2];  // look-back records of the level planners (level k uses rounds[k % 2])
  DevBuf<unsigned long long> jctr[2];  // by level parity, like the job tables
  DevBuf<ExtPart> epart;
  DevBuf<OctPart> opart;     // octagon prefilter: per extremes tile
  DevBuf<OctEdges> oct;      // per request
  DevBuf<uint32_t> tcount;   // kept points per extremes tile
  DevBuf<uint32_t> toff;     // their prefix (ext_tiles + 1)
  DevBuf<uint32_t> tile_req;
  DevBuf<Req> req;
  DevBuf<Job> jobs[2];  // level k's jobs in jobs[k % 2] (the planner of level k writes the other)
  DevBuf<Node> nodes;
  BatchCounts* counts_dev = nullptr;   // the batch's counts (device copy)
  BatchCounts* counts_host = nullptr;  // pinned source of that copy
  DevBuf<uint32_t> level_nodes;        // node count after each level (written by the planners)
  Status* status_dev = nullptr;   // kStatusRing records
  Status* status_host = nullptr;  // pinned copies, read back by copies on the stream (server lanes)
  uint64_t* status_words = nullptr;      // pinned tagged words of the status ring, written by the planners
  uint64_t* status_words_dev = nullptr;  // device view of status_words (null: the planners write none)
  uint32_t status_tag = 0;               // the last tag given to a level
  hipEvent_t staged = nullptr;  // stream-ordered calls: recorded after the copies of the host staging
  // pinned staging
  Req* h_req = nullptr;
  size_t h_req_cap = 0;
  uint32_t* h_u32 = nullptr;
  size_t h_u32_cap = 0;
  std::vector<LevelStat> stats;
  // kernel timing
  std::vector<hipEvent_t> events;
  int next_event = 0;
  std::vector<TimedLaunch> launches;
  std::vector<vqhull_kernel_time> times;
};

}  // namespace vqh

namespace {

std::mutex g_ws_mu;
std::map<int, Context*> g_ws;

struct HipFail {
  hipError_t e;
};

// A caller's workspace is too small for what a call needs.
struct WorkspaceTooSmall {};

inline void ck(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    throw HipFail{e};
  }
}

inline void ck(int e, const char* what) { ck((hipError_t)e, what); }

// Bumped whenever a workspace buffer moves: launch sequences captured in a
// graph hold buffer addresses and must be captured again.
std::atomic<uint64_t> g_alloc_gen{0};

template <typename T>
void ensure(DevBuf<T>& b, size_t n, hipStream_t st, bool keep = false) {
  if (n <= b.cap) return;
  if (b.fixed) {
    g_last_error = "the caller's workspace is too small for this call";
    throw WorkspaceTooSmall{};
  }
  g_alloc_gen.fetch_add(1);
  size_t cap = std::max<size_t>(n, b.cap + b.cap / 2);
  T* p = nullptr;
  ck(hipMalloc(&p, cap * sizeof(T)), "hipMalloc");
  if (b.p) {
    if (keep) ck(hipMemcpyAsync(p, b.p, b.cap * sizeof(T), hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    ck(hipStreamSynchronize(st), "hipStreamSynchronize");
    ck(hipFree(b.p), "hipFree");
  }
  b.p = p;
  b.cap = cap;
}

void ensure_points(Context& w, size_t n, hipStream_t st) {
  if (n <= w.cap_pts) return;
  if (w.fixed) {
    g_last_error = "the caller's workspace is too small for this call";
    throw WorkspaceTooSmall{};
  }
  g_alloc_gen.fetch_add(1);
  ck(hipStreamSynchronize(st), "hipStreamSynchronize");
  for (int k = 0; k < 2; ++k) {
    if (w.wx[k]) ck(hipFree(w.wx[k]), "hipFree");
    if (w.wy[k]) ck(hipFree(w.wy[k]), "hipFree");
    if (w.wi[k]) ck(hipFree(w.wi[k]), "hipFree");
    w.wx[k] = w.wy[k] = nullptr;
    w.wi[k] = nullptr;
  }
  w.cap_pts = 0;
  for (int k = 0; k < 2; ++k) {
    ck(hipMalloc(&w.wx[k], n * sizeof(double)), "hipMalloc");
    ck(hipMalloc(&w.wy[k], n * sizeof(double)), "hipMalloc");
    ck(hipMalloc(&w.wi[k], n * sizeof(uint32_t)), "hipMalloc");
  }
  w.cap_pts = n;
}

void ensure_host_req(Context& w, size_t n) {
  if (n <= w.h_req_cap) return;
  if (w.h_req) ck(hipHostFree(w.h_req), "hipHostFree");
  w.h_req = nullptr;
  w.h_req_cap = 0;
  size_t cap = std::max<size_t>(n, 1024);
  ck(hipHostMalloc((void**)&w.h_req, cap * sizeof(Req), hipHostMallocDefault), "hipHostMalloc");
  w.h_req_cap = cap;
}

void ensure_host_u32(Context& w, size_t n) {
  if (n <= w.h_u32_cap) return;
  if (w.h_u32) ck(hipHostFree(w.h_u32), "hipHostFree");
  w.h_u32 = nullptr;
  w.h_u32_cap = 0;
  size_t cap = std::max<size_t>(n, 4096);
  ck(hipHostMalloc((void**)&w.h_u32, cap * sizeof(uint32_t), hipHostMallocDefault), "hipHostMalloc");
  w.h_u32_cap = cap;
}

// device_tables = false: the context of the _ws calls, whose status ring and
// batch counts are carved from the caller's workspace like everything else.
Context* new_context(bool device_tables = true) {
  int dev = 0;
  ck(hipGetDevice(&dev), "hipGetDevice");
  Context* w = new Context();
  w->device = dev;
  if (device_tables) {
    ck(hipMalloc(&w->status_dev, kStatusRing * sizeof(Status)), "hipMalloc");
    ck(hipMalloc(&w->counts_dev, sizeof(BatchCounts)), "hipMalloc");
  }
  ck(hipHostMalloc((void**)&w->counts_host, sizeof(BatchCounts), hipHostMallocDefault), "hipHostMalloc");
  ck(hipHostMalloc((void**)&w->status_host, kStatusRing * sizeof(Status), hipHostMallocDefault), "hipHostMalloc");
  ck(hipHostMalloc((void**)&w->status_words, kStatusRing * kStatusWords * sizeof(uint64_t),
                   hipHostMallocMapped | hipHostMallocCoherent),
     "hipHostMalloc");
  std::memset(w->status_words, 0, kStatusRing * kStatusWords * sizeof(uint64_t));  // tag 0 is never given
  ck(hipHostGetDevicePointer((void**)&w->status_words_dev, w->status_words, 0), "hipHostGetDevicePointer");
  return w;
}

// The default context of the current device (created on first use).
Context& default_context() {
  std::lock_guard<std::mutex> guard(g_ws_mu);
  int dev = 0;
  ck(hipGetDevice(&dev), "hipGetDevice");
  auto it = g_ws.find(dev);
  if (it != g_ws.end()) return *it->second;
  Context* w = new_context();
  g_ws[dev] = w;
  return *w;
}

void free_workspace(Context* w) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  for (int k = 0; k < 2; ++k) {
    f(w->wx[k]);
    f(w->wy[k]);
    f(w->wi[k]);
    f(w->seg[k].p);
    f(w->ctr[k].p);
    f(w->tile_seg[k].p);
  }
  f(w->part.p);
  f(w->part2.p);
  f(w->fr.p);
  f(w->rounds[0].p);
  f(w->rounds[1].p);
  f(w->jctr[0].p);
  f(w->jctr[1].p);
  f(w->epart.p);
  f(w->opart.p);
  f(w->oct.p);
  f(w->tcount.p);
  f(w->toff.p);
  f(w->tile_req.p);
  f(w->req.p);
  f(w->jobs[0].p);
  f(w->jobs[1].p);
  f(w->nodes.p);
  f(w->status_dev);
  f(w->counts_dev);
  f(w->level_nodes.p);
  if (w->counts_host) (void)hipHostFree(w->counts_host);
  if (w->status_host) (void)hipHostFree(w->status_host);
  if (w->status_words) (void)hipHostFree(w->status_words);
  if (w->h_req) (void)hipHostFree(w->h_req);
  if (w->h_u32) (void)hipHostFree(w->h_u32);
  for (hipEvent_t e : w->events) (void)hipEventDestroy(e);
  if (w->staged) (void)hipEventDestroy(w->staged);
  delete w;
}

vqhull_config sanitized(vqhull_config c) {
  if (!sweep_shape_supported(c.sweep_block, c.sweep_ppt)) {
    c.sweep_block = 256;
    c.sweep_ppt = 16;
  }
  c.lds_limit = std::min(2048, std::max(256, c.lds_limit));
  c.reverse_tiles = c.reverse_tiles ? 1 : 0;
  c.prefilter = c.prefilter ? 1 : 0;
  c.sweep_persistent = c.sweep_persistent ? 1 : 0;
  const int tile = c.sweep_block * c.sweep_ppt;
  if (c.level_block <= 0 || c.level_block == c.sweep_block || tile % c.level_block != 0 ||
      !sweep_shape_supported(c.level_block, tile / c.level_block))
    c.level_block = 0;
  return c;
}

// Shape of the sweep of level k: the top-level passes (k <= 1) use the sweep
// shape; deeper levels level_block threads over the same tile.
void level_shape(const vqhull_config& c, int k, int& block, int& ppt) {
  block = c.sweep_block;
  ppt = c.sweep_ppt;
  if (k >= 2 && c.level_block > 0) {
    ppt = c.sweep_block * c.sweep_ppt / c.level_block;
    block = c.level_block;
  }
}

// Timing events are read only after the stream has finished, so they need no
// system-scope fence (which would write back the L2 and idle the GPU ~6 us
// after the kernel before each one).
int take_event(Context& w) {
  if (w.next_event == (int)w.events.size()) {
    hipEvent_t e;
    ck(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreateWithFlags");
    w.events.push_back(e);
  }
  return w.next_event++;
}

// Launch through f(); with timing enabled, bracket it with events on st.
template <typename F>
size_t timed(Context& w, bool on, hipStream_t st, int kind, int level, int64_t in, int64_t out, F&& f) {
  if (!on) {
    f();
    return (size_t)-1;
  }
  TimedLaunch t{kind, level, in, out, take_event(w), 0};
  ck(hipEventRecord(w.events[t.ev0], st), "hipEventRecord");
  f();
  t.ev1 = take_event(w);
  ck(hipEventRecord(w.events[t.ev1], st), "hipEventRecord");
  w.launches.push_back(t);
  return w.launches.size() - 1;
}

void collect_times(Context& w) {
  w.times.clear();
  for (const TimedLaunch& t : w.launches) {
    float ms = 0.f;
    ck(hipEventElapsedTime(&ms, w.events[t.ev0], w.events[t.ev1]), "hipEventElapsedTime");
    w.times.push_back(vqhull_kernel_time{t.kind, t.level, (double)ms, t.in, t.out});
  }
}

// pf: the octagon prefilter ran, so the top-level passes read its compacted
// copy in buffer A instead of the caller's arrays.
int sweep_mode(int k, bool pf) {
  if (k >= 2) return kSweepLevel;
  if (pf) return k == 0 ? kSweepArgmaxWs : kSweepFusedWs;
  return k == 0 ? kSweepArgmax : kSweepFused;
}

// Arguments of level k's kernels (buffers by the parity of k, status slot k mod
// the ring size).  Level 0 is an argmax-only pass over the roots (sizes and
// farthest points of S1 / S2, nothing written); level 1 re-reads the caller's
// arrays and classifies every point twice (root triangle, then its child's
// triangle), so the top level's subsets are never materialized; levels >= 2
// sweep the workspace.
SweepArgs sweep_args(Context& w, const vqhull_config& cfg, int k, const double* x, const double* y, bool pf) {
  SweepArgs sa{};
  const int in_buf = k <= 1 ? (pf ? 0 : -1) : (k - 1) % 2, out_buf = k % 2, cur = k % 2;
  sa.ix = in_buf < 0 ? x : w.wx[in_buf];
  sa.iy = in_buf < 0 ? y : w.wy[in_buf];
  sa.ii = in_buf < 0 ? nullptr : w.wi[in_buf];
  sa.ox = w.wx[out_buf];
  sa.oy = w.wy[out_buf];
  sa.oi = w.wi[out_buf];
  sa.seg = w.seg[cur].p;
  sa.fr = w.fr.p;
  sa.tile_seg = w.tile_seg[k == 1 ? 0 : cur].p;  // the fused pass walks the roots' tiles again
  sa.ctr = w.ctr[cur].p;
  sa.jctr = w.jctr[k & 1].p;
  sa.part = w.part.p;
  sa.part2 = w.part2.p;
  sa.req = w.req.p;
  sa.st = w.status_dev + k % kStatusRing;
  sa.reverse = (uint32_t)cfg.reverse_tiles;
  return sa;
}

FinishArgs finish_args(Context& w, const double* x, const double* y, int k) {
  FinishArgs fa{};
  fa.jobs = w.jobs[k & 1].p;
  fa.ux = x;
  fa.uy = y;
  fa.req_arrays = 1u;
  for (int b = 0; b < 2; ++b) {
    fa.bx[b] = w.wx[b];
    fa.by[b] = w.wy[b];
    fa.bi[b] = w.wi[b];
  }
  fa.req = w.req.p;
  fa.st = w.status_dev + k % kStatusRing;
  fa.nodes = w.nodes.p;
  return fa;
}

PlanArgs plan_args(Context& w, const vqhull_config& cfg, int k, uint32_t G) {
  const int cur = k % 2;
  PlanArgs pl{};
  pl.seg = w.seg[cur].p;
  pl.ctr = w.ctr[cur].p;
  pl.part = w.part.p;
  pl.part2 = w.part2.p;
  pl.fuse = k == 0 ? 1u : 0u;
  pl.fr_out = w.fr.p;
  pl.jctr_out = w.jctr[(k + 1) & 1].p;
  pl.st_in = w.status_dev + k % kStatusRing;
  pl.sweep_grid = G;
  pl.seg_out = w.seg[cur ^ 1].p;
  pl.ctr_out = w.ctr[cur ^ 1].p;
  pl.tile_seg_out = w.tile_seg[cur ^ 1].p;
  pl.jobs = w.jobs[(k + 1) & 1].p;
  pl.nodes = w.nodes.p;
  pl.node_cap = (uint32_t)std::min<size_t>(w.nodes.cap, 0xFFFFFFFFu);
  pl.out_buf = (uint32_t)(k == 0 ? 1 : k % 2);  // level 0's children are written by the fused pass
  pl.st_out = w.status_dev + (k + 1) % kStatusRing;
  pl.st_host = w.status_words_dev ? w.status_words_dev + (size_t)((k + 1) % kStatusRing) * kStatusWords : nullptr;
  pl.st_tag = 0;
  pl.tile = (uint32_t)(cfg.sweep_block * cfg.sweep_ppt);
  pl.lds_limit = (uint32_t)cfg.lds_limit;
  pl.level_nodes = w.level_nodes.p;
  pl.level = (uint32_t)k;
  pl.counts = w.counts_dev;
  pl.planners = kPlanners;
  pl.rounds = w.rounds[k % 2].p;
  pl.rounds_next = w.rounds[(k + 1) % 2].p;
  pl.rounds_cap = (uint32_t)std::min<size_t>(std::min(w.rounds[0].cap, w.rounds[1].cap), 0xFFFFFFFFu);
  return pl;
}

Plan0Args plan0_args(Context& w, const vqhull_config& cfg) {
  Plan0Args pa{};
  pa.req = w.req.p;
  pa.counts = w.counts_dev;
  pa.level_nodes = w.level_nodes.p;
  pa.epart = w.epart.p;
  pa.seg_out = w.seg[0].p;
  pa.ctr_out = w.ctr[0].p;
  pa.tile_seg_out = w.tile_seg[0].p;
  pa.jobs = w.jobs[0].p;
  pa.nodes = w.nodes.p;
  pa.node_cap = (uint32_t)std::min<size_t>(w.nodes.cap, 0xFFFFFFFFu);
  pa.st_out = w.status_dev + 0;
  pa.st_host = w.status_words_dev;
  pa.st_tag = 0;
  pa.tile = (uint32_t)(cfg.sweep_block * cfg.sweep_ppt);
  pa.lds_limit = (uint32_t)cfg.lds_limit;
  pa.ext_tile = kExtTile;
  pa.toff = nullptr;
  pa.filter_min = 0;
  pa.rounds_next = w.rounds[0].p;
  pa.rounds_cap = (uint32_t)std::min<size_t>(std::min(w.rounds[0].cap, w.rounds[1].cap), 0xFFFFFFFFu);
  return pa;
}

// Tags of the status words: never 0 (the words start at 0), never the tag
// of another level still in the ring.
uint32_t next_status_tag(Context& w) {
  if (++w.status_tag == 0) w.status_tag = 1;
  return w.status_tag;
}

// The status record of a ring slot as the planner wrote it to the pinned
// words, once every word carries `tag`.  The host spins on the words and
// puts nothing on the stream: an event, or a query of the stream, adds a
// marker whose system-scope release (a write-back of the whole L2) leaves
// the GPU idle ~6 us before the next kernel, once per level.  Only a wait
// longer than kStatusCheck asks the stream for an error (a stream that has
// finished without the record is an error too).
constexpr auto kStatusCheck = std::chrono::milliseconds(20);

Status wait_status(Context& w, int slot, uint32_t tag, hipStream_t st) {
  const uint64_t* words = w.status_words + (size_t)slot * kStatusWords;
  int idle_checks = 0;
  auto next_check = std::chrono::steady_clock::now() + kStatusCheck;
  for (uint64_t spin = 1;; ++spin) {
    uint32_t v[kStatusWords];
    bool whole = true;
    for (int i = 0; i < kStatusWords && whole; ++i) {
      const uint64_t x = __atomic_load_n(words + i, __ATOMIC_ACQUIRE);
      whole = (uint32_t)(x >> 32) == tag;
      v[i] = (uint32_t)x;
    }
    if (whole) {
      Status s;
      s.nseg = v[0];
      s.ntiles = v[1];
      s.njobs = v[2];
      s.nnodes = v[3];
      s.swept = v[4];
      s.jobpts = v[5];
      s.survivors = v[6];
      s.overflow = v[7];
      return s;
    }
    if (spin % 1024 == 0 && std::chrono::steady_clock::now() >= next_check) {
      next_check = std::chrono::steady_clock::now() + kStatusCheck;
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        if (++idle_checks > 2) ck(hipErrorUnknown, "a planner's status record never reached the host");
      } else if (e != hipErrorNotReady) {
        ck(e, "hipStreamQuery");
      }
    }
  }
}

// Level k >= 2 of a call with level pairs: its point buffers follow the kinds
// of the levels before it (inb: the buffer holding level k's points; the
// second level of a pair reads the first's points again, and its tiles).
void pair_sweep_buffers(Context& w, int k, int mode, int inb, SweepArgs& sa) {
  sa.ix = w.wx[inb];
  sa.iy = w.wy[inb];
  sa.ii = w.wi[inb];
  sa.ox = w.wx[inb ^ 1];
  sa.oy = w.wy[inb ^ 1];
  sa.oi = w.wi[inb ^ 1];
  if (mode == kSweepFusedPair) sa.tile_seg = w.tile_seg[(k - 1) % 2].p;
}

// The plan of that level: its children are read in place by the next sweep
// (the first level of a pair) or written by this one; either way their points
// and this level's jobs end up in the other buffer.  Advances inb.
void pair_plan(int mode, int& inb, PlanArgs& pl) {
  pl.fuse = mode == kSweepArgmaxPair ? 1u : 0u;
  pl.out_buf = (uint32_t)(inb ^ 1);
  if (mode != kSweepArgmaxPair) inb ^= 1;
}

// Inputs whose levels keep nearly every point they sweep (most points are
// hull vertices, as on a circle) finish faster with the 1024-point LDS
// finisher, two workgroups per CU: under the 2048-point threshold, once a
// level (from the third on) has kept more than 3/4 of the points the level
// before it swept, the later levels plan with 1024.  Tables are sized for
// the lower threshold.
constexpr uint32_t kAdaptLds = 1024;
size_t seg_capacity(size_t N, size_t nreq, const vqhull_config& cfg) {
  return N / (std::min<uint32_t>((uint32_t)cfg.lds_limit, kAdaptLds) + 1) + nreq + 2;
}

// The whole hull computation for nreq requests on one stream.
//
// Level k's kernels read their work counts from the device status record the
// previous plan wrote, so the host enqueues level k before it knows them and
// waits only for the status of level k-1: the GPU never waits for the host
// between levels.  When a status shows an empty level, the loop stops (the
// kernels already enqueued for it find no work).
// ingested: the extremes records were written by the ingest of interleaved
// input (x, y: its copy in buffer A), so the extremes pass is not run.
bool run_once(Context& w, const vqhull_config& cfg, const double* x, const double* y, const double* xy,
              int64_t nreq, int64_t* out_idx, int64_t* out_counts, hipStream_t st, size_t N,
              const uint32_t* tile_req, size_t ext_tiles, uint64_t tiles0, size_t max_tiles, bool ingested) {
  const uint32_t tile = (uint32_t)(cfg.sweep_block * cfg.sweep_ppt);
  const uint32_t lds_limit = (uint32_t)cfg.lds_limit;
  const int tmax = finish_tmax_for(cfg.lds_limit);

  const size_t max_seg = seg_capacity(N, (size_t)nreq, cfg);
  const int tmode = g_timing.load();
  const bool tm = tmode == 1 || tmode == 2;  // sweeps
  const bool tm_all = tmode == 1;            // every other launch too
  const bool tm_fused = tmode != 0;          // the sweep of level 1 (the fused pass) in every mode

  // Octagon prefilter (requests above the LDS threshold only): extremes in
  // eight directions, the edges, the filter into buffer B, the prefix of the
  // kept counts and the compaction into buffer A.  Interleaved input takes
  // the same passes for every request (the filter deinterleaves into buffer
  // A, dropping points only with the prefilter on), so every later kernel
  // reads the workspace.
  const bool aos = xy != nullptr;
  const bool pf = aos || (cfg.prefilter != 0 && tiles0 > 0);
  const uint32_t filter_min = aos ? 0u : lds_limit;
  if (pf) {
    const OctArgs oa{x, y, xy, tile_req, w.req.p, w.epart.p, w.opart.p, w.counts_dev, (uint32_t)ext_tiles};
    timed(w, tm_all, st, VQHULL_K_EXTREMES, 0, (int64_t)N, 0, [&] { ck(launch_octagon(oa, st), "k_octagon"); });
    FilterArgs fa{};
    fa.x = x;
    fa.y = y;
    fa.xy = xy;
    fa.tile_req = tile_req;
    fa.req = w.req.p;
    fa.part = w.epart.p;
    fa.opart = w.opart.p;
    fa.oct = w.oct.p;
    fa.sx = w.wx[1];
    fa.sy = w.wy[1];
    fa.si = w.wi[1];
    fa.cx = w.wx[0];
    fa.cy = w.wy[0];
    fa.ci = w.wi[0];
    fa.tcount = w.tcount.p;
    fa.toff = w.toff.p;
    fa.counts = w.counts_dev;
    fa.ntiles = (uint32_t)ext_tiles;
    fa.min_points = filter_min;
    fa.drop_min = cfg.prefilter ? lds_limit : 0xFFFFFFFFu;
    timed(w, tm_all, st, VQHULL_K_FILTER, 0, (int64_t)N, 0, [&] {
      ck(launch_oct_plan(fa, (uint32_t)nreq, st), "k_oct_plan");
      ck(launch_filter(fa, st), "k_filter");
      ck(launch_filter_scan(fa, st), "k_filter_scan");
    });
    timed(w, tm_all, st, VQHULL_K_COMPACT, 0, 0, 0, [&] { ck(launch_compact(fa, st), "k_compact"); });
  } else if (!ingested) {
    ExtremesArgs ea{x, y, tile_req, w.req.p, w.epart.p, w.counts_dev, (uint32_t)ext_tiles};
    timed(w, tm_all, st, VQHULL_K_EXTREMES, 0, (int64_t)N, 0, [&] { ck(launch_extremes(ea, st), "k_extremes"); });
  }
  ensure(w.level_nodes, 16, st, true);
  Plan0Args pa = plan0_args(w, cfg);
  if (pf) {
    pa.toff = w.toff.p;
    pa.filter_min = filter_min;
  }
  std::vector<uint32_t> tags;  // tags[k]: the tag of level k's status words
  tags.push_back(next_status_tag(w));
  pa.st_tag = tags[0];
  timed(w, tm_all, st, VQHULL_K_PLAN0, 0, nreq, 0, [&] { ck(launch_plan0(pa, st), "k_plan0"); });

  std::vector<Status> known;           // host copies of status[0..]
  std::vector<size_t> sweep_recs;      // timing records of the sweeps, per level
  std::vector<size_t> finish_recs;     // timing records of the finisher + planner launches, per level
  bool overflow = false;
  int64_t known_nodes = (int64_t)nreq, known_seg = (int64_t)std::min<size_t>((size_t)nreq, max_seg);
  uint32_t lds_plan = lds_limit;  // threshold of the next plan
  uint32_t lds_jobs = lds_limit;  // threshold the jobs of the current level were made with
  const bool adapt = lds_limit > kAdaptLds && w.seg[0].cap >= max_seg;
  // Level pairs: a level whose segments are swept without writing (argmax
  // pass) and the next level, whose segments are read in place from the level
  // before and whose children are written (fused pass), as the top level
  // does.  Two reads and one write per point instead of two of each: chosen
  // where the level before kept more than 3/4 of the points it swept.  Such
  // levels halve their segments, so the levels left whose segments still
  // exceed the threshold the plans end with are about log2(average segment /
  // threshold); a pair starts only where that count is even, so that the
  // pairs end on the last of them (a pair whose first level makes only
  // finisher jobs reads them twice and copies them once).
  const int pairs = g_pairs.load();
  const uint32_t lds_end = adapt ? kAdaptLds : lds_limit;
  auto segment_levels_left = [&](const Status& s) {
    if (s.nseg == 0) return 0;
    double a = (double)s.swept / (double)s.nseg / (double)lds_end;
    int n = 0;
    for (; a >= 2.0; a *= 0.5) ++n;
    return n;
  };
  std::vector<int> kinds;  // VQHULL_SWEEP_* of each level enqueued
  int inb = 1;             // the buffer holding the points of level k >= 2
  uint32_t G_prev = 0;
  // Finisher jobs of level k run after sweep k (the fused pass writes the
  // points of level 1's small children), in the same launch as plan k.
  for (int k = 0;; ++k) {
    const int slot = k % kStatusRing, next = (k + 1) % kStatusRing;
    int mode = sweep_mode(k, pf);
    if (k >= 2) {
      const int prev = kinds[k - 1];
      if (prev == VQHULL_SWEEP_ARGMAX) {
        mode = kSweepFusedPair;
      } else if (pairs == 2 ||
                 (pairs == 1 && k >= 3 && known[k - 2].swept >= (1u << 20) &&
                  4ull * known[k - 1].survivors > 3ull * known[k - 2].swept &&
                  segment_levels_left(known[k - 1]) >= 2 && segment_levels_left(known[k - 1]) % 2 == 0)) {
        mode = kSweepArgmaxPair;
      }
    }
    const bool argmax = mode == kSweepArgmax || mode == kSweepArgmaxWs || mode == kSweepArgmaxPair;
    const bool fused = mode == kSweepFused || mode == kSweepFusedWs || mode == kSweepFusedPair;
    kinds.push_back(argmax ? VQHULL_SWEEP_ARGMAX : fused ? VQHULL_SWEEP_FUSED : VQHULL_SWEEP_LEVEL);
    SweepArgs sa = sweep_args(w, cfg, k, x, y, pf);
    if (k >= 2) pair_sweep_buffers(w, k, mode, inb, sa);
    // Grid: persistent, or one workgroup per tile with the tile count bounded
    // from what the host knows (levels 0 and 1 exactly; level k from level
    // k-1: tiles <= ceil(swept(k-1) / tile) + 2 nseg(k-1)); surplus groups exit.
    int blk = 0, ppt = 0;
    level_shape(cfg, k, blk, ppt);
    uint32_t G = sweep_grid(blk, ppt, mode);
    if (!cfg.sweep_persistent) {
      uint64_t bound = k <= 1 ? tiles0
                              : (known[k - 1].swept + (uint64_t)tile - 1) / tile + 2ull * known[k - 1].nseg + 1;
      G = mode == kSweepFusedPair ? G_prev : (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(bound, max_tiles));
    }
    G_prev = G;
    sweep_recs.push_back(timed(w, tm || (tm_fused && k == 1), st, VQHULL_K_SWEEP, k, 0, 0, [&] {
      ck(launch_sweep(sa, mode, blk, ppt, G, st), "k_sweep");
    }));

    // Node capacity for this plan: nodes after it <= nodes(k) + 2 nseg(k), with
    // nodes(k) <= nodes(k-1) + 2 nseg(k-1) and nseg(k) <= min(2 nseg(k-1), max_seg).
    // A grown table is copied on the stream before the launch below, which
    // takes the new pointer for both its planner and its finisher.
    const int64_t need = known_nodes + 2 * known_seg + 2 * std::min<int64_t>(2 * known_seg, (int64_t)max_seg) + 16;
    if (!w.nodes.fixed) ensure(w.nodes, (size_t)need, st, true);  // a fixed table holds every vertex
    ensure(w.level_nodes, (size_t)k + 3, st, true);
    // (with interleaved input no job reads the caller's arrays: every root
    // went through the filter into buffer A)
    const FinishArgs fa = finish_args(w, aos ? xy : x, aos ? xy : y, k);
    vqhull_config cfg_k = cfg;
    cfg_k.lds_limit = (int)lds_plan;
    PlanArgs pl = plan_args(w, cfg_k, k, G);
    if (k >= 2) pair_plan(mode, inb, pl);
    tags.push_back(next_status_tag(w));
    pl.st_tag = tags[k + 1];
    const int tmax_k = finish_tmax_for((int)lds_jobs);
    finish_recs.push_back(timed(w, tm_all, st, VQHULL_K_PLAN, k, 0, 0,
                                [&] { ck(launch_finish_plan(fa, pl, tmax_k, st), "k_finish_plan"); }));
    lds_jobs = lds_plan;

    // Wait for the status of level k (written by the previous plan).
    const Status sk = wait_status(w, slot, tags[k], st);
    known.push_back(sk);
    w.stats.push_back({(int64_t)sk.nseg, (int64_t)sk.swept, (int64_t)sk.njobs, (int64_t)sk.jobpts, kinds[k]});
    // sweep k reads status[k].swept points (a fused pass: the points of the
    // level before again) and writes what plan k counts as survivors (an
    // argmax pass writes nothing), a fused pass also the pass-through copies
    if (k >= 2 && sweep_recs[k - 1] != (size_t)-1 && kinds[k - 1] != VQHULL_SWEEP_ARGMAX)
      w.launches[sweep_recs[k - 1]].out += sk.survivors;
    if (sweep_recs[k] != (size_t)-1)
      w.launches[sweep_recs[k]].in = kinds[k] == VQHULL_SWEEP_FUSED ? known[k - 1].swept : sk.swept;
    if (kinds[k] == VQHULL_SWEEP_FUSED && sweep_recs[k] != (size_t)-1) w.launches[sweep_recs[k]].out += sk.jobpts;
    if (finish_recs[k] != (size_t)-1) w.launches[finish_recs[k]].in = sk.jobpts;
    if (sk.overflow) {
      overflow = true;
      break;
    }
    known_nodes = sk.nnodes;
    known_seg = sk.nseg;
    if (adapt && lds_plan > kAdaptLds && k >= 3 && known[k - 1].swept >= (1u << 20) &&
        4ull * sk.survivors > 3ull * known[k - 1].swept)
      lds_plan = kAdaptLds;  // from plan k + 1 on (plan k is already enqueued)
    if (sk.nseg == 0) {
      // Level k had no segment: plan(k) wrote an empty status (its jobs = 0).
      // The node count after level k is final.
      break;
    }
  }
  if (overflow) {
    ck(hipStreamSynchronize(st), "hipStreamSynchronize");
    return false;
  }

  // assembly: node level boundaries are the node counts after each plan,
  // recorded on the device by the planners
  const size_t nlevels = known.size();
  AssembleArgs aa{};
  aa.nodes = w.nodes.p;
  aa.level_begin = w.level_nodes.p;
  aa.nlevels = (uint32_t)nlevels;
  aa.req = w.req.p;
  aa.counts = w.counts_dev;
  aa.lists[0] = w.wi[0];
  aa.lists[1] = w.wi[1];
  aa.out_idx = out_idx;
  aa.out_count = out_counts;
  aa.max_nodes = known.back().nnodes;
  timed(w, tm_all, st, VQHULL_K_ASSEMBLE, (int)nlevels, aa.max_nodes, 0, [&] {
    ck(launch_assemble(aa, st), "k_assemble");
    ck(launch_copy_lists(aa, st), "k_copy_lists");
  });
  // The staging buffers are reused by the next call: wait for the copies.
  ck(hipStreamSynchronize(st), "hipStreamSynchronize");
  return true;
}

vqhull_config current_config() {
  std::lock_guard<std::mutex> g(g_cfg_mu);
  return sanitized(g_cfg);
}

// Device capacity for batches of up to N points in nreq requests.
struct Caps {
  size_t max_seg, max_tiles;
};

Caps reserve(Context& w, const vqhull_config& cfg, size_t N, size_t nreq, size_t ext_tiles, hipStream_t st,
             bool aos = false) {
  const uint32_t tile = (uint32_t)(cfg.sweep_block * cfg.sweep_ppt);
  const uint32_t lds_limit = (uint32_t)cfg.lds_limit;
  ensure(w.req, std::max<size_t>(nreq, 1), st);
  ensure(w.epart, std::max<size_t>(ext_tiles, 1), st);
  if (cfg.prefilter || aos) {
    ensure(w.opart, std::max<size_t>(ext_tiles, 1), st);
    ensure(w.oct, std::max<size_t>(nreq, 1), st);
    ensure(w.tcount, std::max<size_t>(ext_tiles, 1), st);
    ensure(w.toff, ext_tiles + 1, st);
  }
  ensure_points(w, std::max<size_t>(N, 1), st);
  Caps c;
  c.max_seg = seg_capacity(N, nreq, cfg);
  c.max_tiles = N / tile + c.max_seg + 2;
  for (int k = 0; k < 2; ++k) {
    ensure(w.seg[k], c.max_seg, st);
    ensure(w.ctr[k], c.max_seg * kCtrStride, st);
    ensure(w.tile_seg[k], c.max_tiles, st);
  }
  ensure(w.part, c.max_tiles, st);
  ensure(w.part2, c.max_tiles, st);
  ensure(w.fr, c.max_seg, st);
  for (int k = 0; k < 2; ++k) ensure(w.rounds[k], c.max_seg / kPlanRoundMin + 3, st);
  for (int k = 0; k < 2; ++k) {
    ensure(w.jobs[k], 2 * c.max_seg + nreq, st);
    ensure(w.jctr[k], (2 * c.max_seg + nreq) * kCtrStride, st);
  }
  ensure(w.nodes, std::max<size_t>(3 * nreq + 64, 4096), st);
  return c;
}

// xy: interleaved input (x and y unused), or nullptr.
void run(Context& w, const vqhull_config& cfg, const double* x, const double* y, const int64_t* offsets, int64_t nreq,
         int64_t* out_idx, int64_t* out_counts, hipStream_t st, const double* xy = nullptr) {
  const uint32_t tile = (uint32_t)(cfg.sweep_block * cfg.sweep_ppt);
  const uint32_t lds_limit = (uint32_t)cfg.lds_limit;
  const size_t N = (size_t)offsets[nreq];

  std::lock_guard<std::mutex> guard(w.mu);
  ck(hipSetDevice(w.device), "hipSetDevice");

  // Interleaved input without the prefilter: copy x and y into buffer A and
  // run the plain path on that copy (with the prefilter, the filter pass
  // deinterleaves the points it keeps instead).
  const double* const xy_in = xy;
  const bool deint = xy != nullptr && !cfg.prefilter;
  if (deint) {
    ensure_points(w, std::max<size_t>(N, 1), st);
    x = w.wx[0];
    y = w.wy[0];
    xy = nullptr;
  }
  auto ingest = [&](const uint32_t* tile_req, size_t ext_tiles) {
    if (!deint) return;
    timed(w, g_timing.load() == 1, st, VQHULL_K_INGEST, 0, (int64_t)N, (int64_t)N, [&] {
      if (ext_tiles == 0) {  // the one-launch small path: a plain copy
        ck(launch_deinterleave(xy_in, w.wx[0], w.wy[0], (uint64_t)N, st), "k_deinterleave");
      } else {
        const IngestArgs ia{xy_in, w.wx[0], w.wy[0], tile_req, w.req.p, w.epart.p, w.counts_dev,
                            (uint32_t)ext_tiles};
        ck(launch_ingest(ia, st), "k_ingest");
      }
    });
  };

  // A single request small enough for the LDS finisher: one launch does it
  // all (extremes, Algorithm 1 in LDS, the clockwise list).
  if (nreq == 1 && N <= lds_limit && !xy) {
    ensure_points(w, std::max<size_t>(N, 1), st);
    ensure(w.nodes, 4096, st);
    ensure(w.req, 1, st);
    w.stats.clear();
    w.launches.clear();
    w.next_event = 0;
    ingest(nullptr, 0);
    SmallArgs sa{x, y, (uint32_t)N, out_idx, out_counts, w.wi[0], w.nodes.p, w.req.p};
    timed(w, g_timing.load() == 1, st, VQHULL_K_FINISH, 0, (int64_t)N, 0,
          [&] { ck(launch_small(sa, finish_tmax_for(cfg.lds_limit), st), "k_small"); });
    // The workspace is reused by the next call: wait for the kernel.
    ck(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (g_timing.load()) collect_times(w);
    return;
  }

  // request table and extremes tile map
  ensure_host_req(w, (size_t)nreq);
  size_t ext_tiles = 0;
  uint64_t tiles0 = 0;  // level-0 sweep tiles (requests too big for the LDS finisher)
  for (int64_t i = 0; i < nreq; ++i) {
    Req r{};
    r.off = (uint32_t)offsets[i];
    r.n = (uint32_t)(offsets[i + 1] - offsets[i]);
    r.root = -1;
    r.tile0 = (uint32_t)ext_tiles;
    r.x = x ? x + offsets[i] : nullptr;
    r.y = y ? y + offsets[i] : nullptr;
    ext_tiles += (r.n + kExtTile - 1) / kExtTile;
    if (r.n > lds_limit) tiles0 += (r.n + tile - 1) / tile;
    w.h_req[i] = r;
  }
  const Caps caps = reserve(w, cfg, N, (size_t)nreq, ext_tiles, st, xy != nullptr);
  const uint32_t* tile_req = nullptr;
  if (nreq > 1 && ext_tiles > 0) {
    ensure_host_u32(w, ext_tiles);
    size_t t = 0;
    for (int64_t i = 0; i < nreq; ++i) {
      const size_t nt = (w.h_req[i].n + kExtTile - 1) / kExtTile;
      for (size_t k = 0; k < nt; ++k) w.h_u32[t++] = (uint32_t)i;
    }
    ensure(w.tile_req, ext_tiles, st);
    ck(hipMemcpyAsync(w.tile_req.p, w.h_u32, ext_tiles * sizeof(uint32_t), hipMemcpyHostToDevice, st),
       "hipMemcpyAsync");
    tile_req = w.tile_req.p;
  }

  w.counts_host->nreq = (uint32_t)nreq;
  w.counts_host->ext_tiles = (uint32_t)ext_tiles;
  w.counts_host->overflow = 0;
  w.counts_host->pad = 0;
  ck(hipMemcpyAsync(w.counts_dev, w.counts_host, sizeof(BatchCounts), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
  for (int attempt = 0;; ++attempt) {
    ck(hipMemcpyAsync(w.req.p, w.h_req, (size_t)nreq * sizeof(Req), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    w.stats.clear();
    w.launches.clear();
    w.next_event = 0;
    ingest(tile_req, ext_tiles);  // again on a retry: the failed attempt may have overwritten buffer A
    if (run_once(w, cfg, x, y, xy, nreq, out_idx, out_counts, st, N, tile_req, ext_tiles, tiles0, caps.max_tiles,
                 deint))
      break;
    // The node table was too small for a level (not expected with the host's
    // bound): grow it and start over.
    ensure(w.nodes, 2 * w.nodes.cap, st);
    if (attempt > 8) ck(hipErrorOutOfMemory, "node table");
  }
  if (g_timing.load()) collect_times(w);
}

template <typename F>
int guard_status(F&& f) {
  try {
    f();
  } catch (const HipFail& e) {
    return e.e == hipErrorOutOfMemory ? VQHULL_ERR_OUT_OF_MEMORY : VQHULL_ERR_HIP;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return VQHULL_ERR_OUT_OF_MEMORY;
  } catch (const WorkspaceTooSmall&) {
    return VQHULL_ERR_OUT_OF_MEMORY;
  }
  return VQHULL_OK;
}

// Level statistics and kernel times of the last public hull call per device
// (whichever context ran it), for vqhull_last_level_stats / _kernel_times.
struct LastCall {
  std::vector<LevelStat> stats;
  std::vector<vqhull_kernel_time> times;
};
std::mutex g_last_mu;
std::map<int, LastCall> g_last;

void publish_last(const Context& w) {
  std::lock_guard<std::mutex> g(g_last_mu);
  LastCall& L = g_last[w.device];
  L.stats = w.stats;
  if (g_timing.load())
    L.times = w.times;
  else
    L.times.clear();
}

int guarded(const double* x, const double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
            int64_t* out_counts, vqhull_stream_t stream, const double* xy = nullptr) {
  return guard_status([&] {
    Context& w = default_context();
    run(w, current_config(), x, y, offsets, nreq, out_idx, out_counts, (hipStream_t)stream, xy);
    publish_last(w);
  });
}

// ------------------------------------------------- caller-owned workspace

constexpr size_t kWsAlign = 256;

// Every device table a call with N points in nreq requests can use, carved
// in order from the workspace at `base` (with base null, only the size is
// computed and w is left as it is).  The sizes are those the library-owned
// path reserves; the node table holds one node per input point plus three per
// request (every vertex the recursion can emit outside the LDS finisher), and
// the per-level node counts cover up to 2^20 levels.  Returns the bytes used.
// inplace: buffer A's coordinate arrays are the caller's x and y (set by the
// caller of this function), so only its index array is carved.
size_t ws_layout(Context& w, char* base, size_t N, size_t nreq, const vqhull_config& cfg, bool inplace = false) {
  N = std::max<size_t>(N, 1);
  nreq = std::max<size_t>(nreq, 1);
  const size_t tile = (size_t)cfg.sweep_block * (size_t)cfg.sweep_ppt;
  const size_t ext_tiles = N / kExtTile + nreq;  // >= the sum over requests of ceil(n_i / kExtTile)
  const size_t max_seg = seg_capacity(N, nreq, cfg);
  const size_t max_tiles = N / tile + max_seg + 2;
  const size_t njobs = 2 * max_seg + nreq;
  size_t off = 0;
  auto raw = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + kWsAlign - 1) / kWsAlign * kWsAlign;
    return p;
  };
  auto take = [&](auto& b, size_t n) {
    using T = std::remove_pointer_t<decltype(b.p)>;
    T* p = reinterpret_cast<T*>(raw(n * sizeof(T)));
    if (base) {
      b.p = p;
      b.cap = n;
      b.fixed = true;
    }
  };
  for (int k = 0; k < 2; ++k) {
    const bool own = !(inplace && k == 0);
    double* px = own ? reinterpret_cast<double*>(raw(N * sizeof(double))) : nullptr;
    double* py = own ? reinterpret_cast<double*>(raw(N * sizeof(double))) : nullptr;
    uint32_t* pi = reinterpret_cast<uint32_t*>(raw(N * sizeof(uint32_t)));
    if (base) {
      w.wx[k] = px;
      w.wy[k] = py;
      w.wi[k] = pi;
    }
  }
  for (int k = 0; k < 2; ++k) {
    take(w.seg[k], max_seg);
    take(w.ctr[k], max_seg * kCtrStride);
    take(w.tile_seg[k], max_tiles);
    take(w.jobs[k], njobs);
    take(w.jctr[k], njobs * kCtrStride);
  }
  take(w.part, max_tiles);
  take(w.part2, max_tiles);
  take(w.fr, max_seg);
  take(w.rounds[0], max_seg / kPlanRoundMin + 3);
  take(w.rounds[1], max_seg / kPlanRoundMin + 3);
  take(w.epart, ext_tiles);
  take(w.opart, ext_tiles);
  take(w.oct, nreq);
  take(w.tcount, ext_tiles);
  take(w.toff, ext_tiles + 1);
  take(w.tile_req, ext_tiles);
  take(w.req, nreq);
  take(w.nodes, std::max<size_t>(N + 3 * nreq + 64, 4096));
  take(w.level_nodes, std::min<size_t>(N, size_t(1) << 20) + 64);
  BatchCounts* counts = reinterpret_cast<BatchCounts*>(raw(sizeof(BatchCounts)));
  Status* status = reinterpret_cast<Status*>(raw(kStatusRing * sizeof(Status)));
  if (base) {
    w.counts_dev = counts;
    w.status_dev = status;
    w.cap_pts = N;
    w.fixed = true;
  }
  return off;
}

size_t ws_bytes(size_t N, size_t nreq, const vqhull_config& cfg, bool inplace = false) {
  Context sizing;
  return ws_layout(sizing, nullptr, N, nreq, cfg, inplace);
}

// The contexts of the _ws calls: host-side state only (pinned staging, the
// pinned status copies, events), one per concurrent call, pooled per device.
std::mutex g_wsc_mu;
std::map<int, std::vector<Context*>> g_wsc_free;

Context* acquire_ws_context() {
  int dev = 0;
  ck(hipGetDevice(&dev), "hipGetDevice");
  {
    std::lock_guard<std::mutex> g(g_wsc_mu);
    auto& v = g_wsc_free[dev];
    if (!v.empty()) {
      Context* c = v.back();
      v.pop_back();
      return c;
    }
  }
  return new_context(false);
}

// Forget every view into the caller's workspace, then return the context to
// its device's pool.
void release_ws_context(Context* c) {
  for (int k = 0; k < 2; ++k) {
    c->wx[k] = c->wy[k] = nullptr;
    c->wi[k] = nullptr;
    c->seg[k] = {};
    c->ctr[k] = {};
    c->tile_seg[k] = {};
    c->jobs[k] = {};
    c->jctr[k] = {};
  }
  c->part = {};
  c->part2 = {};
  c->fr = {};
  c->rounds[0] = {};
  c->rounds[1] = {};
  c->epart = {};
  c->opart = {};
  c->oct = {};
  c->tcount = {};
  c->toff = {};
  c->tile_req = {};
  c->req = {};
  c->nodes = {};
  c->level_nodes = {};
  c->counts_dev = nullptr;
  c->status_dev = nullptr;
  c->cap_pts = 0;
  c->fixed = false;
  std::lock_guard<std::mutex> g(g_wsc_mu);
  g_wsc_free[c->device].push_back(c);
}

// inplace: x and y (the caller's, writable) also serve as buffer A's
// coordinate arrays from the first recursion level that writes buffer A on.
int guarded_ws(const double* x, const double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
               int64_t* out_counts, void* ws, size_t ws_size, vqhull_stream_t stream, bool inplace = false) {
  const vqhull_config cfg = current_config();
  const size_t N = (size_t)offsets[nreq];
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kWsAlign) != 0 ||
      ws_size < ws_bytes(N, (size_t)nreq, cfg, inplace)) {
    g_last_error = "workspace missing, misaligned or smaller than vqhull_workspace_bytes()";
    return VQHULL_ERR_INVALID_ARGUMENT;
  }
  Context* c = nullptr;
  int st = guard_status([&] { c = acquire_ws_context(); });
  if (st != VQHULL_OK) return st;
  st = guard_status([&] {
    ws_layout(*c, static_cast<char*>(ws), N, (size_t)nreq, cfg, inplace);
    if (inplace) {
      c->wx[0] = const_cast<double*>(x);
      c->wy[0] = const_cast<double*>(y);
    }
    run(*c, cfg, x, y, offsets, nreq, out_idx, out_counts, (hipStream_t)stream);
    publish_last(*c);
  });
  release_ws_context(c);
  return st;
}

// ------------------------------------------------- stream-ordered batched call

// Host-side contexts of the stream-ordered calls, pooled per device.  A
// context returns to the pool at once, but is taken again only after the
// stream has copied its staging (its `staged` event has completed); otherwise
// a new one is made, so a call does not wait for earlier work, up to
// kAsyncMaxContexts per device: past that, a call waits for the oldest
// staging copy (the pool's host memory stays bounded).
std::mutex g_asc_mu;
std::map<int, std::vector<Context*>> g_asc_free;
std::map<int, int> g_asc_count;
constexpr int kAsyncMaxLevels = 4096;
constexpr int kAsyncMaxContexts = 32;

Context* acquire_async_context() {
  int dev = 0;
  ck(hipGetDevice(&dev), "hipGetDevice");
  Context* wait_for = nullptr;
  {
    std::lock_guard<std::mutex> g(g_asc_mu);
    auto& v = g_asc_free[dev];
    for (size_t i = 0; i < v.size(); ++i) {
      if (hipEventQuery(v[i]->staged) == hipSuccess) {
        Context* c = v[i];
        v.erase(v.begin() + (ptrdiff_t)i);
        return c;
      }
    }
    if (g_asc_count[dev] >= kAsyncMaxContexts && !v.empty()) {
      wait_for = v.front();  // the longest in the pool
      v.erase(v.begin());
    } else {
      ++g_asc_count[dev];
    }
  }
  if (wait_for) {
    ck(hipEventSynchronize(wait_for->staged), "hipEventSynchronize");
    return wait_for;
  }
  Context* c = new_context(false);
  ck(hipEventCreateWithFlags(&c->staged, hipEventDisableTiming), "hipEventCreateWithFlags");
  return c;
}

void release_async_context(Context* c) {
  std::lock_guard<std::mutex> g(g_asc_mu);
  g_asc_free[c->device].push_back(c);
}

// Extremes, root planning, `levels` levels of sweeps and finisher + planner
// launches with persistent grids, and the assembly, all enqueued on the stream
// with no host wait.  The planners write no status to the host; the assembly
// reads the device status of the level after the last and, if it still has
// work, marks every request incomplete instead of writing lists.
void enqueue_async(Context& w, vqhull_config cfg, const double* x, const double* y, const int64_t* offsets,
                   int64_t nreq, int64_t* out_idx, int64_t* out_counts, int levels, hipStream_t st) {
  const size_t N = (size_t)offsets[nreq];
  size_t ext_tiles = 0;
  ensure_host_req(w, (size_t)nreq);
  for (int64_t i = 0; i < nreq; ++i) {
    Req r{};
    r.off = (uint32_t)offsets[i];
    r.n = (uint32_t)(offsets[i + 1] - offsets[i]);
    r.root = -1;
    r.tile0 = (uint32_t)ext_tiles;
    r.x = x + offsets[i];
    r.y = y + offsets[i];
    ext_tiles += (r.n + kExtTile - 1) / kExtTile;
    w.h_req[i] = r;
  }
  if (ext_tiles > w.tile_req.cap) ck(hipErrorInvalidValue, "extremes tiles beyond the workspace");
  ensure_host_u32(w, std::max<size_t>(ext_tiles, 1));
  size_t t = 0;
  for (int64_t i = 0; i < nreq; ++i) {
    const size_t nt = (w.h_req[i].n + kExtTile - 1) / kExtTile;
    for (size_t k = 0; k < nt; ++k) w.h_u32[t++] = (uint32_t)i;
  }
  w.counts_host->nreq = (uint32_t)nreq;
  w.counts_host->ext_tiles = (uint32_t)ext_tiles;
  w.counts_host->overflow = 0;
  w.counts_host->pad = 0;
  ck(hipMemcpyAsync(w.req.p, w.h_req, (size_t)nreq * sizeof(Req), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
  if (ext_tiles)
    ck(hipMemcpyAsync(w.tile_req.p, w.h_u32, ext_tiles * sizeof(uint32_t), hipMemcpyHostToDevice, st),
       "hipMemcpyAsync");
  ck(hipMemcpyAsync(w.counts_dev, w.counts_host, sizeof(BatchCounts), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
  ck(hipEventRecord(w.staged, st), "hipEventRecord");

  // The recursion of n points is at most n + 2 levels deep, and the table of
  // per-level node counts holds min(N, 2^20) + 64 entries: a longer budget
  // would only add empty levels.
  levels = (int)std::min<size_t>((size_t)levels, w.level_nodes.cap - 3);
  const int tmax = finish_tmax_for(cfg.lds_limit);
  const ExtremesArgs ea{x, y, w.tile_req.p, w.req.p, w.epart.p, w.counts_dev, (uint32_t)ext_tiles};
  ck(launch_extremes(ea, st), "k_extremes");
  Plan0Args pa = plan0_args(w, cfg);
  pa.st_host = nullptr;
  ck(launch_plan0(pa, st), "k_plan0");
  for (int k = 0; k < levels; ++k) {
    const int mode = sweep_mode(k, false);
    int blk = 0, ppt = 0;
    level_shape(cfg, k, blk, ppt);
    const uint32_t G = sweep_grid(blk, ppt, mode);
    ck(launch_sweep(sweep_args(w, cfg, k, x, y, false), mode, blk, ppt, G, st), "k_sweep");
    PlanArgs pl = plan_args(w, cfg, k, G);
    pl.st_host = nullptr;
    ck(launch_finish_plan(finish_args(w, x, y, k), pl, tmax, st), "k_finish_plan");
  }
  AssembleArgs aa{};
  aa.nodes = w.nodes.p;
  aa.level_begin = w.level_nodes.p;
  aa.nlevels = (uint32_t)levels + 1u;
  aa.req = w.req.p;
  aa.counts = w.counts_dev;
  aa.lists[0] = w.wi[0];
  aa.lists[1] = w.wi[1];
  aa.out_idx = out_idx;
  aa.out_count = out_counts;
  aa.max_nodes = (uint32_t)std::min<size_t>(w.nodes.cap, 0xFFFFFFFFu);
  aa.last = w.status_dev + levels % kStatusRing;
  ck(launch_assemble(aa, st), "k_assemble");
  ck(launch_copy_lists(aa, st), "k_copy_lists");
  (void)N;
}

int guarded_async(const double* x, const double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
                  int64_t* out_counts, int levels, void* ws, size_t ws_size, vqhull_stream_t stream) {
  vqhull_config cfg = current_config();
  cfg.sweep_persistent = 1;  // grids must not depend on counts the host does not read
  cfg.prefilter = 0;
  const size_t N = (size_t)offsets[nreq];
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kWsAlign) != 0 || ws_size < ws_bytes(N, (size_t)nreq, cfg)) {
    g_last_error = "workspace missing, misaligned or smaller than vqhull_workspace_bytes()";
    return VQHULL_ERR_INVALID_ARGUMENT;
  }
  Context* c = nullptr;
  int st = guard_status([&] { c = acquire_async_context(); });
  if (st != VQHULL_OK) return st;
  st = guard_status([&] {
    ws_layout(*c, static_cast<char*>(ws), N, (size_t)nreq, cfg);
    enqueue_async(*c, cfg, x, y, offsets, nreq, out_idx, out_counts, levels, (hipStream_t)stream);
  });
  release_async_context(c);
  return st;
}

// ------------------------------------------ the entry point that allocates nothing
//
// vqhull_hull_noalloc keeps every device table of a call in `scratch`, a
// static device array of the library (one copy per GPU, at that GPU's own
// address, taken once per device with hipGetSymbolAddress).  It sizes the
// tables for VQHULL_NOALLOC_MAX_POINTS points under the most demanding
// configuration (LDS threshold 256, 4096-point tiles: 81.9 MiB).  The level
// loop is device-driven: levels are enqueued in chunks whose kernels read
// their work counts from the device, and the host reads one status record per
// chunk (a copy into static host memory), so no event, pinned buffer or other
// allocation is needed.

constexpr size_t kNoAllocBytes = size_t(84) << 20;
constexpr int kNoAllocChunk = 8;  // levels enqueued between two status reads
constexpr int kMaxDevices = 64;

}  // namespace

namespace vqh {
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
}  // namespace vqh

namespace {

struct NoAllocDevice {
  std::mutex mu;          // calls on one GPU run one at a time (they share its scratch)
  char* ptr = nullptr;    // this device's address of scratch
  Context ctx;            // views into scratch; no host staging
  Req req{};              // host staging of the request table and counts (static storage:
  BatchCounts counts{};   // a pageable source that outlives the asynchronous copy)
  Status status{};
  BatchCounts counts_back{};
};
NoAllocDevice g_noalloc[kMaxDevices];

// One request of n > 0 points; every table already laid out in w.
void run_fixed_single(Context& w, vqhull_config cfg, const double* x, const double* y, uint32_t n, int64_t* out_idx,
                      int64_t* out_count, hipStream_t st, NoAllocDevice& d) {
  cfg.sweep_persistent = 1;  // grids must not depend on counts the host has not read
  if (n <= (uint32_t)cfg.lds_limit) {
    SmallArgs sa{x, y, n, out_idx, out_count, w.wi[0], w.nodes.p, w.req.p};
    ck(launch_small(sa, finish_tmax_for(cfg.lds_limit), st), "k_small");
    ck(hipStreamSynchronize(st), "hipStreamSynchronize");
    return;
  }
  d.req = Req{};
  d.req.off = 0;
  d.req.n = n;
  d.req.root = -1;
  d.req.tile0 = 0;
  d.req.x = x;
  d.req.y = y;
  d.counts = BatchCounts{1u, (n + kExtTile - 1) / kExtTile, 0u, 0u};
  ck(hipMemcpyAsync(w.req.p, &d.req, sizeof(Req), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
  ck(hipMemcpyAsync(w.counts_dev, &d.counts, sizeof(BatchCounts), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
  const ExtremesArgs ea{x, y, nullptr, w.req.p, w.epart.p, w.counts_dev, d.counts.ext_tiles};
  ck(launch_extremes(ea, st), "k_extremes");
  ck(launch_plan0(plan0_args(w, cfg), st), "k_plan0");
  const int tmax = finish_tmax_for(cfg.lds_limit);
  int k = 0;
  for (;;) {
    for (int j = 0; j < kNoAllocChunk; ++j, ++k) {
      if ((size_t)k + 3 > w.level_nodes.cap) ck(hipErrorOutOfMemory, "recursion deeper than the level table");
      const int mode = sweep_mode(k, false);
      int blk = 0, ppt = 0;
      level_shape(cfg, k, blk, ppt);
      const uint32_t G = sweep_grid(blk, ppt, mode);
      ck(launch_sweep(sweep_args(w, cfg, k, x, y, false), mode, blk, ppt, G, st), "k_sweep");
      ck(launch_finish_plan(finish_args(w, x, y, k), plan_args(w, cfg, k, G), tmax, st), "k_finish_plan");
    }
    ck(hipMemcpyAsync(&d.status, w.status_dev + k % kStatusRing, sizeof(Status), hipMemcpyDeviceToHost, st),
       "hipMemcpyAsync");
    ck(hipMemcpyAsync(&d.counts_back, w.counts_dev, sizeof(BatchCounts), hipMemcpyDeviceToHost, st),
       "hipMemcpyAsync");
    ck(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (d.status.overflow || d.counts_back.overflow) ck(hipErrorOutOfMemory, "node table");
    if (d.status.nseg == 0 && d.status.njobs == 0) break;  // level k has no work: the recursion is done
  }
  AssembleArgs aa{};
  aa.nodes = w.nodes.p;
  aa.level_begin = w.level_nodes.p;
  aa.nlevels = (uint32_t)k + 1u;
  aa.req = w.req.p;
  aa.counts = w.counts_dev;
  aa.lists[0] = w.wi[0];
  aa.lists[1] = w.wi[1];
  aa.out_idx = out_idx;
  aa.out_count = out_count;
  aa.max_nodes = (uint32_t)std::min<size_t>(w.nodes.cap, 0xFFFFFFFFu);
  ck(launch_assemble(aa, st), "k_assemble");
  ck(launch_copy_lists(aa, st), "k_copy_lists");
  ck(hipStreamSynchronize(st), "hipStreamSynchronize");
}

// Offsets: offsets[0] = 0, non-decreasing, total below 2^31.
bool offsets_valid(const int64_t* offsets, int64_t nreq) {
  if (offsets[0] != 0) return false;
  for (int64_t i = 0; i < nreq; ++i)
    if (offsets[i + 1] < offsets[i]) return false;
  return offsets[nreq] < (int64_t(1) << 31);
}

}  // namespace

namespace vqh {

int context_create(Context** out) {
  return guard_status([&] { *out = new_context(); });
}

void context_destroy(Context* c) {
  if (!c) return;
  {
    std::lock_guard<std::mutex> guard(c->mu);
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
  }
  free_workspace(c);
}

int context_reserve(Context* c, int64_t npoints, int64_t nreq, void* stream) {
  return guard_status([&] {
    std::lock_guard<std::mutex> guard(c->mu);
    ck(hipSetDevice(c->device), "hipSetDevice");
    const vqhull_config cfg = current_config();
    hipStream_t st = (hipStream_t)stream;
    const size_t ext_tiles = (size_t)npoints / kExtTile + (size_t)nreq;
    reserve(*c, cfg, (size_t)npoints, (size_t)nreq, ext_tiles, st);
    ensure(c->tile_req, ext_tiles, st);
    ensure(c->nodes, (size_t)npoints + 3 * (size_t)nreq + 64, st);
    ensure_host_req(*c, (size_t)nreq);
    ensure_host_u32(*c, ext_tiles);
    ck(hipStreamSynchronize(st), "hipStreamSynchronize");
  });
}

// The server's lanes run the plain method: their graph replays never use the
// octagon prefilter, so neither does their plain fallback.
int context_run(Context* c, const double* x, const double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
                int64_t* out_counts, void* stream) {
  if (nreq == 0) return VQHULL_OK;
  vqhull_config cfg = current_config();
  cfg.prefilter = 0;
  return guard_status([&] { run(*c, cfg, x, y, offsets, nreq, out_idx, out_counts, (hipStream_t)stream); });
}

const char* context_last_error() { return g_last_error.c_str(); }

uint64_t allocation_generation() { return g_alloc_gen.load(); }

int context_reserve_fixed(Context* c, int64_t npoints, int64_t nreq, int levels, void* stream) {
  int st = context_reserve(c, npoints, nreq, stream);
  if (st != VQHULL_OK) return st;
  return guard_status([&] {
    std::lock_guard<std::mutex> guard(c->mu);
    ck(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    ensure(c->level_nodes, (size_t)levels + 3, s);
    // grid sizes are cached on the host here, before any capture
    const vqhull_config cfg = current_config();
    for (int m = 0; m < 3; ++m) (void)sweep_grid(cfg.sweep_block, cfg.sweep_ppt, m);
    int lb = 0, lp = 0;
    level_shape(cfg, 2, lb, lp);
    (void)sweep_grid(lb, lp, kSweepLevel);
    (void)finish_grid(finish_tmax_for(cfg.lds_limit));
    ck(hipStreamSynchronize(s), "hipStreamSynchronize");
  });
}

int context_stage(Context* c, const int64_t* offsets, int64_t nreq, const double* const* xs,
                  const double* const* ys) {
  std::lock_guard<std::mutex> guard(c->mu);
  const vqhull_config cfg = current_config();
  const uint32_t tile = (uint32_t)(cfg.sweep_block * cfg.sweep_ppt);
  const size_t N = (size_t)offsets[nreq];
  if (nreq < 1 || N > c->cap_pts || (size_t)nreq > c->req.cap || (size_t)nreq > c->h_req_cap)
    return VQHULL_ERR_INVALID_ARGUMENT;
  size_t ext_tiles = 0;
  for (int64_t i = 0; i < nreq; ++i) {
    Req r{};
    r.off = (uint32_t)offsets[i];
    r.n = (uint32_t)(offsets[i + 1] - offsets[i]);
    r.root = -1;
    r.tile0 = (uint32_t)ext_tiles;
    r.x = xs[i];
    r.y = ys[i];
    ext_tiles += (r.n + kExtTile - 1) / kExtTile;
    c->h_req[i] = r;
  }
  (void)tile;
  if (ext_tiles > c->tile_req.cap || ext_tiles > c->h_u32_cap || ext_tiles > c->epart.cap)
    return VQHULL_ERR_INVALID_ARGUMENT;
  size_t t = 0;
  for (int64_t i = 0; i < nreq; ++i) {
    const size_t nt = (c->h_req[i].n + kExtTile - 1) / kExtTile;
    for (size_t k = 0; k < nt; ++k) c->h_u32[t++] = (uint32_t)i;
  }
  c->counts_host->nreq = (uint32_t)nreq;
  c->counts_host->ext_tiles = (uint32_t)ext_tiles;
  c->counts_host->overflow = 0;
  c->counts_host->pad = 0;
  return VQHULL_OK;
}

int context_enqueue_fixed(Context* c, const double* x, const double* y, int64_t* out_idx, int64_t* out_counts,
                          int levels, void* stream) {
  return guard_status([&] {
    std::lock_guard<std::mutex> guard(c->mu);
    Context& w = *c;
    const vqhull_config cfg = current_config();
    if (!cfg.sweep_persistent || levels < 1 || w.level_nodes.cap < (size_t)levels + 3)
      ck(hipErrorInvalidValue, "fixed launch sequence");
    hipStream_t st = (hipStream_t)stream;
    const int tmax = finish_tmax_for(cfg.lds_limit);
    const size_t nreq_cap = std::min(w.req.cap, w.h_req_cap);
    const size_t tiles_cap = std::min(std::min(w.tile_req.cap, w.h_u32_cap), w.epart.cap);
    ck(hipMemcpyAsync(w.req.p, w.h_req, nreq_cap * sizeof(Req), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    ck(hipMemcpyAsync(w.tile_req.p, w.h_u32, tiles_cap * sizeof(uint32_t), hipMemcpyHostToDevice, st),
       "hipMemcpyAsync");
    ck(hipMemcpyAsync(w.counts_dev, w.counts_host, sizeof(BatchCounts), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    const ExtremesArgs ea{x, y, w.tile_req.p, w.req.p, w.epart.p, w.counts_dev, (uint32_t)tiles_cap};
    ck(launch_extremes(ea, st), "k_extremes");
    // The lane reads its last status by a copy on the stream: the planners
    // write no host words.
    Plan0Args pa = plan0_args(w, cfg);
    pa.st_host = nullptr;
    ck(launch_plan0(pa, st), "k_plan0");
    for (int k = 0; k < levels; ++k) {
      const int mode = sweep_mode(k, false);
      int blk = 0, ppt = 0;
      level_shape(cfg, k, blk, ppt);
      const uint32_t G = sweep_grid(blk, ppt, mode);
      ck(launch_sweep(sweep_args(w, cfg, k, x, y, false), mode, blk, ppt, G, st), "k_sweep");
      PlanArgs pl = plan_args(w, cfg, k, G);
      pl.st_host = nullptr;
      ck(launch_finish_plan(finish_args(w, x, y, k), pl, tmax, st), "k_finish_plan");
    }
    const int last = levels % kStatusRing;
    ck(hipMemcpyAsync(w.status_host + last, w.status_dev + last, sizeof(Status), hipMemcpyDeviceToHost, st),
       "hipMemcpyAsync");
    ck(hipMemcpyAsync(w.counts_host, w.counts_dev, sizeof(BatchCounts), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    AssembleArgs aa{};
    aa.nodes = w.nodes.p;
    aa.level_begin = w.level_nodes.p;
    aa.nlevels = (uint32_t)levels + 1u;
    aa.req = w.req.p;
    aa.counts = w.counts_dev;
    aa.lists[0] = w.wi[0];
    aa.lists[1] = w.wi[1];
    aa.out_idx = out_idx;
    aa.out_count = out_counts;
    aa.max_nodes = (uint32_t)std::min<size_t>(w.nodes.cap, 0xFFFFFFFFu);
    ck(launch_assemble(aa, st), "k_assemble");
    ck(launch_copy_lists(aa, st), "k_copy_lists");
  });
}

bool context_fixed_done(Context* c, int levels) {
  std::lock_guard<std::mutex> guard(c->mu);
  const Status& s = c->status_host[levels % kStatusRing];
  return s.nseg == 0 && s.njobs == 0 && s.overflow == 0 && c->counts_host->overflow == 0;
}

}  // namespace vqh

extern "C" {

int vqhull_hull(const double* x, const double* y, int64_t n, int64_t* out_idx, int64_t* out_count,
                vqhull_stream_t stream) {
  if (n < 0 || n >= (int64_t(1) << 31) || !out_idx || !out_count || (n > 0 && (!x || !y)))
    return VQHULL_ERR_INVALID_ARGUMENT;
  const int64_t offsets[2] = {0, n};
  return guarded(x, y, offsets, 1, out_idx, out_count, stream);
}

int vqhull_hull_batched(const double* x, const double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
                        int64_t* out_counts, vqhull_stream_t stream) {
  if (nreq < 0 || !offsets || nreq >= (int64_t(1) << 31)) return VQHULL_ERR_INVALID_ARGUMENT;
  if (nreq == 0) return VQHULL_OK;
  if (offsets[0] != 0 || !out_counts || !out_idx) return VQHULL_ERR_INVALID_ARGUMENT;
  for (int64_t i = 0; i < nreq; ++i)
    if (offsets[i + 1] < offsets[i]) return VQHULL_ERR_INVALID_ARGUMENT;
  if (offsets[nreq] >= (int64_t(1) << 31)) return VQHULL_ERR_INVALID_ARGUMENT;
  if (offsets[nreq] > 0 && (!x || !y)) return VQHULL_ERR_INVALID_ARGUMENT;
  return guarded(x, y, offsets, nreq, out_idx, out_counts, stream);
}

size_t vqhull_workspace_bytes(int64_t n_total, int64_t nreq) {
  if (n_total < 0 || n_total >= (int64_t(1) << 31) || nreq < 0 || nreq >= (int64_t(1) << 31)) return 0;
  try {
    return ws_bytes((size_t)n_total, (size_t)nreq, current_config());
  } catch (...) {
    return 0;
  }
}

int vqhull_hull_ws(const double* x, const double* y, int64_t n, int64_t* out_idx, int64_t* out_count,
                   void* workspace, size_t workspace_bytes, vqhull_stream_t stream) {
  if (n < 0 || n >= (int64_t(1) << 31) || !out_idx || !out_count || (n > 0 && (!x || !y)))
    return VQHULL_ERR_INVALID_ARGUMENT;
  const int64_t offsets[2] = {0, n};
  return guarded_ws(x, y, offsets, 1, out_idx, out_count, workspace, workspace_bytes, stream);
}

int vqhull_hull_batched_ws(const double* x, const double* y, const int64_t* offsets, int64_t nreq,
                           int64_t* out_idx, int64_t* out_counts, void* workspace, size_t workspace_bytes,
                           vqhull_stream_t stream) {
  if (nreq < 0 || !offsets || nreq >= (int64_t(1) << 31)) return VQHULL_ERR_INVALID_ARGUMENT;
  if (nreq == 0) return VQHULL_OK;
  if (!out_counts || !out_idx || !offsets_valid(offsets, nreq)) return VQHULL_ERR_INVALID_ARGUMENT;
  if (offsets[nreq] > 0 && (!x || !y)) return VQHULL_ERR_INVALID_ARGUMENT;
  return guarded_ws(x, y, offsets, nreq, out_idx, out_counts, workspace, workspace_bytes, stream);
}

int vqhull_hull_noalloc(const double* x, const double* y, int64_t n, int64_t* out_idx, int64_t* out_count,
                        vqhull_stream_t stream) {
  if (n < 0 || n > VQHULL_NOALLOC_MAX_POINTS || !out_idx || !out_count || (n > 0 && (!x || !y))) {
    g_last_error = "vqhull_hull_noalloc: invalid argument or more than VQHULL_NOALLOC_MAX_POINTS points";
    return VQHULL_ERR_INVALID_ARGUMENT;
  }
  const vqhull_config cfg = current_config();
  if (ws_bytes((size_t)n, 1, cfg) > kNoAllocBytes) {  // cannot happen for n within the limit
    g_last_error = "vqhull_hull_noalloc: the static scratch array is too small for this configuration";
    return VQHULL_ERR_INVALID_ARGUMENT;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    g_last_error = "vqhull_hull_noalloc: no usable current device";
    return VQHULL_ERR_HIP;
  }
  NoAllocDevice& d = g_noalloc[dev];
  std::lock_guard<std::mutex> guard(d.mu);
  return guard_status([&] {
    hipStream_t st = (hipStream_t)stream;
    if (!d.ptr) {  // once per device, with that device current: its own address of the array
      void* p = nullptr;
      ck(hipGetSymbolAddress(&p, HIP_SYMBOL(vqh::scratch)), "hipGetSymbolAddress");
      d.ptr = static_cast<char*>(p);
      d.ctx.device = dev;
    }
    Context& w = d.ctx;
    ws_layout(w, d.ptr, (size_t)n, 1, cfg);  // its context has no pinned status words: the planners write none
    run_fixed_single(w, cfg, x, y, (uint32_t)n, out_idx, out_count, st, d);
  });
}

int vqhull_hull_batched_async(const double* x, const double* y, const int64_t* offsets, int64_t nreq,
                              int64_t* out_idx, int64_t* out_counts, int32_t levels, void* workspace,
                              size_t workspace_bytes, vqhull_stream_t stream) {
  if (nreq < 0 || !offsets || nreq >= (int64_t(1) << 31) || levels < 1 || levels > kAsyncMaxLevels)
    return VQHULL_ERR_INVALID_ARGUMENT;
  if (nreq == 0) return VQHULL_OK;
  if (!out_counts || !out_idx || !offsets_valid(offsets, nreq)) return VQHULL_ERR_INVALID_ARGUMENT;
  if (offsets[nreq] > 0 && (!x || !y)) return VQHULL_ERR_INVALID_ARGUMENT;
  return guarded_async(x, y, offsets, nreq, out_idx, out_counts, levels, workspace, workspace_bytes, stream);
}

size_t vqhull_workspace_bytes_inplace(int64_t n_total, int64_t nreq) {
  if (n_total < 0 || n_total >= (int64_t(1) << 31) || nreq < 0 || nreq >= (int64_t(1) << 31)) return 0;
  try {
    return ws_bytes((size_t)n_total, (size_t)nreq, current_config(), true);
  } catch (...) {
    return 0;
  }
}

int vqhull_hull_inplace(double* x, double* y, int64_t n, int64_t* out_idx, int64_t* out_count, void* workspace,
                        size_t workspace_bytes, vqhull_stream_t stream) {
  if (n < 0 || n >= (int64_t(1) << 31) || !out_idx || !out_count || (n > 0 && (!x || !y)))
    return VQHULL_ERR_INVALID_ARGUMENT;
  const int64_t offsets[2] = {0, n};
  return guarded_ws(x, y, offsets, 1, out_idx, out_count, workspace, workspace_bytes, stream, true);
}

int vqhull_hull_batched_inplace(double* x, double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
                                int64_t* out_counts, void* workspace, size_t workspace_bytes,
                                vqhull_stream_t stream) {
  if (nreq < 0 || !offsets || nreq >= (int64_t(1) << 31)) return VQHULL_ERR_INVALID_ARGUMENT;
  if (nreq == 0) return VQHULL_OK;
  if (!out_counts || !out_idx || !offsets_valid(offsets, nreq)) return VQHULL_ERR_INVALID_ARGUMENT;
  if (offsets[nreq] > 0 && (!x || !y)) return VQHULL_ERR_INVALID_ARGUMENT;
  return guarded_ws(x, y, offsets, nreq, out_idx, out_counts, workspace, workspace_bytes, stream, true);
}

int vqhull_hull_xy(const double* xy, int64_t n, int64_t* out_idx, int64_t* out_count, vqhull_stream_t stream) {
  if (n < 0 || n >= (int64_t(1) << 31) || !out_idx || !out_count || (n > 0 && !xy) ||
      (reinterpret_cast<uintptr_t>(xy) & 15u) != 0)
    return VQHULL_ERR_INVALID_ARGUMENT;
  const int64_t offsets[2] = {0, n};
  return guarded(nullptr, nullptr, offsets, 1, out_idx, out_count, stream, n > 0 ? xy : nullptr);
}

int vqhull_hull_batched_xy(const double* xy, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
                           int64_t* out_counts, vqhull_stream_t stream) {
  if (nreq < 0 || !offsets || nreq >= (int64_t(1) << 31)) return VQHULL_ERR_INVALID_ARGUMENT;
  if (nreq == 0) return VQHULL_OK;
  if (!out_counts || !out_idx || !offsets_valid(offsets, nreq)) return VQHULL_ERR_INVALID_ARGUMENT;
  if (offsets[nreq] > 0 && (!xy || (reinterpret_cast<uintptr_t>(xy) & 15u) != 0)) return VQHULL_ERR_INVALID_ARGUMENT;
  return guarded(nullptr, nullptr, offsets, nreq, out_idx, out_counts, stream, offsets[nreq] > 0 ? xy : nullptr);
}

int vqhull_autotune(const double* x, const double* y, int64_t n, int32_t repeats, vqhull_tune_entry* entries,
                    int64_t cap, int64_t* count, vqhull_config* best, vqhull_stream_t stream) {
  if (n < 1 || n >= (int64_t(1) << 31) || !x || !y || repeats < 1 || repeats > 100 || !count || !best ||
      cap < 0 || (cap > 0 && !entries))
    return VQHULL_ERR_INVALID_ARGUMENT;
  static const int shapes[][2] = {{256, 16}, {256, 32}, {512, 8}, {512, 16}, {1024, 8}};
  static const int lds_limits[] = {512, 1024, 2048};
  std::vector<vqhull_config> cands;
  for (const auto& sh : shapes)
    for (int lds : lds_limits)
      for (int pers = 1; pers >= 0; --pers)
        cands.push_back(sanitized(vqhull_config{sh[0], sh[1], lds, 0, pers, 256, 0}));
  hipStream_t st = (hipStream_t)stream;
  int64_t* d_idx = nullptr;
  int64_t* d_cnt = nullptr;
  int status = guard_status([&] {
    ck(hipMalloc(&d_idx, (size_t)n * sizeof(int64_t)), "hipMalloc");
    ck(hipMalloc(&d_cnt, sizeof(int64_t)), "hipMalloc");
  });
  std::vector<int64_t> ref, cur;
  int64_t ref_cnt = 0;
  double best_ms = 1e300;
  int64_t k = 0;
  const int64_t offsets[2] = {0, n};
  for (size_t c = 0; c < cands.size() && status == VQHULL_OK; ++c) {
    std::vector<double> ms;
    int64_t cnt = 0;
    status = guard_status([&] {
      Context& w = default_context();
      for (int r = 0; r <= repeats; ++r) {  // the first run warms up
        ck(hipStreamSynchronize(st), "hipStreamSynchronize");
        const auto t0 = std::chrono::steady_clock::now();
        run(w, cands[c], x, y, offsets, 1, d_idx, d_cnt, st);  // returns after the result is written
        const auto t1 = std::chrono::steady_clock::now();
        if (r) ms.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
      }
      ck(hipMemcpy(&cnt, d_cnt, sizeof(int64_t), hipMemcpyDeviceToHost), "hipMemcpy");
      cur.assign((size_t)std::max<int64_t>(cnt, 0), 0);
      if (cnt > 0) ck(hipMemcpy(cur.data(), d_idx, (size_t)cnt * sizeof(int64_t), hipMemcpyDeviceToHost), "hipMemcpy");
    });
    if (status != VQHULL_OK) break;
    std::sort(ms.begin(), ms.end());
    const double med = ms[ms.size() / 2];
    if (c == 0) {
      ref = cur;
      ref_cnt = cnt;
    }
    const bool same = cnt == ref_cnt && cur == ref;
    if (k < cap) entries[k] = vqhull_tune_entry{cands[c], med, same ? 1 : 0, 0};
    ++k;
    if (same && med < best_ms) {
      best_ms = med;
      *best = cands[c];
    }
  }
  if (d_idx) (void)hipFree(d_idx);
  if (d_cnt) (void)hipFree(d_cnt);
  *count = k;
  return status;
}

int vqhull_get_config(vqhull_config* cfg) {
  if (!cfg) return VQHULL_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> g(g_cfg_mu);
  *cfg = g_cfg;
  return VQHULL_OK;
}

int vqhull_set_config(const vqhull_config* cfg) {
  if (!cfg) return VQHULL_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> g(g_cfg_mu);
  g_cfg = sanitized(*cfg);
  return VQHULL_OK;
}

int64_t vqhull_last_level_stats(int64_t* out, int64_t cap) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> g(g_last_mu);
  auto it = g_last.find(dev);
  if (it == g_last.end()) return 0;
  const auto& st = it->second.stats;
  for (int64_t i = 0; i < (int64_t)st.size() && i < cap && out; ++i) {
    out[4 * i + 0] = st[i].segs;
    out[4 * i + 1] = st[i].swept;
    out[4 * i + 2] = st[i].jobs;
    out[4 * i + 3] = st[i].jobpts;
  }
  return (int64_t)st.size();
}

int64_t vqhull_last_level_kinds(int32_t* out, int64_t cap) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> g(g_last_mu);
  auto it = g_last.find(dev);
  if (it == g_last.end()) return 0;
  const auto& st = it->second.stats;
  for (int64_t i = 0; i < (int64_t)st.size() && i < cap && out; ++i) out[i] = st[i].kind;
  return (int64_t)st.size();
}

int vqhull_set_level_pairs(int mode) {
  if (mode < 0 || mode > 2) return VQHULL_ERR_INVALID_ARGUMENT;
  g_pairs.store(mode);
  return VQHULL_OK;
}

int vqhull_orient(const double* abc, int64_t n, double* out, vqhull_stream_t stream) {
  if (n < 0 || (n > 0 && (!abc || !out))) return VQHULL_ERR_INVALID_ARGUMENT;
  const int e = launch_orient(abc, (uint64_t)n, out, stream);
  if (e != 0) {
    g_last_error = std::string("k_orient: ") + hipGetErrorString((hipError_t)e);
    return VQHULL_ERR_HIP;
  }
  return VQHULL_OK;
}

int vqhull_stream_scale(const double* in, double* out, int64_t n, double s, vqhull_stream_t stream) {
  if (n < 0 || (n > 0 && (!in || !out))) return VQHULL_ERR_INVALID_ARGUMENT;
  const int e = launch_stream_scale(in, out, (uint64_t)n, s, stream);
  if (e != 0) {
    g_last_error = std::string("k_stream_scale: ") + hipGetErrorString((hipError_t)e);
    return VQHULL_ERR_HIP;
  }
  return VQHULL_OK;
}

int vqhull_set_timing(int enable) {
  if (enable < 0 || enable > 3) return VQHULL_ERR_INVALID_ARGUMENT;
  g_timing.store(enable);
  return VQHULL_OK;
}

int64_t vqhull_last_kernel_times(vqhull_kernel_time* out, int64_t cap) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> g(g_last_mu);
  auto it = g_last.find(dev);
  if (it == g_last.end()) return 0;
  const auto& t = it->second.times;
  for (int64_t i = 0; i < (int64_t)t.size() && i < cap && out; ++i) out[i] = t[i];
  return (int64_t)t.size();
}

int vqhull_release_workspace(void) {
  std::lock_guard<std::mutex> guard(g_ws_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VQHULL_ERR_HIP;
  auto it = g_ws.find(dev);
  if (it == g_ws.end()) return VQHULL_OK;
  Context* c = it->second;
  {
    std::lock_guard<std::mutex> cguard(c->mu);
    if (hipDeviceSynchronize() != hipSuccess) return VQHULL_ERR_HIP;
  }
  g_ws.erase(it);
  free_workspace(c);
  return VQHULL_OK;
}

const char* vqhull_status_string(int status) {
  switch (status) {
    case VQHULL_OK:
      return "ok";
    case VQHULL_ERR_INVALID_ARGUMENT:
      return "invalid argument";
    case VQHULL_ERR_OUT_OF_MEMORY:
      return "out of device memory";
    case VQHULL_ERR_NONFINITE:
      return "non-finite coordinate in the input";
    case VQHULL_ERR_HIP:
      return "HIP runtime error";
    case VQHULL_ERR_TIMEOUT:
      return "request not done before the deadline";
    case VQHULL_ERR_INCOMPLETE:
      return "the level budget ended before the recursion";
    default:
      return "unknown status";
  }
}

const char* vqhull_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
