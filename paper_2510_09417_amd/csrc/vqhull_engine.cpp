// Host engine and C ABI of the gfx950 planar Quickhull.
//
// The recursion of Algorithm 1 runs breadth-first: each level is one sweep
// launch over every live segment of every request, followed by a one-workgroup
// planning kernel that lays out the next level and hands small subproblems to
// the LDS finisher.  The host reads the planner's small status record after
// each level to size the next launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vqhull.h"
#include "vqhull_internal.h"

using namespace vqh;

namespace {

thread_local std::string g_last_error;

std::mutex g_cfg_mu;
vqhull_config g_cfg = {512, 8, 2048, 0};

struct LevelStat {
  int64_t segs, swept, jobs, jobpts;
};

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
};

struct Workspace {
  int device = -1;
  size_t cap_pts = 0;
  double* wx[2] = {nullptr, nullptr};
  double* wy[2] = {nullptr, nullptr};
  uint32_t* wi[2] = {nullptr, nullptr};
  DevBuf<Seg> seg[2];
  DevBuf<unsigned long long> ctr[2];
  DevBuf<uint32_t> tile_seg[2];
  DevBuf<TilePart> part;
  DevBuf<ExtPart> epart;
  DevBuf<uint32_t> tile_req;
  DevBuf<Req> req;
  DevBuf<Job> jobs;
  DevBuf<Node> nodes;
  DevBuf<uint32_t> level_begin;
  Status* status_dev = nullptr;
  Status* status_host = nullptr;
  // pinned staging
  Req* h_req = nullptr;
  size_t h_req_cap = 0;
  uint32_t* h_u32 = nullptr;
  size_t h_u32_cap = 0;
  std::vector<LevelStat> stats;
};

std::mutex g_ws_mu;
std::map<int, Workspace*> g_ws;

struct HipFail {
  hipError_t e;
};

inline void ck(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    throw HipFail{e};
  }
}

inline void ck(int e, const char* what) { ck((hipError_t)e, what); }

template <typename T>
void ensure(DevBuf<T>& b, size_t n, hipStream_t st, bool keep = false) {
  if (n <= b.cap) return;
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

void ensure_points(Workspace& w, size_t n, hipStream_t st) {
  if (n <= w.cap_pts) return;
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

void ensure_host_req(Workspace& w, size_t n) {
  if (n <= w.h_req_cap) return;
  if (w.h_req) ck(hipHostFree(w.h_req), "hipHostFree");
  w.h_req = nullptr;
  w.h_req_cap = 0;
  size_t cap = std::max<size_t>(n, 1024);
  ck(hipHostMalloc((void**)&w.h_req, cap * sizeof(Req), hipHostMallocDefault), "hipHostMalloc");
  w.h_req_cap = cap;
}

void ensure_host_u32(Workspace& w, size_t n) {
  if (n <= w.h_u32_cap) return;
  if (w.h_u32) ck(hipHostFree(w.h_u32), "hipHostFree");
  w.h_u32 = nullptr;
  w.h_u32_cap = 0;
  size_t cap = std::max<size_t>(n, 4096);
  ck(hipHostMalloc((void**)&w.h_u32, cap * sizeof(uint32_t), hipHostMallocDefault), "hipHostMalloc");
  w.h_u32_cap = cap;
}

Workspace& workspace_for_current_device() {
  int dev = 0;
  ck(hipGetDevice(&dev), "hipGetDevice");
  auto it = g_ws.find(dev);
  if (it != g_ws.end()) return *it->second;
  Workspace* w = new Workspace();
  w->device = dev;
  ck(hipMalloc(&w->status_dev, sizeof(Status)), "hipMalloc");
  ck(hipHostMalloc((void**)&w->status_host, sizeof(Status), hipHostMallocDefault), "hipHostMalloc");
  g_ws[dev] = w;
  return *w;
}

void free_workspace(Workspace* w) {
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
  f(w->epart.p);
  f(w->tile_req.p);
  f(w->req.p);
  f(w->jobs.p);
  f(w->nodes.p);
  f(w->level_begin.p);
  f(w->status_dev);
  if (w->status_host) (void)hipHostFree(w->status_host);
  if (w->h_req) (void)hipHostFree(w->h_req);
  if (w->h_u32) (void)hipHostFree(w->h_u32);
  delete w;
}

vqhull_config sanitized(vqhull_config c) {
  if (!sweep_shape_supported(c.sweep_block, c.sweep_ppt)) {
    c.sweep_block = 512;
    c.sweep_ppt = 8;
  }
  c.lds_limit = std::min(2048, std::max(256, c.lds_limit));
  c.reverse_tiles = c.reverse_tiles ? 1 : 0;
  return c;
}

Status read_status(Workspace& w, hipStream_t st) {
  ck(hipMemcpyAsync(w.status_host, w.status_dev, sizeof(Status), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  ck(hipStreamSynchronize(st), "hipStreamSynchronize");
  return *w.status_host;
}

// The whole hull computation for nreq requests on one stream.
void run(const double* x, const double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
         int64_t* out_counts, hipStream_t st) {
  vqhull_config cfg;
  {
    std::lock_guard<std::mutex> g(g_cfg_mu);
    cfg = sanitized(g_cfg);
  }
  const uint32_t tile = (uint32_t)(cfg.sweep_block * cfg.sweep_ppt);
  const uint32_t lds_limit = (uint32_t)cfg.lds_limit;
  const int tmax = finish_tmax_for(cfg.lds_limit);
  const size_t N = (size_t)offsets[nreq];

  std::lock_guard<std::mutex> guard(g_ws_mu);
  Workspace& w = workspace_for_current_device();
  w.stats.clear();

  // request table and extremes tile map
  ensure_host_req(w, (size_t)nreq);
  size_t ext_tiles = 0;
  for (int64_t i = 0; i < nreq; ++i) {
    Req r{};
    r.off = (uint32_t)offsets[i];
    r.n = (uint32_t)(offsets[i + 1] - offsets[i]);
    r.root = -1;
    r.tile0 = (uint32_t)ext_tiles;
    ext_tiles += (r.n + kExtTile - 1) / kExtTile;
    w.h_req[i] = r;
  }
  ensure(w.req, (size_t)std::max<int64_t>(nreq, 1), st);
  ck(hipMemcpyAsync(w.req.p, w.h_req, (size_t)nreq * sizeof(Req), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
  ensure(w.epart, std::max<size_t>(ext_tiles, 1), st);
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

  // capacities
  ensure_points(w, std::max<size_t>(N, 1), st);
  const size_t max_seg = N / (lds_limit + 1) + (size_t)nreq + 2;
  const size_t max_tiles = N / tile + max_seg + 2;
  for (int k = 0; k < 2; ++k) {
    ensure(w.seg[k], max_seg, st);
    ensure(w.ctr[k], max_seg, st);
    ensure(w.tile_seg[k], max_tiles, st);
  }
  ensure(w.part, max_tiles, st);
  ensure(w.jobs, 2 * max_seg + (size_t)nreq, st);
  ensure(w.nodes, std::max<size_t>((size_t)nreq + 1, 1024), st);

  // extremes and root plan
  ExtremesArgs ea{x, y, tile_req, w.req.p, w.epart.p, (uint32_t)ext_tiles};
  ck(launch_extremes(ea, st), "k_extremes");
  Plan0Args pa{};
  pa.req = w.req.p;
  pa.nreq = (uint32_t)nreq;
  pa.epart = w.epart.p;
  pa.seg_out = w.seg[0].p;
  pa.ctr_out = w.ctr[0].p;
  pa.tile_seg_out = w.tile_seg[0].p;
  pa.jobs = w.jobs.p;
  pa.nodes = w.nodes.p;
  pa.status = w.status_dev;
  pa.tile = tile;
  pa.lds_limit = lds_limit;
  pa.ext_tile = kExtTile;
  ck(launch_plan0(pa, st), "k_plan0");
  Status s = read_status(w, st);
  w.stats.push_back({(int64_t)s.nseg, (int64_t)s.swept, (int64_t)s.njobs, (int64_t)s.jobpts});

  std::vector<uint32_t> level_begin = {0u, s.nnodes};
  FinishArgs fa{};
  fa.jobs = w.jobs.p;
  fa.ux = x;
  fa.uy = y;
  for (int k = 0; k < 2; ++k) {
    fa.bx[k] = w.wx[k];
    fa.by[k] = w.wy[k];
    fa.bi[k] = w.wi[k];
  }
  fa.nodes = w.nodes.p;
  fa.req = w.req.p;
  ck(launch_finish(fa, s.njobs, tmax, st), "k_finish");

  uint32_t nseg = s.nseg, ntiles = s.ntiles, nnodes = s.nnodes;
  int cur = 0;      // segment table / tile map / counter parity of the current level
  int in_buf = -1;  // -1: caller arrays (level 0)
  int out_buf = 0;
  while (nseg > 0) {
    SweepArgs sa{};
    sa.ix = in_buf < 0 ? x : w.wx[in_buf];
    sa.iy = in_buf < 0 ? y : w.wy[in_buf];
    sa.ii = in_buf < 0 ? nullptr : w.wi[in_buf];
    sa.ox = w.wx[out_buf];
    sa.oy = w.wy[out_buf];
    sa.oi = w.wi[out_buf];
    sa.seg = w.seg[cur].p;
    sa.tile_seg = w.tile_seg[cur].p;
    sa.ctr = w.ctr[cur].p;
    sa.part = w.part.p;
    sa.req = w.req.p;
    sa.ntiles = ntiles;
    sa.reverse = (uint32_t)cfg.reverse_tiles;
    ck(launch_sweep(sa, in_buf < 0, cfg.sweep_block, cfg.sweep_ppt, st), "k_sweep");

    ensure(w.nodes, (size_t)nnodes + 2 * (size_t)nseg, st, true);
    fa.nodes = w.nodes.p;
    PlanArgs pl{};
    pl.seg = w.seg[cur].p;
    pl.nseg = nseg;
    pl.ctr = w.ctr[cur].p;
    pl.part = w.part.p;
    pl.seg_out = w.seg[cur ^ 1].p;
    pl.ctr_out = w.ctr[cur ^ 1].p;
    pl.tile_seg_out = w.tile_seg[cur ^ 1].p;
    pl.jobs = w.jobs.p;
    pl.nodes = w.nodes.p;
    pl.node_base = nnodes;
    pl.out_buf = (uint32_t)out_buf;
    pl.status = w.status_dev;
    pl.tile = tile;
    pl.lds_limit = lds_limit;
    ck(launch_plan(pl, st), "k_plan");
    s = read_status(w, st);
    w.stats.push_back({(int64_t)s.nseg, (int64_t)s.swept, (int64_t)s.njobs, (int64_t)s.jobpts});
    ck(launch_finish(fa, s.njobs, tmax, st), "k_finish");
    nseg = s.nseg;
    ntiles = s.ntiles;
    nnodes = s.nnodes;
    level_begin.push_back(nnodes);
    cur ^= 1;
    in_buf = out_buf;
    out_buf ^= 1;
  }

  // assembly
  ensure(w.level_begin, level_begin.size(), st);
  ensure_host_u32(w, level_begin.size());
  std::memcpy(w.h_u32, level_begin.data(), level_begin.size() * sizeof(uint32_t));
  ck(hipMemcpyAsync(w.level_begin.p, w.h_u32, level_begin.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st),
     "hipMemcpyAsync");
  AssembleArgs aa{};
  aa.nodes = w.nodes.p;
  aa.level_begin = w.level_begin.p;
  aa.nlevels = (uint32_t)(level_begin.size() - 1);
  aa.req = w.req.p;
  aa.nreq = (uint32_t)nreq;
  aa.lists[0] = w.wi[0];
  aa.lists[1] = w.wi[1];
  aa.out_idx = out_idx;
  aa.out_count = out_counts;
  aa.nnodes = nnodes;
  ck(launch_assemble(aa, st), "k_assemble");
  ck(launch_copy_lists(aa, st), "k_copy_lists");
  // The staging buffers are reused by the next call: wait for the copies.
  ck(hipStreamSynchronize(st), "hipStreamSynchronize");
}

int guarded(const double* x, const double* y, const int64_t* offsets, int64_t nreq, int64_t* out_idx,
            int64_t* out_counts, vqhull_stream_t stream) {
  try {
    run(x, y, offsets, nreq, out_idx, out_counts, (hipStream_t)stream);
  } catch (const HipFail& f) {
    return f.e == hipErrorOutOfMemory ? VQHULL_ERR_OUT_OF_MEMORY : VQHULL_ERR_HIP;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return VQHULL_ERR_OUT_OF_MEMORY;
  }
  return VQHULL_OK;
}

}  // namespace

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
  std::lock_guard<std::mutex> guard(g_ws_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  auto it = g_ws.find(dev);
  if (it == g_ws.end()) return 0;
  const auto& st = it->second->stats;
  for (int64_t i = 0; i < (int64_t)st.size() && i < cap && out; ++i) {
    out[4 * i + 0] = st[i].segs;
    out[4 * i + 1] = st[i].swept;
    out[4 * i + 2] = st[i].jobs;
    out[4 * i + 3] = st[i].jobpts;
  }
  return (int64_t)st.size();
}

int vqhull_release_workspace(void) {
  std::lock_guard<std::mutex> guard(g_ws_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VQHULL_ERR_HIP;
  auto it = g_ws.find(dev);
  if (it == g_ws.end()) return VQHULL_OK;
  if (hipDeviceSynchronize() != hipSuccess) return VQHULL_ERR_HIP;
  free_workspace(it->second);
  g_ws.erase(it);
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
    default:
      return "unknown status";
  }
}

const char* vqhull_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
