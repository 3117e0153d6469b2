// Continuous-batching hull server (C ABI in include/vqhull.h).
//
// Requests (device arrays owned by the caller) enter a FIFO.  The server runs
// `lanes` batch lanes, each with its own HIP stream, engine context and
// pre-allocated batch buffers, and a host thread that loops:
//   take the oldest pending requests that fit the lane (points and request
//   count), run the batched hull on the lane's context (a captured graph whose
//   kernels read each request's points where the caller keeps them; the
//   rare plain fallback first gathers them into the lane's staging arrays),
//   scatter every request's vertex list and count into the caller's buffers
//   (one kernel), then mark the requests done.
// A request that arrives while batches are on the GPU is taken by the next
// lane that frees up, so work of different batches overlaps on the device;
// admission is by the lane's fixed device memory, sized once at creation, so
// serving allocates nothing.  The tickets, the FIFO and its admission rule
// live in serve_queue.h, which holds no GPU state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/vqhull.h"
#include "serve_queue.h"
#include "vqhull_internal.h"

using namespace vqh;

namespace {

struct Lane {
  int index = 0;
  Context* ctx = nullptr;
  hipStream_t st = nullptr;
  std::thread th;
  // device batch buffers
  double* sx = nullptr;
  double* sy = nullptr;
  int64_t* sidx = nullptr;
  int64_t* scnt = nullptr;
  ServedReq* d_reqs = nullptr;
  ServedChunk* d_chunks = nullptr;
  // pinned host tables
  ServedReq* h_reqs = nullptr;
  ServedChunk* h_chunks = nullptr;
  int64_t* h_off = nullptr;
  int64_t* h_cnt = nullptr;
  uint32_t* d_nchunks = nullptr;
  uint32_t* h_nchunks = nullptr;
  // each request's own arrays, for the graph path (its kernels read them in place)
  std::vector<const double*> xs, ys;
  // the batch step as one hipGraph (graph_levels > 0)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t graph_gen = 0;
  vqhull_config graph_cfg{};
  bool graph_broken = false;
  std::atomic<int64_t> graph_batches{0}, fallback_batches{0};
};

}  // namespace

struct vqhull_server {
  vqhull_server_config cfg{};
  int device = 0;
  int64_t max_chunks = 0;
  std::vector<Lane*> lanes;
  std::unique_ptr<ServeQueue<ServedReq>> q;  // tickets, FIFO admission, completion
};

namespace {

int hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? VQHULL_ERR_OUT_OF_MEMORY : VQHULL_ERR_HIP; }

void free_lane(Lane* L) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  auto h = [](void* p) {
    if (p) (void)hipHostFree(p);
  };
  if (L->st) (void)hipStreamSynchronize(L->st);
  if (L->exec) (void)hipGraphExecDestroy(L->exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  f(L->d_nchunks);
  h(L->h_nchunks);
  f(L->sx);
  f(L->sy);
  f(L->sidx);
  f(L->scnt);
  f(L->d_reqs);
  f(L->d_chunks);
  h(L->h_reqs);
  h(L->h_chunks);
  h(L->h_off);
  h(L->h_cnt);
  context_destroy(L->ctx);
  if (L->st) (void)hipStreamDestroy(L->st);
  delete L;
}

int make_lane(vqhull_server* s, int index, Lane** out) {
  Lane* L = new Lane();
  L->index = index;
  const size_t P = (size_t)s->cfg.lane_points, R = (size_t)s->cfg.lane_requests, C = (size_t)s->max_chunks;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
  };
  chk(hipStreamCreateWithFlags(&L->st, hipStreamNonBlocking));
  chk(hipMalloc(&L->sx, std::max<size_t>(P, 1) * sizeof(double)));
  chk(hipMalloc(&L->sy, std::max<size_t>(P, 1) * sizeof(double)));
  chk(hipMalloc(&L->sidx, std::max<size_t>(P, 1) * sizeof(int64_t)));
  chk(hipMalloc(&L->scnt, R * sizeof(int64_t)));
  chk(hipMalloc(&L->d_reqs, R * sizeof(ServedReq)));
  chk(hipMalloc(&L->d_chunks, C * sizeof(ServedChunk)));
  chk(hipHostMalloc((void**)&L->h_reqs, R * sizeof(ServedReq), hipHostMallocDefault));
  chk(hipHostMalloc((void**)&L->h_chunks, C * sizeof(ServedChunk), hipHostMallocDefault));
  chk(hipHostMalloc((void**)&L->h_off, (R + 1) * sizeof(int64_t), hipHostMallocDefault));
  chk(hipHostMalloc((void**)&L->h_cnt, R * sizeof(int64_t), hipHostMallocDefault));
  chk(hipMalloc(&L->d_nchunks, sizeof(uint32_t)));
  chk(hipHostMalloc((void**)&L->h_nchunks, sizeof(uint32_t), hipHostMallocDefault));
  if (e != hipSuccess) {
    free_lane(L);
    return hip_status(e);
  }
  int st = context_create(&L->ctx);
  if (st == VQHULL_OK)
    st = s->cfg.graph_levels > 0
             ? context_reserve_fixed(L->ctx, (int64_t)P, (int64_t)R, s->cfg.graph_levels, L->st)
             : context_reserve(L->ctx, (int64_t)P, (int64_t)R, L->st);
  if (st != VQHULL_OK) {
    free_lane(L);
    return st;
  }
  *out = L;
  return VQHULL_OK;
}

bool same_config(const vqhull_config& a, const vqhull_config& b) {
  return a.sweep_block == b.sweep_block && a.sweep_ppt == b.sweep_ppt && a.lds_limit == b.lds_limit &&
         a.reverse_tiles == b.reverse_tiles && a.sweep_persistent == b.sweep_persistent &&
         a.level_block == b.level_block;
}

// Capture the lane's whole batch step (table copies, the fixed sequence of
// `levels` recursion levels, assembly, scatter, count copy) as one graph.
// The kernels read every request's points where the caller keeps them (the
// request table carries its arrays), so nothing is gathered.  Every count the
// kernels need is read from device memory, so the graph serves every batch;
// it is captured again when the library's configuration changes or a
// workspace buffer has moved.
bool capture_graph(vqhull_server* s, Lane* L, const vqhull_config& cfg) {
  if (L->exec) (void)hipGraphExecDestroy(L->exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->exec = nullptr;
  L->graph = nullptr;
  const size_t R = (size_t)s->cfg.lane_requests, C = (size_t)s->max_chunks;
  const uint64_t gen = allocation_generation();
  if (hipStreamBeginCapture(L->st, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  bool ok = hipMemcpyAsync(L->d_reqs, L->h_reqs, R * sizeof(ServedReq), hipMemcpyHostToDevice, L->st) == hipSuccess;
  ok = ok && hipMemcpyAsync(L->d_chunks, L->h_chunks, C * sizeof(ServedChunk), hipMemcpyHostToDevice, L->st) ==
                 hipSuccess;
  ok = ok && hipMemcpyAsync(L->d_nchunks, L->h_nchunks, sizeof(uint32_t), hipMemcpyHostToDevice, L->st) == hipSuccess;
  ok = ok && context_enqueue_fixed(L->ctx, L->sx, L->sy, L->sidx, L->scnt, s->cfg.graph_levels, L->st) == VQHULL_OK;
  ok = ok && launch_scatter(L->d_reqs, L->d_chunks, L->d_nchunks, (uint32_t)C, L->sidx, L->scnt, L->st) == 0;
  ok = ok && hipMemcpyAsync(L->h_cnt, L->scnt, R * sizeof(int64_t), hipMemcpyDeviceToHost, L->st) == hipSuccess;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(L->st, &g);
  if (!ok || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  }
  if (hipGraphInstantiate(&L->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    L->exec = nullptr;
    return false;
  }
  L->graph = g;
  L->graph_gen = gen;
  L->graph_cfg = cfg;
  return true;
}

// Run one batch on lane L (the requests as copied from their tickets under the
// server lock); returns a VQHULL status for the batch.
int run_batch(vqhull_server* s, Lane* L, const std::vector<ServedReq>& reqs) {
  const size_t nreq = reqs.size();
  size_t nch = 0;
  int64_t off = 0;
  L->xs.resize(nreq);
  L->ys.resize(nreq);
  for (size_t i = 0; i < nreq; ++i) {
    ServedReq r = reqs[i];
    r.off = (uint64_t)off;
    L->h_reqs[i] = r;
    L->h_off[i] = off;
    L->xs[i] = r.x;
    L->ys[i] = r.y;
    const uint64_t nc = r.n > 0 ? (r.n + kServeChunk - 1) / kServeChunk : 1;
    for (uint64_t c = 0; c < nc; ++c) L->h_chunks[nch++] = ServedChunk{(uint32_t)i, (uint32_t)(c * kServeChunk)};
    off += (int64_t)r.n;
  }
  L->h_off[nreq] = off;
  *L->h_nchunks = (uint32_t)nch;

  if (s->cfg.graph_levels > 0 && !L->graph_broken) {
    vqhull_config cfg;
    (void)vqhull_get_config(&cfg);
    if (cfg.sweep_persistent &&
        context_stage(L->ctx, L->h_off, (int64_t)nreq, L->xs.data(), L->ys.data()) == VQHULL_OK) {
      if (!L->exec || L->graph_gen != allocation_generation() || !same_config(cfg, L->graph_cfg)) {
        if (!capture_graph(s, L, cfg)) L->graph_broken = true;  // this lane stays on the plain path
      }
      if (L->exec) {
        hipError_t e = hipGraphLaunch(L->exec, L->st);
        if (e == hipSuccess) e = hipStreamSynchronize(L->st);
        if (e != hipSuccess) return hip_status(e);
        if (context_fixed_done(L->ctx, s->cfg.graph_levels)) {
          ++L->graph_batches;
          return VQHULL_OK;
        }
        // deeper recursion than captured, or a full table: compute again below
      }
    }
  }

  // plain launches on a gathered copy of the batch (the recursion went deeper
  // than the captured levels, or no graph): rare
  ++L->fallback_batches;
  hipError_t e = hipMemcpyAsync(L->d_reqs, L->h_reqs, nreq * sizeof(ServedReq), hipMemcpyHostToDevice, L->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(L->d_chunks, L->h_chunks, nch * sizeof(ServedChunk), hipMemcpyHostToDevice, L->st);
  if (e == hipSuccess) e = hipMemcpyAsync(L->d_nchunks, L->h_nchunks, sizeof(uint32_t), hipMemcpyHostToDevice, L->st);
  if (e == hipSuccess)
    e = (hipError_t)launch_gather(L->d_reqs, L->d_chunks, L->d_nchunks, (uint32_t)nch, L->sx, L->sy, L->st);
  if (e != hipSuccess) return hip_status(e);
  const int st = context_run(L->ctx, L->sx, L->sy, L->h_off, (int64_t)nreq, L->sidx, L->scnt, L->st);
  if (st != VQHULL_OK) return st;
  e = (hipError_t)launch_scatter(L->d_reqs, L->d_chunks, L->d_nchunks, (uint32_t)nch, L->sidx, L->scnt, L->st);
  if (e == hipSuccess) e = hipMemcpyAsync(L->h_cnt, L->scnt, nreq * sizeof(int64_t), hipMemcpyDeviceToHost, L->st);
  if (e == hipSuccess) e = hipStreamSynchronize(L->st);
  return e == hipSuccess ? VQHULL_OK : hip_status(e);
}

void lane_loop(vqhull_server* s, Lane* L) {
  (void)hipSetDevice(s->device);
  std::vector<int64_t> ids;
  std::vector<ServedReq> reqs;
  std::vector<int32_t> status;
  while (s->q->take(L->index, ids, reqs)) {
    const double tb = s->q->now();
    const int st = run_batch(s, L, reqs);
    const double te = s->q->now();
    status.resize(ids.size());
    for (size_t i = 0; i < ids.size(); ++i)
      status[i] = st != VQHULL_OK ? st : L->h_cnt[i] < 0 ? (int32_t)(-L->h_cnt[i]) : VQHULL_OK;
    s->q->complete(ids, status, tb, te);
  }
}

}  // namespace

extern "C" {

int vqhull_server_create(const vqhull_server_config* cfg, vqhull_server** out) {
  if (!cfg || !out) return VQHULL_ERR_INVALID_ARGUMENT;
  if (cfg->lanes < 1 || cfg->lanes > 8 || cfg->lane_points < 1 || cfg->lane_points >= (int64_t(1) << 31) ||
      cfg->lane_requests < 1 || cfg->lane_requests > (int64_t(1) << 24) || cfg->graph_levels < 0 ||
      cfg->graph_levels > 64)
    return VQHULL_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  vqhull_server* s = new vqhull_server();
  s->cfg = *cfg;
  s->q.reset(new ServeQueue<ServedReq>(cfg->lane_points, cfg->lane_requests));
  s->max_chunks = cfg->lane_points / kServeChunk + cfg->lane_requests + 1;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return VQHULL_ERR_HIP;
  }
  for (int i = 0; i < cfg->lanes; ++i) {
    Lane* L = nullptr;
    const int st = make_lane(s, i, &L);
    if (st != VQHULL_OK) {
      for (Lane* l : s->lanes) free_lane(l);
      delete s;
      return st;
    }
    s->lanes.push_back(L);
  }
  for (Lane* L : s->lanes) L->th = std::thread(lane_loop, s, L);
  *out = s;
  return VQHULL_OK;
}

int vqhull_server_submit(vqhull_server* s, const double* x, const double* y, int64_t n, int64_t* out_idx,
                         int64_t* out_count, int64_t* ticket) {
  if (!s || !ticket || !out_count || n < 0 || n > s->cfg.lane_points) return VQHULL_ERR_INVALID_ARGUMENT;
  if (n > 0 && (!x || !y || !out_idx)) return VQHULL_ERR_INVALID_ARGUMENT;
  ServedReq r{};
  r.x = x;
  r.y = y;
  r.out_idx = out_idx;
  r.out_count = out_count;
  r.n = (uint64_t)n;
  return s->q->submit(&r, &n, 1, ticket) ? VQHULL_OK : VQHULL_ERR_INVALID_ARGUMENT;
}

int vqhull_server_submit_batch(vqhull_server* s, int64_t count, const double* const* x, const double* const* y,
                               const int64_t* n, int64_t* const* out_idx, int64_t* const* out_count,
                               int64_t* first_ticket) {
  if (!s || !first_ticket || count < 0) return VQHULL_ERR_INVALID_ARGUMENT;
  if (count > 0 && (!x || !y || !n || !out_idx || !out_count)) return VQHULL_ERR_INVALID_ARGUMENT;
  for (int64_t i = 0; i < count; ++i) {
    if (!out_count[i] || n[i] < 0 || n[i] > s->cfg.lane_points) return VQHULL_ERR_INVALID_ARGUMENT;
    if (n[i] > 0 && (!x[i] || !y[i] || !out_idx[i])) return VQHULL_ERR_INVALID_ARGUMENT;
  }
  std::vector<ServedReq> r((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    r[(size_t)i].x = x[i];
    r[(size_t)i].y = y[i];
    r[(size_t)i].out_idx = out_idx[i];
    r[(size_t)i].out_count = out_count[i];
    r[(size_t)i].n = (uint64_t)n[i];
  }
  return s->q->submit(r.data(), n, count, first_ticket) ? VQHULL_OK : VQHULL_ERR_INVALID_ARGUMENT;
}

int vqhull_server_wait(vqhull_server* s, int64_t ticket) {
  if (!s) return VQHULL_ERR_INVALID_ARGUMENT;
  int32_t st = 0;
  return s->q->wait(ticket, &st) ? st : VQHULL_ERR_INVALID_ARGUMENT;
}

int vqhull_server_wait_timeout(vqhull_server* s, int64_t ticket, double seconds) {
  if (!s || !(seconds >= 0.0 && seconds <= 1e6)) return VQHULL_ERR_INVALID_ARGUMENT;
  int32_t st = 0;
  const int r = s->q->wait_for(ticket, seconds, &st);
  return r > 0 ? st : r == 0 ? VQHULL_ERR_TIMEOUT : VQHULL_ERR_INVALID_ARGUMENT;
}

int64_t vqhull_server_poll(vqhull_server* s, int64_t* tickets, int64_t cap) {
  if (!s || cap < 0 || (cap > 0 && !tickets)) return -VQHULL_ERR_INVALID_ARGUMENT;
  return s->q->poll(tickets, cap);
}

int vqhull_server_drain(vqhull_server* s) {
  if (!s) return VQHULL_ERR_INVALID_ARGUMENT;
  s->q->drain();
  return VQHULL_OK;
}

int vqhull_server_ticket_info(vqhull_server* s, int64_t ticket, vqhull_ticket_info* out) {
  if (!s || !out) return VQHULL_ERR_INVALID_ARGUMENT;
  ServeQueue<ServedReq>::Ticket t;
  if (!s->q->info(ticket, &t)) return VQHULL_ERR_INVALID_ARGUMENT;
  out->n = t.n;
  out->batch = t.batch;
  out->lane = t.lane;
  out->status = t.status;
  out->done = t.done ? 1 : 0;
  out->t_submit = t.t_submit;
  out->t_start = t.t_start;
  out->t_done = t.t_done;
  return VQHULL_OK;
}

int vqhull_server_stats(vqhull_server* s, vqhull_server_counters* out) {
  if (!s || !out) return VQHULL_ERR_INVALID_ARGUMENT;
  const ServeQueue<ServedReq>::Counters c = s->q->counters();
  out->submitted = c.submitted;
  out->completed = c.completed;
  out->failed = c.failed;
  out->batches = c.batches;
  out->points = c.points;
  out->pending = c.pending;
  out->busy_seconds = c.busy_seconds;
  out->now = c.now;
  out->graph_batches = 0;
  out->plain_batches = 0;
  for (const Lane* L : s->lanes) {
    out->graph_batches += L->graph_batches.load();
    out->plain_batches += L->fallback_batches.load();
  }
  return VQHULL_OK;
}

int vqhull_server_destroy(vqhull_server* s) {
  if (!s) return VQHULL_ERR_INVALID_ARGUMENT;
  s->q->stop();
  for (Lane* L : s->lanes)
    if (L->th.joinable()) L->th.join();
  for (Lane* L : s->lanes) free_lane(L);
  delete s;
  return VQHULL_OK;
}

}  // extern "C"
