// The batching server's queue (serve_queue.h) driven on the CPU: host lane
// threads take batches exactly as the GPU lanes do and run each request with
// the oracle's hull instead of the device pipeline.  Built with g++ by
// tests/test_serve_queue.py, which writes the requests, runs this program and
// checks what it records.
//
// usage: fake_serve IN OUT lanes lane_points lane_requests submitters chunk delay_us stop_early
//   IN   int64 count, int64 n[count], then x and y of every request (float64,
//        requests one after another)
//   OUT  int64 header {count, submit_after_stop_rejected, unknown_ticket_rejected,
//        polled, watchdog_early, watchdog_late, watchdog_unknown}, the polled
//        ticket ids in poll order, int64 counters
//        {submitted, completed, failed, batches, points, pending}, float64
//        {busy_seconds, now}, then per ticket, in ticket order, int64
//        {request from the payload, request from the submit's first ticket,
//        n, batch, lane, status, done, wait_status, count} + float64
//        {t_submit, t_start, t_done} and `count` int64 vertex indices.
// Requests are submitted by `submitters` threads, request i by thread
// i % submitters in groups of `chunk` (chunk 1: one submit per request); each
// lane sleeps delay_us per batch so that requests pile up.  stop_early: stop
// the queue right after the last submit, before any wait.  Watchdog: the last
// ticket is looked at once (zero timeout) right after the last submit, then
// waited for with a 60 s timeout after the drain; the ticket after it (unknown)
// with a short timeout.  Each records wait_for's result (1 done, 0 timed out,
// -1 unknown ticket).
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "serve_queue.h"

extern "C" int vqhull_oracle_hull(const double* x, const double* y, int64_t n, int64_t* out_idx,
                                  int64_t* out_count);

namespace {

struct Req {
  int64_t id;  // request number in the input file
};

bool read_all(FILE* f, void* p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; }

}  // namespace

int main(int argc, char** argv) {
  if (argc != 10) {
    fprintf(stderr, "usage: fake_serve IN OUT lanes lane_points lane_requests submitters chunk delay_us stop_early\n");
    return 2;
  }
  const int lanes = atoi(argv[3]);
  const int64_t lane_points = atoll(argv[4]), lane_requests = atoll(argv[5]);
  const int submitters = atoi(argv[6]);
  const int64_t chunk = atoll(argv[7]);
  const int delay_us = atoi(argv[8]);
  const bool stop_early = atoi(argv[9]) != 0;

  FILE* in = fopen(argv[1], "rb");
  if (!in) return 3;
  int64_t count = 0;
  if (!read_all(in, &count, 8) || count < 0) return 3;
  std::vector<int64_t> n((size_t)count), off((size_t)count + 1, 0);
  if (!read_all(in, n.data(), 8 * (size_t)count)) return 3;
  for (int64_t i = 0; i < count; ++i) off[(size_t)i + 1] = off[(size_t)i] + n[(size_t)i];
  const int64_t total = off[(size_t)count];
  std::vector<double> x((size_t)total), y((size_t)total);
  if (!read_all(in, x.data(), 8 * (size_t)total) || !read_all(in, y.data(), 8 * (size_t)total)) return 3;
  fclose(in);

  std::vector<int64_t> out_idx((size_t)total), out_cnt((size_t)count, -1), ticket_of((size_t)count, -1);
  vqh::ServeQueue<Req> q(lane_points, lane_requests);

  std::vector<std::thread> lane_threads;
  for (int l = 0; l < lanes; ++l)
    lane_threads.emplace_back([&, l] {
      std::vector<int64_t> ids;
      std::vector<Req> reqs;
      std::vector<int32_t> status;
      while (q.take(l, ids, reqs)) {
        const double tb = q.now();
        if (delay_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(delay_us));
        status.resize(ids.size());
        for (size_t i = 0; i < reqs.size(); ++i) {
          const int64_t r = reqs[i].id;
          status[i] = vqhull_oracle_hull(x.data() + off[(size_t)r], y.data() + off[(size_t)r], n[(size_t)r],
                                         out_idx.data() + off[(size_t)r], &out_cnt[(size_t)r]);
        }
        q.complete(ids, status, tb, q.now());
      }
    });

  // a poller runs beside the submitters and the lanes until every ticket is back
  std::vector<int64_t> polled;
  std::atomic<bool> submitted_all{false};
  std::thread poller([&] {
    std::vector<int64_t> buf(7);
    for (;;) {
      const int64_t k = q.poll(buf.data(), (int64_t)buf.size());
      polled.insert(polled.end(), buf.begin(), buf.begin() + k);
      if ((int64_t)polled.size() >= count && submitted_all.load()) break;
      if (k == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
  });

  std::vector<std::thread> subs;
  std::atomic<int> submit_failures{0};
  for (int s = 0; s < submitters; ++s)
    subs.emplace_back([&, s] {
      std::vector<Req> group;
      std::vector<int64_t> sizes, which;
      auto flush = [&] {
        if (group.empty()) return;
        int64_t first = -1;
        if (!q.submit(group.data(), sizes.data(), (int64_t)group.size(), &first)) ++submit_failures;
        for (size_t k = 0; k < which.size(); ++k) ticket_of[(size_t)which[k]] = first + (int64_t)k;
        group.clear();
        sizes.clear();
        which.clear();
      };
      for (int64_t i = s; i < count; i += submitters) {
        group.push_back(Req{i});
        sizes.push_back(n[(size_t)i]);
        which.push_back(i);
        if ((int64_t)group.size() == chunk) flush();
      }
      flush();
    });
  for (auto& t : subs) t.join();
  submitted_all = true;
  int32_t wd_status = 0;
  const int64_t wd_early = count > 0 ? q.wait_for(count - 1, 0.0, &wd_status) : -2;

  int64_t after_stop_rejected = 0;
  if (stop_early) {
    q.stop();
    for (auto& t : lane_threads) t.join();  // the lanes finish everything pending first
    Req r{0};
    int64_t one = 1, first = -1;
    after_stop_rejected = q.submit(&r, &one, 1, &first) ? 0 : 1;
  } else {
    q.drain();
  }
  poller.join();
  std::vector<int32_t> wait_status((size_t)count, -1);
  for (int64_t t = 0; t < count; ++t) q.wait(t, &wait_status[(size_t)t]);
  int32_t dummy = 0;
  vqh::ServeQueue<Req>::Ticket probe;
  const int64_t unknown_rejected = (!q.wait(count, &dummy) && !q.wait(-1, &dummy) && !q.info(count, &probe)) ? 1 : 0;
  const auto c = q.counters();
  const int64_t wd_late = count > 0 ? q.wait_for(count - 1, 60.0, &wd_status) : -2;
  const int64_t wd_unknown = q.wait_for(count, 0.01, &wd_status);
  if (!stop_early) {
    q.stop();
    for (auto& t : lane_threads) t.join();
    Req r{0};
    int64_t one = 1, first = -1;
    after_stop_rejected = q.submit(&r, &one, 1, &first) ? 0 : 1;
  }
  if (submit_failures.load() != 0) return 4;

  FILE* out = fopen(argv[2], "wb");
  if (!out) return 5;
  const int64_t head[7] = {count, after_stop_rejected, unknown_rejected, (int64_t)polled.size(),
                           wd_early, wd_late, wd_unknown};
  fwrite(head, 8, 7, out);
  fwrite(polled.data(), 8, polled.size(), out);
  const int64_t ci[6] = {c.submitted, c.completed, c.failed, c.batches, c.points, c.pending};
  const double cd[2] = {c.busy_seconds, c.now};
  fwrite(ci, 8, 6, out);
  fwrite(cd, 8, 2, out);
  std::vector<int64_t> req_of((size_t)count, -1);
  for (int64_t r = 0; r < count; ++r)
    if (ticket_of[(size_t)r] >= 0 && ticket_of[(size_t)r] < count) req_of[(size_t)ticket_of[(size_t)r]] = r;
  for (int64_t t = 0; t < count; ++t) {
    vqh::ServeQueue<Req>::Ticket k;
    q.info(t, &k);
    const int64_t r = req_of[(size_t)t];
    const int64_t cnt = r >= 0 && out_cnt[(size_t)r] > 0 ? out_cnt[(size_t)r] : 0;
    const int64_t vi[9] = {k.r.id, r, k.n, k.batch, k.lane, k.status, k.done ? 1 : 0, wait_status[(size_t)t], cnt};
    const double vd[3] = {k.t_submit, k.t_start, k.t_done};
    fwrite(vi, 8, 9, out);
    fwrite(vd, 8, 3, out);
    if (cnt > 0) fwrite(out_idx.data() + off[(size_t)r], 8, (size_t)cnt, out);
  }
  fclose(out);
  return 0;
}
