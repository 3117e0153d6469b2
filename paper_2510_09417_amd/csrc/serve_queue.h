// The host-side request queue of the batching server, with no GPU types: the
// server's lanes run the batches on the device; the CPU tests run them with a
// host executor.
//
// Requests enter a FIFO.  A lane takes the oldest pending requests that fit
// it: at most `lane_requests` requests and at most `lane_points` points in
// total (the first request is always taken; submitters reject requests larger
// than a lane).  The lane runs them and completes them together; completed
// tickets are kept for wait / poll / info with their submit, start and done
// times on one steady clock.  After stop(), lanes still take every pending
// request and then see take() return false.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <vector>

namespace vqh {

template <typename Payload>
class ServeQueue {
 public:
  struct Ticket {
    Payload r{};
    int64_t n = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    int64_t batch = -1;
    int32_t lane = -1;
    int32_t status = 0;
    bool done = false;
  };
  struct Counters {
    int64_t submitted = 0, completed = 0, failed = 0, batches = 0, points = 0, pending = 0;
    double busy_seconds = 0, now = 0;
  };

  ServeQueue(int64_t lane_points, int64_t lane_requests)
      : lane_points_(lane_points), lane_requests_(lane_requests), t0_(std::chrono::steady_clock::now()) {}

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count(); }

  // Enqueue count requests (payload and size each); false once stopping.
  bool submit(const Payload* r, const int64_t* n, int64_t count, int64_t* first_ticket) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopping_) return false;
      const double t = now();
      *first_ticket = (int64_t)tickets_.size();
      for (int64_t i = 0; i < count; ++i) {
        Ticket k;
        k.r = r[i];
        k.n = n[i];
        k.t_submit = t;
        pending_.push_back((int64_t)tickets_.size());
        tickets_.push_back(k);
      }
    }
    if (count == 1)
      cv_work_.notify_one();
    else
      cv_work_.notify_all();
    return true;
  }

  // Block until there is work; take the oldest pending requests that fit the
  // lane.  False when stopping with nothing pending.
  bool take(int lane, std::vector<int64_t>& ids, std::vector<Payload>& reqs) {
    ids.clear();
    reqs.clear();
    std::unique_lock<std::mutex> lk(mu_);
    cv_work_.wait(lk, [&] { return stopping_ || !pending_.empty(); });
    if (pending_.empty()) return false;
    int64_t pts = 0;
    while (!pending_.empty() && (int64_t)ids.size() < lane_requests_) {
      const Ticket& t = tickets_[(size_t)pending_.front()];
      if (!ids.empty() && pts + t.n > lane_points_) break;
      pts += t.n;
      ids.push_back(pending_.front());
      reqs.push_back(t.r);
      pending_.pop_front();
    }
    const double ts = now();
    for (int64_t id : ids) {
      tickets_[(size_t)id].t_start = ts;
      tickets_[(size_t)id].lane = lane;
    }
    return true;
  }

  // Complete a taken batch: status[i] for ids[i]; the batch ran on the lane
  // from t_begin to t_end.
  void complete(const std::vector<int64_t>& ids, const std::vector<int32_t>& status, double t_begin, double t_end) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      const int64_t b = batches_++;
      busy_ += t_end - t_begin;
      for (size_t i = 0; i < ids.size(); ++i) {
        Ticket& t = tickets_[(size_t)ids[i]];
        t.batch = b;
        t.t_done = t_end;
        t.status = status[i];
        if (t.status != 0) ++failed_;
        t.done = true;
        points_ += t.n;
        ++completed_;
        unpolled_.push_back(ids[i]);
      }
    }
    cv_done_.notify_all();
  }

  // The status of a ticket once done; false for an unknown ticket.
  bool wait(int64_t ticket, int32_t* status) {
    std::unique_lock<std::mutex> lk(mu_);
    if (ticket < 0 || ticket >= (int64_t)tickets_.size()) return false;
    cv_done_.wait(lk, [&] { return tickets_[(size_t)ticket].done; });
    *status = tickets_[(size_t)ticket].status;
    return true;
  }

  // As wait, for at most `seconds` (0: look once): 1 with the status once
  // done, 0 if the ticket is still pending or running at the deadline (it is
  // not cancelled and completes later), -1 for an unknown ticket.
  int wait_for(int64_t ticket, double seconds, int32_t* status) {
    std::unique_lock<std::mutex> lk(mu_);
    if (ticket < 0 || ticket >= (int64_t)tickets_.size()) return -1;
    const bool done = cv_done_.wait_for(lk, std::chrono::duration<double>(seconds),
                                        [&] { return tickets_[(size_t)ticket].done; });
    if (!done) return 0;
    *status = tickets_[(size_t)ticket].status;
    return 1;
  }

  // Completed tickets not returned before, oldest first, up to cap.
  int64_t poll(int64_t* out, int64_t cap) {
    std::lock_guard<std::mutex> lk(mu_);
    int64_t k = 0;
    while (k < cap && !unpolled_.empty()) {
      out[k++] = unpolled_.front();
      unpolled_.pop_front();
    }
    return k;
  }

  void drain() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return completed_ == (int64_t)tickets_.size(); });
  }

  bool info(int64_t ticket, Ticket* out) {
    std::lock_guard<std::mutex> lk(mu_);
    if (ticket < 0 || ticket >= (int64_t)tickets_.size()) return false;
    *out = tickets_[(size_t)ticket];
    return true;
  }

  Counters counters() {
    std::lock_guard<std::mutex> lk(mu_);
    Counters c;
    c.submitted = (int64_t)tickets_.size();
    c.completed = completed_;
    c.failed = failed_;
    c.batches = batches_;
    c.points = points_;
    c.pending = (int64_t)pending_.size();
    c.busy_seconds = busy_;
    c.now = now();
    return c;
  }

  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stopping_ = true;
    }
    cv_work_.notify_all();
  }

 private:
  const int64_t lane_points_, lane_requests_;
  const std::chrono::steady_clock::time_point t0_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<int64_t> pending_;   // ticket ids, FIFO
  std::vector<Ticket> tickets_;   // by id
  std::deque<int64_t> unpolled_;  // completed, not yet returned by poll
  bool stopping_ = false;
  int64_t batches_ = 0, completed_ = 0, points_ = 0, failed_ = 0;
  double busy_ = 0;  // summed batch time over lanes
};

}  // namespace vqh
