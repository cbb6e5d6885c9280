// Request scheduler of the serving loop: a fixed number of slots (worker
// threads, one device stream each) and a device-memory budget.  A request is
// admitted when a slot is free and its footprint fits into the unreserved
// budget; the queue is FIFO, except that a later request that fits may start
// ahead of a head that does not, at most max_skips times per head (no
// starvation).  Completed requests are handed back in completion order.
//
// Plain C++ (no device code), so the admission logic can be exercised on the
// host with mock jobs.
#pragma once
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

namespace nqs {

inline double mono_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class Job>
class Scheduler {
 public:
  struct Done {
    int64_t ticket = -1;
    Job job{};
    size_t bytes = 0;
    double t_submit = 0, t_start = 0, t_end = 0;
    int status = 0;
  };
  using Runner = std::function<int(Job&, int slot)>;

  Scheduler(int slots, size_t budget, Runner run, int max_skips = 8)
      : budget_(budget), run_(std::move(run)), max_skips_(max_skips) {
    for (int s = 0; s < slots; ++s) workers_.emplace_back([this, s] { worker(s); });
  }

  ~Scheduler() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stopping_ = true;
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }

  // 0: queued; 1: the footprint exceeds the whole budget (never admissible)
  int submit(Job job, size_t bytes, double t_submit, int64_t* ticket) {
    if (bytes > budget_) return 1;
    {
      std::lock_guard<std::mutex> lk(mu_);
      Pending p;
      p.ticket = next_ticket_++;
      p.job = std::move(job);
      p.bytes = bytes;
      p.t_submit = t_submit;
      if (ticket) *ticket = p.ticket;
      queue_.push_back(std::move(p));
    }
    cv_.notify_all();
    return 0;
  }

  bool try_pop_done(Done* out) {
    std::lock_guard<std::mutex> lk(mu_);
    if (done_.empty()) return false;
    *out = std::move(done_.front());
    done_.pop_front();
    return true;
  }

  bool wait_done(Done* out, double timeout_s) {
    std::unique_lock<std::mutex> lk(mu_);
    const auto dl = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    if (!done_cv_.wait_until(lk, dl, [&] { return !done_.empty(); })) return false;
    *out = std::move(done_.front());
    done_.pop_front();
    return true;
  }

  size_t budget() const { return budget_; }
  size_t reserved() { std::lock_guard<std::mutex> lk(mu_); return reserved_; }
  size_t peak_reserved() { std::lock_guard<std::mutex> lk(mu_); return peak_; }
  int in_flight() { std::lock_guard<std::mutex> lk(mu_); return in_flight_; }
  int peak_in_flight() { std::lock_guard<std::mutex> lk(mu_); return peak_in_flight_; }
  size_t queued() { std::lock_guard<std::mutex> lk(mu_); return queue_.size(); }
  int64_t skips() { std::lock_guard<std::mutex> lk(mu_); return total_skips_; }

 private:
  struct Pending {
    int64_t ticket;
    Job job;
    size_t bytes;
    double t_submit;
    int skipped = 0;
  };

  // index of the request to admit next, -1 if none fits now
  long peek_locked() const {
    if (queue_.empty()) return -1;
    const size_t free_b = budget_ - reserved_;
    if (queue_.front().bytes <= free_b) return 0;
    if (queue_.front().skipped >= max_skips_) return -1;
    for (size_t k = 1; k < queue_.size(); ++k)
      if (queue_[k].bytes <= free_b) return long(k);
    return -1;
  }

  void worker(int slot) {
    for (;;) {
      Pending p;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return (stopping_ && queue_.empty()) || peek_locked() >= 0; });
        const long k = peek_locked();
        if (k < 0) return;   // stopping with an empty queue
        if (k > 0) { ++queue_.front().skipped; ++total_skips_; }
        p = std::move(queue_[size_t(k)]);
        queue_.erase(queue_.begin() + k);
        reserved_ += p.bytes;
        if (reserved_ > peak_) peak_ = reserved_;
        ++in_flight_;
        if (in_flight_ > peak_in_flight_) peak_in_flight_ = in_flight_;
      }
      Done d;
      d.ticket = p.ticket;
      d.bytes = p.bytes;
      d.t_submit = p.t_submit;
      d.t_start = mono_seconds();
      d.status = run_(p.job, slot);
      d.t_end = mono_seconds();
      d.job = std::move(p.job);
      {
        std::lock_guard<std::mutex> lk(mu_);
        reserved_ -= p.bytes;
        --in_flight_;
        done_.push_back(std::move(d));
      }
      cv_.notify_all();
      done_cv_.notify_all();
    }
  }

  const size_t budget_;
  Runner run_;
  const int max_skips_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<Pending> queue_;
  std::deque<Done> done_;
  std::vector<std::thread> workers_;
  size_t reserved_ = 0, peak_ = 0;
  int in_flight_ = 0, peak_in_flight_ = 0;
  int64_t next_ticket_ = 0, total_skips_ = 0;
  bool stopping_ = false;
};

}  // namespace nqs
