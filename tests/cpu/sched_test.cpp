// Host-only exercise of the serving scheduler with mock jobs (sleep for a
// given time): prints one line per scenario with the quantities the Python
// test asserts on.
#include "admission.h"

#include <atomic>
#include <cstdio>
#include <random>
#include <vector>

struct MockJob {
  int id = 0;
  int ms = 0;
  int status = 0;
};

int main() {
  using S = nqs::Scheduler<MockJob>;
  // 1. random mix: budget respected, slots respected, all complete, concurrency > 1
  {
    const size_t budget = 1000;
    std::atomic<int> running{0}, max_running{0};
    std::atomic<long> over_budget{0};
    S* sp = nullptr;
    S sched(4, budget, [&](MockJob& j, int) {
      int r = ++running;
      int m = max_running.load();
      while (r > m && !max_running.compare_exchange_weak(m, r)) {}
      if (sp && sp->reserved() > budget) ++over_budget;
      std::this_thread::sleep_for(std::chrono::milliseconds(j.ms));
      --running;
      return j.status;
    });
    sp = &sched;
    std::mt19937 rng(7);
    const int n = 200;
    for (int k = 0; k < n; ++k) {
      MockJob j{k, 1 + int(rng() % 4), 0};
      sched.submit(j, 1 + rng() % 500, nqs::mono_seconds(), nullptr);
    }
    int done = 0;
    S::Done d;
    while (done < n && sched.wait_done(&d, 30.0)) ++done;
    printf("mix done=%d peak_reserved=%zu budget=%zu peak_inflight=%d max_running=%d over=%ld reserved_end=%zu\n",
           done, sched.peak_reserved(), budget, sched.peak_in_flight(), max_running.load(), over_budget.load(),
           sched.reserved());
  }
  // 2. failures free their slot and budget
  {
    S sched(2, 100, [&](MockJob& j, int) {
      std::this_thread::sleep_for(std::chrono::milliseconds(j.ms));
      return j.status;
    });
    for (int k = 0; k < 20; ++k) sched.submit(MockJob{k, 2, k % 3 == 0 ? 2 : 0}, 60, nqs::mono_seconds(), nullptr);
    int done = 0, failed = 0;
    S::Done d;
    while (done < 20 && sched.wait_done(&d, 30.0)) { ++done; failed += d.status != 0; }
    printf("fail done=%d failed=%d reserved_end=%zu inflight_end=%d\n", done, failed, sched.reserved(),
           sched.in_flight());
  }
  // 3. never admissible
  {
    S sched(1, 100, [&](MockJob&, int) { return 0; });
    int64_t t = -1;
    const int rc = sched.submit(MockJob{}, 101, nqs::mono_seconds(), &t);
    printf("oversize rc=%d\n", rc);
  }
  // 4. skip-ahead with aging: a head needing the whole budget behind a running
  //    job, while small jobs keep arriving
  {
    std::vector<int> order;
    std::mutex om;
    S sched(2, 100, [&](MockJob& j, int) {
      { std::lock_guard<std::mutex> lk(om); order.push_back(j.id); }
      std::this_thread::sleep_for(std::chrono::milliseconds(j.ms));
      return 0;
    }, 3);
    sched.submit(MockJob{0, 30, 0}, 50, nqs::mono_seconds(), nullptr);     // occupies half the budget
    std::this_thread::sleep_for(std::chrono::milliseconds(5));
    sched.submit(MockJob{1, 1, 0}, 100, nqs::mono_seconds(), nullptr);     // head: needs everything
    for (int k = 2; k < 12; ++k) sched.submit(MockJob{k, 20, 0}, 40, nqs::mono_seconds(), nullptr);
    int done = 0;
    S::Done d;
    while (done < 12 && sched.wait_done(&d, 30.0)) ++done;
    int pos_big = -1;
    for (size_t k = 0; k < order.size(); ++k) if (order[k] == 1) pos_big = int(k);
    printf("aging done=%d big_started_at=%d skips=%lld\n", done, pos_big, (long long)sched.skips());
  }
  // 5. FIFO with one slot and equal sizes
  {
    std::vector<int> order;
    S sched(1, 10, [&](MockJob& j, int) { order.push_back(j.id); return 0; });
    for (int k = 0; k < 30; ++k) sched.submit(MockJob{k, 0, 0}, 10, nqs::mono_seconds(), nullptr);
    int done = 0;
    S::Done d;
    while (done < 30 && sched.wait_done(&d, 30.0)) ++done;
    bool inorder = order.size() == 30;
    for (int k = 0; k < int(order.size()); ++k) inorder = inorder && order[k] == k;
    printf("fifo done=%d inorder=%d\n", done, inorder ? 1 : 0);
  }
  return 0;
}
