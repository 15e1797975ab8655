// Counting semaphore for the coarsest-level solves that use grid barriers.
//
// Such a solve launches at most 1/16 of the device's resident work-groups
// and spins at software grid barriers until every one of its work-groups has
// arrived, so it is only safe while all of them are resident at once: at
// most kGridSolves such solves may be in flight on one device.  A scene holds
// a ticket for the whole quasi-Newton solve of a step (its last
// synchronisation ends every solve it launched) and waits for one when all
// are taken, so that its arithmetic never depends on what else runs.
#pragma once

#include <condition_variable>
#include <mutex>

namespace hot {

constexpr int kGridSolves = 16;

class TicketPool {
 public:
  explicit TicketPool(int n) : free_(n) {}
  bool try_acquire() {
    std::lock_guard<std::mutex> lk(mu_);
    if (free_ == 0) return false;
    --free_;
    return true;
  }
  void acquire() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return free_ > 0; });
    --free_;
  }
  void release() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      ++free_;
    }
    cv_.notify_one();
  }
  int available() {
    std::lock_guard<std::mutex> lk(mu_);
    return free_;
  }

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  int free_;
};

}  // namespace hot
