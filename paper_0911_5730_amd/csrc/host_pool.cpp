// A small persistent pool of host threads for the set-up's per-substructure
// and per-node loops.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "common.hpp"

namespace bddc {

namespace {

class Pool {
 public:
  Pool() {
    unsigned hw = std::thread::hardware_concurrency();
    nthreads_ = (int)std::max(1u, std::min(hw ? hw : 1u, 8u));
    for (int t = 1; t < nthreads_; ++t) std::thread([this] { worker(); }).detach();
  }
  int size() const { return nthreads_; }

  void run(int n, int chunk, const std::function<void(int, int)>& body) {
    std::unique_lock<std::mutex> run_lk(run_mu_);   // one parallel loop at a time
    {
      std::lock_guard<std::mutex> lk(mu_);
      body_ = &body;
      n_ = n;
      chunk_ = chunk;
      next_.store(0);
      active_.store(nthreads_ - 1);
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    work();
    // the loops of a set-up are short: wait for the workers by spinning
    while (active_.load(std::memory_order_acquire) != 0) std::this_thread::yield();
    body_ = nullptr;
  }

 private:
  void work() {
    for (;;) {
      const int b = next_.fetch_add(chunk_);
      if (b >= n_) break;
      (*body_)(b, std::min(n_, b + chunk_));
    }
  }
  void worker() {
    unsigned seen = 0;
    for (;;) {
      // a set-up issues its parallel loops in quick succession: spin for a
      // while (about a millisecond) before sleeping on the condition variable
      bool got = false;
      for (int i = 0; i < 20000 && !got; ++i) {
        got = gen_.load(std::memory_order_acquire) != seen;
        if (!got && (i & 63) == 63) std::this_thread::yield();
      }
      if (!got) {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_.load(std::memory_order_acquire) != seen; });
      }
      seen = gen_.load(std::memory_order_acquire);
      work();
      active_.fetch_sub(1, std::memory_order_acq_rel);
    }
  }
  int nthreads_ = 1;
  std::mutex run_mu_, mu_;
  std::condition_variable cv_;
  const std::function<void(int, int)>* body_ = nullptr;
  std::atomic<int> next_{0};
  int n_ = 0, chunk_ = 1;
  std::atomic<int> active_{0};
  std::atomic<unsigned> gen_{0};
};

Pool& pool() {
  static Pool* p = new Pool();   // never destroyed: its threads are detached
  return *p;
}

}  // namespace

void parallel_for(int n, int chunk, const std::function<void(int, int)>& body) {
  if (n <= 0) return;
  chunk = std::max(1, chunk);
  Pool& P = pool();
  if (P.size() == 1 || n <= chunk) {
    body(0, n);
    return;
  }
  P.run(n, chunk, body);
}

}  // namespace bddc
