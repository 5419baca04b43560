// Host threads that share the step rule of long active lists (host code only).
#pragma once

#include <condition_variable>
#include <cstdint>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace tsbts {

// Host threads for the step rule of long active lists: run(f) calls f(part, parts) for
// every part, the calling thread taking part 0, and returns when all have returned.
class RulePool {
 public:
  // Throws if a thread cannot be started; the threads started until then are joined.
  explicit RulePool(int threads) : parts_(threads) {
    try {
      for (int w = 1; w < threads; ++w) workers_.emplace_back([this, w] { loop(w); });
    } catch (...) {
      stop_all();
      throw;
    }
  }
  ~RulePool() { stop_all(); }
  int parts() const { return parts_; }
  // f(part, parts) for every part, part 0 on the calling thread; returns when all parts
  // have ended, then rethrows the first exception a part threw (if any).
  void run(const std::function<void(int, int)> &f) {
    {
      std::lock_guard<std::mutex> lk(m_);
      job_ = &f;
      remaining_ = parts_ - 1;
      error_ = nullptr;
      ++generation_;
    }
    start_.notify_all();
    std::exception_ptr own;
    try {
      f(0, parts_);
    } catch (...) {
      own = std::current_exception();
    }
    std::unique_lock<std::mutex> lk(m_);
    done_.wait(lk, [this] { return remaining_ == 0; });
    job_ = nullptr;
    if (own) std::rethrow_exception(own);
    if (error_) std::rethrow_exception(error_);
  }

 private:
  void stop_all() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
    }
    start_.notify_all();
    for (auto &th : workers_) th.join();
    workers_.clear();
  }
  void loop(int w) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int, int)> *job;
      {
        std::unique_lock<std::mutex> lk(m_);
        start_.wait(lk, [&] { return stop_ || generation_ != seen; });
        if (stop_) return;
        seen = generation_;
        job = job_;
      }
      std::exception_ptr err;
      try {
        (*job)(w, parts_);
      } catch (...) {
        err = std::current_exception();
      }
      std::lock_guard<std::mutex> lk(m_);
      if (err && !error_) error_ = err;
      if (--remaining_ == 0) done_.notify_one();
    }
  }
  int parts_;
  std::vector<std::thread> workers_;
  std::mutex m_;
  std::condition_variable start_, done_;
  const std::function<void(int, int)> *job_ = nullptr;
  std::exception_ptr error_;
  uint64_t generation_ = 0;
  int remaining_ = 0;
  bool stop_ = false;
};

}  // namespace tsbts
