// Concurrent execution of complete solves (rfd_batch_run, rfd_server_*):
// worker threads with one HIP stream each, a request queue with admission by
// device-memory footprint, one job at a time per pencil, and release of idle
// pencils' caches (least recently used first) when memory is short.
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/rfd.h"
#include "rfd_common.hpp"

namespace rfd {

// Pencil-side hooks (capi.cpp).
int64_t pencil_estimate(rfd_pencil_t p, const rfd_job& j);  // footprint of a job
int64_t pencil_held(rfd_pencil_t p);                        // bytes the pencil holds now
void pencil_release(rfd_pencil_t p);                        // drop its solve caches
void pencil_check(rfd_pencil_t p);                          // partition set, else throws

class Executor {
 public:
  Executor(int workers, int64_t budget);
  ~Executor();  // finishes every submitted request
  Executor(const Executor&) = delete;
  Executor& operator=(const Executor&) = delete;

  int64_t submit(rfd_pencil_t pencil, const rfd_job& job);
  // 1: finished (result copied, id retired); 0: pending; throws for an unknown id
  int poll(int64_t id, bool wait, rfd_result* out);
  void stats(int32_t* queued, int32_t* running, int64_t* bytes_running, int64_t* bytes_cached,
             int64_t* evictions);
  // admitted jobs whose pencil still held device caches from an earlier job
  // (hits) or held none (first use, or released for room: misses)
  void cache_stats(int64_t* hits, int64_t* misses);

 private:
  using Clock = std::chrono::steady_clock;
  struct Req {
    int64_t id = 0;
    rfd_pencil_t pencil = nullptr;
    rfd_job job{};
    int64_t bytes = 0;
    Clock::time_point t_sub, t_start;
    int state = 0;  // 0 queued, 1 running, 2 done
    int bypassed = 0;
    rfd_result res{};
  };

  void loop(int w);
  Req* pick_locked();
  bool fits_locked(const Req& r);
  void run(Req& r, hipStream_t st, DevBuf& Q, int w);

  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<int64_t> queue_;
  std::map<int64_t, Req> reqs_;
  std::map<rfd_pencil_t, bool> busy_;
  std::map<rfd_pencil_t, int64_t> held_, lru_;
  std::vector<std::thread> threads_;
  int64_t budget_ = 0, running_bytes_ = 0, next_id_ = 1, tick_ = 0, evictions_ = 0;
  int64_t hits_ = 0, misses_ = 0;
  int running_ = 0, nworkers_ = 0, dev_ = 0;
  bool stop_ = false;
};

}  // namespace rfd
