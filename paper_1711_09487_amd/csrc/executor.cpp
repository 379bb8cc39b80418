// Concurrent execution of complete solves (see executor.hpp).
#include "executor.hpp"

#include <algorithm>
#include <cstring>

#include "rfd_capi_util.hpp"

namespace rfd {

Executor::Executor(int workers, int64_t budget) {
  if (workers <= 0) workers = 4;
  if (workers > 64) throw Error(ST_EINVAL, "at most 64 workers");
  RFD_HIP(hipGetDevice(&dev_));
  if (budget <= 0) {
    size_t fr = 0, tot = 0;
    RFD_HIP(hipMemGetInfo(&fr, &tot));
    budget = (int64_t)(0.9 * (double)fr);
  }
  budget_ = budget;
  nworkers_ = workers;
  for (int w = 0; w < workers; ++w) threads_.emplace_back([this, w] { loop(w); });
}

Executor::~Executor() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_work_.notify_all();
  for (auto& t : threads_) t.join();
}

int64_t Executor::submit(rfd_pencil_t pencil, const rfd_job& j) {
  if (!pencil) throw Error(ST_EINVAL, "null pencil");
  pencil_check(pencil);
  if (!(j.alpha < j.beta)) throw Error(ST_EINVAL, "need alpha < beta");
  if (j.n_c < 1 || j.m < 1 || j.steps < 1 || j.psi < 1 || j.nev_b < 0 || j.max_out < 0)
    throw Error(ST_EINVAL, "job needs n_c, m, steps, psi >= 1 and nev_b, max_out >= 0");
  if (!j.Y0 || (j.max_out > 0 && !j.evals)) throw Error(ST_EINVAL, "null Y0 or evals");
  Req r;
  r.pencil = pencil;
  r.job = j;
  r.bytes = pencil_estimate(pencil, j);
  r.t_sub = Clock::now();
  int64_t id;
  {
    std::lock_guard<std::mutex> g(mu_);
    if (stop_) throw Error(ST_ESTATE, "the executor is stopping");
    id = r.id = next_id_++;
    reqs_.emplace(id, r);
    queue_.push_back(id);
    busy_.emplace(pencil, false);
  }
  cv_work_.notify_all();
  return id;
}

int Executor::poll(int64_t id, bool wait, rfd_result* out) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = reqs_.find(id);
  if (it == reqs_.end()) throw Error(ST_EINVAL, "unknown request id");
  if (wait) cv_done_.wait(lk, [&] { return it->second.state == 2; });
  if (it->second.state != 2) return 0;
  if (out) *out = it->second.res;
  reqs_.erase(it);
  return 1;
}

void Executor::stats(int32_t* queued, int32_t* running, int64_t* bytes_running,
                     int64_t* bytes_cached, int64_t* evictions) {
  std::lock_guard<std::mutex> g(mu_);
  if (queued) *queued = (int32_t)queue_.size();
  if (running) *running = running_;
  if (bytes_running) *bytes_running = running_bytes_;
  if (bytes_cached) {
    int64_t c = 0;
    for (auto& kv : held_)
      if (!busy_[kv.first]) c += kv.second;
    *bytes_cached = c;
  }
  if (evictions) *evictions = evictions_;
}

void Executor::cache_stats(int64_t* hits, int64_t* misses) {
  std::lock_guard<std::mutex> g(mu_);
  if (hits) *hits = hits_;
  if (misses) *misses = misses_;
}

// Room for r next to the running jobs and the idle pencils' caches; idle
// caches are released (least recently used first) while that is short.
bool Executor::fits_locked(const Req& r) {
  auto cached = [&] {
    int64_t c = 0;
    for (auto& kv : held_)
      if (kv.first != r.pencil && !busy_[kv.first]) c += kv.second;
    return c;
  };
  while (running_bytes_ + r.bytes + cached() > budget_) {
    rfd_pencil_t victim = nullptr;
    int64_t best = 0;
    for (auto& kv : held_) {
      if (kv.first == r.pencil || busy_[kv.first] || kv.second <= 0) continue;
      if (!victim || lru_[kv.first] < best) {
        victim = kv.first;
        best = lru_[kv.first];
      }
    }
    if (!victim) break;
    pencil_release(victim);
    held_[victim] = pencil_held(victim);
    ++evictions_;
  }
  if (running_bytes_ + r.bytes + cached() <= budget_) return true;
  return running_ == 0;  // larger than the whole budget: runs alone
}

Executor::Req* Executor::pick_locked() {
  const int limit = 2 * nworkers_;
  std::vector<Req*> skipped;
  for (size_t qi = 0; qi < queue_.size(); ++qi) {
    Req* r = &reqs_[queue_[qi]];
    if (busy_[r->pencil]) continue;
    bool earlier = false;  // jobs on one pencil keep their submission order
    for (size_t q2 = 0; q2 < qi && !earlier; ++q2) earlier = reqs_[queue_[q2]].pencil == r->pencil;
    if (earlier) continue;
    if (!fits_locked(*r)) {
      if (r->bypassed >= limit) return nullptr;  // no more passing: wait for room
      skipped.push_back(r);
      continue;
    }
    for (Req* s : skipped) ++s->bypassed;
    queue_.erase(queue_.begin() + (std::ptrdiff_t)qi);
    return r;
  }
  return nullptr;
}

void Executor::loop(int w) {
  (void)hipSetDevice(dev_);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    st = nullptr;
  }
  DevBuf Q;  // this worker's interface basis
  std::unique_lock<std::mutex> lk(mu_);
  for (;;) {
    Req* r = nullptr;
    cv_work_.wait(lk, [&] { return (r = pick_locked()) != nullptr || (stop_ && queue_.empty()); });
    if (!r) break;
    if (held_[r->pencil] > 0)
      ++hits_;
    else
      ++misses_;
    r->state = 1;
    r->t_start = Clock::now();
    running_bytes_ += r->bytes;
    busy_[r->pencil] = true;
    ++running_;
    lk.unlock();
    run(*r, st, Q, w);
    const int64_t h = pencil_held(r->pencil);
    lk.lock();
    running_bytes_ -= r->bytes;
    busy_[r->pencil] = false;
    --running_;
    held_[r->pencil] = h;
    lru_[r->pencil] = ++tick_;
    r->state = 2;
    cv_done_.notify_all();
    cv_work_.notify_all();
  }
  lk.unlock();
  if (st) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
}

void Executor::run(Req& r, hipStream_t st, DevBuf& Q, int w) {
  rfd_result& out = r.res;
  std::memset(&out, 0, sizeof(out));
  out.worker = w;
  out.bytes = r.bytes;
  const rfd_job& j = r.job;
  rfd_pencil_t P = r.pencil;
  rfd_status s = RFD_OK;
  auto fail = [&](rfd_status code) {
    out.status = code;
    std::strncpy(out.message, rfd_last_error(), sizeof(out.message) - 1);
  };
  do {
    if ((s = rfd_set_interval_and_poles(P, j.alpha, j.beta, j.n_c, j.rule, nullptr, nullptr))) break;
    if ((s = rfd_set_precision(P, j.mode, j.refine_tol, j.max_sweeps))) break;
    int64_t n = 0, sz = 0;
    int32_t pp = 0;
    if ((s = rfd_pencil_info(P, &n, &pp, &sz, nullptr, nullptr))) break;
    const int64_t cols = std::max<int64_t>(1, std::min<int64_t>(sz, (int64_t)j.steps * j.m));
    const int code = capi_guard([&] { Q.alloc(sizeof(double) * (size_t)(sz * cols)); });
    if (code) {
      s = (rfd_status)code;
      break;
    }
    // the Q-independent interior caches run beside the filter
    if ((s = rfd_prepare_interior(P, j.sigma, j.nev_b))) break;
    int32_t mu = 0;
    if ((s = rfd_filter_interface(P, j.m, j.Y0, j.steps, Q.as<double>(), cols, &mu, st))) break;
    out.mu = mu;
    int64_t k = 0;
    if ((s = rfd_solve_interior(P, j.sigma, j.nev_b, j.psi, &k, st))) break;
    out.k = k;
    int32_t nf = 0;
    s = rfd_rayleigh_ritz(P, j.max_out, j.evals, j.evecs, j.resid, &nf, st);
    out.nfound = nf;
  } while (false);
  if (s == RFD_OK && hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    s = RFD_EDEVICE;
  }
  if (s) fail(s);
  const auto t_end = Clock::now();
  out.queued_s = std::chrono::duration<double>(r.t_start - r.t_sub).count();
  out.run_s = std::chrono::duration<double>(t_end - r.t_start).count();
}

}  // namespace rfd
