// The C ABI (include/rfd.h): argument checks, handle lifetime, and the map
// from C++ exceptions to rfd_status codes.
#include <cmath>
#include <cstring>
#include <memory>

#include "../../include/rfd.h"
#include "engine.hpp"
#include "pencil.hpp"
#include "dense.hpp"
#include "executor.hpp"
#include "rfd_capi_util.hpp"

namespace rfd {
std::string& last_error_slot() {
  static thread_local std::string msg;
  return msg;
}
}  // namespace rfd

using namespace rfd;

struct rfd_pencil_s {
  Csr A, M;
  std::unique_ptr<Partition> part;
  Poles poles;
  int mode = RFD_FP64;
  double tol = 1e-13;
  int sweeps = 8;
  bool timing = false;
  int window = 0;
  int interior_solver = RFD_INTERIOR_LU;
  std::unique_ptr<Engine> eng;
  DevBuf slice_q;  // interface basis of rfd_solve_slices
};

static rfd_pencil_s* need(rfd_pencil_t p) {
  if (!p) throw Error(ST_EINVAL, "null pencil handle");
  return p;
}

static Engine& need_engine(rfd_pencil_s* p) {
  if (!p->part || !p->eng) throw Error(ST_ESTATE, "rfd_set_partition has not been called");
  return *p->eng;
}

namespace rfd {
int64_t pencil_estimate(rfd_pencil_t p, const rfd_job& j) {
  Engine& E = need_engine(need(p));
  return E.estimate_bytes(j.mode, j.n_c, j.m, j.steps, j.nev_b, j.psi);
}
int64_t pencil_held(rfd_pencil_t p) { return p && p->eng ? p->eng->device_bytes() : 0; }
void pencil_release(rfd_pencil_t p) {
  if (p && p->eng) p->eng->reset_caches(true);
}
void pencil_check(rfd_pencil_t p) { (void)need_engine(need(p)); }
}  // namespace rfd

extern "C" {

rfd_status rfd_create_pencil(int64_t n, const int64_t* A_ptr, const int32_t* A_idx,
                             const double* A_val, const int64_t* M_ptr, const int32_t* M_idx,
                             const double* M_val, rfd_pencil_t* out) {
  return (rfd_status)capi_guard([&] {
    if (!out) throw Error(ST_EINVAL, "null output handle");
    *out = nullptr;
    auto p = std::make_unique<rfd_pencil_s>();
    p->A = make_csr(n, A_ptr, A_idx, A_val, "A");
    p->M = make_csr(n, M_ptr, M_idx, M_val, "M");
    check_symmetric(p->A, "A");
    check_symmetric(p->M, "M");
    for (int64_t i = 0; i < n; ++i) {
      double d = 0;
      for (int64_t e = p->M.ptr[i]; e < p->M.ptr[i + 1]; ++e)
        if (p->M.idx[e] == i) d += p->M.val[e];
      if (!(d > 0)) throw Error(ST_EINVAL, "M has a non-positive diagonal entry");
    }
    *out = p.release();
  });
}

rfd_status rfd_set_partition(rfd_pencil_t pencil, int32_t p, const int32_t* part) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    P->eng.reset();
    P->part.reset();
    auto pt = std::make_unique<Partition>(make_partition(P->A, P->M, p, part));
    P->eng = std::make_unique<Engine>(P->A, P->M, *pt);
    P->part = std::move(pt);
    P->eng->set_precision(P->mode, P->tol, P->sweeps);
    P->eng->set_timing(P->timing);
    P->eng->set_pole_window(P->window);
    if (P->interior_solver != RFD_INTERIOR_LU) P->eng->set_interior_solver(P->interior_solver);
    if (P->poles.set) P->eng->set_poles(P->poles);
  });
}

rfd_status rfd_set_interval_and_poles(rfd_pencil_t pencil, double alpha, double beta, int32_t n_c,
                                      int32_t rule, const double* zeta, const double* omega) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Poles q;
    make_poles(q, alpha, beta, n_c, rule, zeta, omega);
    P->poles = q;
    if (P->eng) P->eng->set_poles(P->poles);
  });
}

rfd_status rfd_set_precision(rfd_pencil_t pencil, int32_t mode, double refine_tol,
                             int32_t max_sweeps) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    if (mode != RFD_FP64 && mode != RFD_FP32_REFINE && mode != RFD_FP32_AUTO)
      throw Error(ST_EINVAL, "unknown precision mode");
    P->mode = mode;
    P->tol = refine_tol > 0 ? refine_tol : 1e-13;
    P->sweeps = max_sweeps > 0 ? max_sweeps : 8;
    if (P->eng) P->eng->set_precision(P->mode, P->tol, P->sweeps);
  });
}

rfd_status rfd_filter_interface(rfd_pencil_t pencil, int32_t m, const double* Y0, int32_t steps,
                                double* Q, int64_t ldq_cols, int32_t* mu, rfd_stream_t stream) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    if (!P->poles.set) throw Error(ST_ESTATE, "rfd_set_interval_and_poles has not been called");
    const int64_t s = (int64_t)P->part->iface.size();
    if (m < 1 || m > s) throw Error(ST_EINVAL, "need 1 <= m <= s");
    if (steps < 1) throw Error(ST_EINVAL, "need steps >= 1");
    if (!Y0 || !Q || !mu) throw Error(ST_EINVAL, "null pointer argument");
    if (ldq_cols < std::min<int64_t>(s, (int64_t)steps * m))
      throw Error(ST_EINVAL, "Q has too few columns");
    int mu_i = 0;
    E.filter_interface((hipStream_t)stream, m, Y0, steps, Q, ldq_cols, &mu_i);
    *mu = mu_i;
  });
}

rfd_status rfd_filter_apply(rfd_pencil_t pencil, int32_t m, const double* Y, double* W,
                            rfd_stream_t stream) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    if (!P->poles.set) throw Error(ST_ESTATE, "rfd_set_interval_and_poles has not been called");
    if (m < 1) throw Error(ST_EINVAL, "need m >= 1");
    if (!Y || !W || Y == W) throw Error(ST_EINVAL, "null or aliased pointer argument");
    E.filter_apply((hipStream_t)stream, m, Y, W);
  });
}

rfd_status rfd_filter_lanczos(rfd_pencil_t pencil, int32_t m, const double* Y0, double tol,
                              int32_t max_steps, int32_t test_every, double* Q, int64_t ldq_cols,
                              int32_t* mu, int32_t* steps, double* traces, int32_t* converged,
                              rfd_stream_t stream) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    if (!P->poles.set) throw Error(ST_ESTATE, "rfd_set_interval_and_poles has not been called");
    const int64_t s = (int64_t)P->part->iface.size();
    if (m < 1 || m > s) throw Error(ST_EINVAL, "need 1 <= m <= s");
    if (max_steps < 1) throw Error(ST_EINVAL, "need max_steps >= 1");
    if (!(tol >= 0.0)) throw Error(ST_EINVAL, "need tol >= 0");
    if (!Y0 || !Q || !mu || !steps || !converged) throw Error(ST_EINVAL, "null pointer argument");
    if (ldq_cols < std::min<int64_t>(s, (int64_t)m)) throw Error(ST_EINVAL, "Q has too few columns");
    int mu_i = 0, st_i = 0, cv = 0;
    E.filter_lanczos((hipStream_t)stream, m, Y0, tol, max_steps, test_every > 0 ? test_every : 10,
                     Q, ldq_cols, &mu_i, &st_i, traces, &cv);
    *mu = mu_i;
    *steps = st_i;
    *converged = cv;
  });
}

rfd_status rfd_prepare_interior(rfd_pencil_t pencil, double sigma, int32_t nev_b) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    if (nev_b < 0) throw Error(ST_EINVAL, "need nev_b >= 0");
    if (!std::isfinite(sigma)) throw Error(ST_EINVAL, "sigma is not finite");
    E.prepare_interior(sigma, nev_b);
  });
}

rfd_status rfd_solve_interior(rfd_pencil_t pencil, double sigma, int32_t nev_b, int32_t psi,
                              int64_t* k_out, rfd_stream_t stream) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    if (nev_b < 0) throw Error(ST_EINVAL, "need nev_b >= 0");
    if (psi < 1) throw Error(ST_EINVAL, "need psi >= 1");
    if (!std::isfinite(sigma)) throw Error(ST_EINVAL, "sigma is not finite");
    int64_t k = 0;
    E.solve_interior((hipStream_t)stream, sigma, nev_b, psi, &k);
    if (k_out) *k_out = k;
  });
}

rfd_status rfd_rayleigh_ritz(rfd_pencil_t pencil, int32_t max_out, double* evals, double* evecs,
                             double* resid, int32_t* nfound, rfd_stream_t stream) {
  int found = 0;
  rfd_status st = (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    if (max_out < 0) throw Error(ST_EINVAL, "need max_out >= 0");
    if (!nfound) throw Error(ST_EINVAL, "null nfound");
    if (max_out > 0 && !evals) throw Error(ST_EINVAL, "null evals");
    E.rayleigh_ritz((hipStream_t)stream, max_out, evals, evecs, resid, &found);
    *nfound = found;
    if (found > max_out)
      throw Error(ST_EINVAL, "more Ritz values in [alpha, beta] than max_out");
  });
  return st;
}

rfd_status rfd_inertia_count(rfd_pencil_t pencil, double alpha, double beta, int64_t* count,
                             rfd_stream_t stream) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    if (!count) throw Error(ST_EINVAL, "null count");
    if (!(alpha < beta) || !std::isfinite(alpha) || !std::isfinite(beta))
      throw Error(ST_EINVAL, "need finite alpha < beta");
    const hipStream_t st = (hipStream_t)stream;
    const int64_t lo = E.inertia(st, alpha);
    const int64_t hi = E.inertia(st, beta);
    *count = hi - lo;
  });
}

rfd_status rfd_solve_slices(rfd_pencil_t pencil, int32_t nslices, const double* cuts, int32_t n_c,
                            int32_t rule, int32_t m, const double* Y0, int32_t steps, double sigma,
                            int32_t nev_b, int32_t psi, int32_t max_out, double* evals,
                            double* evecs, double* resid, int32_t* nfound, int32_t* counts,
                            int64_t* inertia, rfd_stream_t stream) {
  int total = 0;
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    const int64_t s = (int64_t)P->part->iface.size(), n = P->A.n;
    if (nslices < 1 || !cuts) throw Error(ST_EINVAL, "need nslices >= 1 and the cuts");
    for (int i = 0; i < nslices; ++i)
      if (!(cuts[i] < cuts[i + 1]) || !std::isfinite(cuts[i]) || !std::isfinite(cuts[i + 1]))
        throw Error(ST_EINVAL, "cuts must be finite and strictly increasing");
    if (m < 1 || m > s || steps < 1 || nev_b < 0 || psi < 1 || max_out < 0)
      throw Error(ST_EINVAL, "bad m, steps, nev_b, psi or max_out");
    if (!Y0 || !nfound || (max_out > 0 && !evals)) throw Error(ST_EINVAL, "null pointer argument");
    const hipStream_t st = (hipStream_t)stream;
    const int64_t cols = std::min<int64_t>(s, (int64_t)steps * m);
    P->slice_q.alloc(sizeof(double) * s * cols);
    bool overflow = false;
    for (int i = 0; i < nslices; ++i) {
      Poles q;
      make_poles(q, cuts[i], cuts[i + 1], n_c, rule, nullptr, nullptr);
      P->poles = q;
      E.set_poles(q);
      int mu = 0;
      E.filter_interface(st, m, Y0, steps, P->slice_q.as<double>(), cols, &mu);
      const double sig = std::isnan(sigma) ? 0.5 * (cuts[i] + cuts[i + 1]) : sigma;
      int64_t k = 0;
      E.solve_interior(st, sig, nev_b, psi, &k);
      const int room = std::max(0, max_out - total);
      int nf = 0;
      E.rayleigh_ritz(st, room, room > 0 ? evals + total : nullptr,
                      (evecs && room > 0) ? evecs + (int64_t)total * n : nullptr,
                      (resid && room > 0) ? resid + total : nullptr, &nf);
      if (counts) counts[i] = nf;
      if (nf > room) overflow = true;
      total += nf;
    }
    *nfound = total;
    if (inertia) {
      const int64_t lo = E.inertia(st, cuts[0]);
      const int64_t hi = E.inertia(st, cuts[nslices]);
      *inertia = hi - lo;
    }
    if (overflow) throw Error(ST_EINVAL, "more Ritz values in the slices than max_out");
  });
}

rfd_status rfd_reset_caches(rfd_pencil_t pencil, int32_t release) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    if (P->eng) P->eng->reset_caches(release != 0);
  });
}

rfd_status rfd_destroy_pencil(rfd_pencil_t pencil) {
  return (rfd_status)capi_guard([&] { delete pencil; });
}

const char* rfd_last_error(void) { return last_error_slot().c_str(); }

rfd_status rfd_pencil_info(rfd_pencil_t pencil, int64_t* n, int32_t* p, int64_t* s,
                           int64_t* d_max, int64_t* device_bytes) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    if (n) *n = P->A.n;
    if (p) *p = P->part ? P->part->p : 0;
    if (s) *s = P->part ? (int64_t)P->part->iface.size() : 0;
    if (d_max) *d_max = P->part ? P->part->d_max : 0;
    if (device_bytes) *device_bytes = P->eng ? P->eng->device_bytes() : 0;
  });
}

rfd_status rfd_set_timing(rfd_pencil_t pencil, int32_t on) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    P->timing = on != 0;
    if (P->eng) P->eng->set_timing(P->timing);
  });
}

rfd_status rfd_set_pole_window(rfd_pencil_t pencil, int32_t max_poles) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    if (max_poles < 0) throw Error(ST_EINVAL, "need max_poles >= 0");
    P->window = max_poles;
    if (P->eng) P->eng->set_pole_window(max_poles);
  });
}

rfd_status rfd_set_interior_solver(rfd_pencil_t pencil, int32_t kind) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    E.set_interior_solver(kind);
    P->interior_solver = kind;
  });
}

int rfd_test_spectral_orthogonality(void* pencil, double* dev) {
  return capi_guard([&] {
    auto* P = need(static_cast<rfd_pencil_t>(pencil));
    if (!dev) throw Error(ST_EINVAL, "null output");
    *dev = need_engine(P).spectral_orthogonality();
  });
}

rfd_status rfd_set_interface_groups(rfd_pencil_t pencil, int32_t ngroups, const int32_t* group) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    Engine& E = need_engine(P);
    if (ngroups < 0) throw Error(ST_EINVAL, "need ngroups >= 0");
    if (ngroups > 0 && !group) throw Error(ST_EINVAL, "null group array");
    E.set_interface_groups(ngroups, group);
  });
}

rfd_status rfd_phase_times(rfd_pencil_t pencil, double* ms16) {
  return (rfd_status)capi_guard([&] {
    auto* P = need(pencil);
    if (!ms16) throw Error(ST_EINVAL, "null output");
    for (int i = 0; i < 16; ++i) ms16[i] = 0;
    if (P->eng) P->eng->phase_times(ms16);
  });
}

rfd_status rfd_set_gemm_tuning(const int32_t* entries, int32_t count) {
  return (rfd_status)capi_guard([&] { set_gemm_tuning(entries, count); });
}

rfd_status rfd_device_arch(char* buf, int32_t len) {
  return (rfd_status)capi_guard([&] {
    if (!buf || len < 2) throw Error(ST_EINVAL, "need a buffer of at least 2 bytes");
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(ST_EDEVICE, "no HIP device");
    }
    std::string a(prop.gcnArchName);
    a = a.substr(0, a.find(':'));
    std::strncpy(buf, a.c_str(), (size_t)len - 1);
    buf[len - 1] = 0;
  });
}

rfd_status rfd_kernel_accounting(int32_t every) {
  return (rfd_status)capi_guard([&] {
    if (every < 0) throw Error(ST_EINVAL, "need every >= 0");
    KernelAccount& k = KernelAccount::get();
    std::lock_guard<std::mutex> g(k.mu);
    k.every = every;
  });
}

rfd_status rfd_kernel_stats(double* launches, double* sampled, double* ms, double* flops,
                            double* bytes) {
  return (rfd_status)capi_guard([&] {
    if (!launches || !sampled || !ms || !flops || !bytes) throw Error(ST_EINVAL, "null output");
    KernelAccount::get().collect(launches, sampled, ms, flops, bytes, KA_KEYS);
  });
}

// ---------------------------------------------------------------------------
// Batching and serving (executor.cpp)
// ---------------------------------------------------------------------------
struct rfd_server_s {
  std::unique_ptr<Executor> ex;
};

rfd_status rfd_batch_run(int32_t nb, const rfd_pencil_t* pencils, const rfd_job* jobs,
                         rfd_result* results, int32_t workers, int64_t hbm_budget) {
  rfd_status first = RFD_OK;
  rfd_status st = (rfd_status)capi_guard([&] {
    if (nb < 1 || !pencils || !jobs || !results) throw Error(ST_EINVAL, "need nb >= 1 and arrays");
    for (int32_t i = 0; i < nb; ++i) {
      if (!pencils[i]) throw Error(ST_EINVAL, "null pencil in the batch");
      pencil_check(pencils[i]);
    }
    Executor ex(workers, hbm_budget);
    std::vector<int64_t> ids((size_t)nb);
    for (int32_t i = 0; i < nb; ++i) ids[i] = ex.submit(pencils[i], jobs[i]);
    for (int32_t i = 0; i < nb; ++i) {
      ex.poll(ids[i], true, &results[i]);
      if (results[i].status != RFD_OK && first == RFD_OK) first = (rfd_status)results[i].status;
    }
  });
  if (st != RFD_OK) return st;
  if (first != RFD_OK) last_error_slot() = "a job of the batch failed (see its result)";
  return first;
}

rfd_status rfd_server_create(int32_t workers, int64_t hbm_budget, rfd_server_t* out) {
  return (rfd_status)capi_guard([&] {
    if (!out) throw Error(ST_EINVAL, "null output handle");
    *out = nullptr;
    auto s = std::make_unique<rfd_server_s>();
    s->ex = std::make_unique<Executor>(workers, hbm_budget);
    *out = s.release();
  });
}

rfd_status rfd_server_submit(rfd_server_t server, rfd_pencil_t pencil, const rfd_job* job,
                             int64_t* request_id) {
  return (rfd_status)capi_guard([&] {
    if (!server || !job || !request_id) throw Error(ST_EINVAL, "null argument");
    *request_id = server->ex->submit(pencil, *job);
  });
}

rfd_status rfd_server_poll(rfd_server_t server, int64_t request_id, int32_t wait,
                           rfd_result* out) {
  int done = 0;
  rfd_status st = (rfd_status)capi_guard([&] {
    if (!server) throw Error(ST_EINVAL, "null server");
    done = server->ex->poll(request_id, wait != 0, out);
  });
  if (st != RFD_OK) return st;
  return done ? RFD_OK : RFD_EPENDING;
}

rfd_status rfd_server_destroy(rfd_server_t server) {
  return (rfd_status)capi_guard([&] { delete server; });
}

rfd_status rfd_server_stats(rfd_server_t server, int32_t* queued, int32_t* running,
                            int64_t* bytes_running, int64_t* bytes_cached, int64_t* evictions) {
  return (rfd_status)capi_guard([&] {
    if (!server) throw Error(ST_EINVAL, "null server");
    server->ex->stats(queued, running, bytes_running, bytes_cached, evictions);
  });
}

rfd_status rfd_server_cache_stats(rfd_server_t server, int64_t* hits, int64_t* misses) {
  return (rfd_status)capi_guard([&] {
    if (!server) throw Error(ST_EINVAL, "null server");
    server->ex->cache_stats(hits, misses);
  });
}

int rfd_test_basis(void* pencil, double* dst, int64_t cap, int64_t* k_out, void* stream) {
  return capi_guard([&] {
    auto* P = need((rfd_pencil_t)pencil);
    Engine& E = need_engine(P);
    E.copy_basis((hipStream_t)stream, dst, cap, k_out);
  });
}

}  // extern "C"
