// Device-side execution of the RF-DDES path for one pencil (engine.hpp):
//   factor():            B_j(zeta_l) LU, Schur contributions with FP64 refinement,
//                        S(zeta_l) assembly and LU                      (Sec. 3.1)
//   apply_filter():      W = 2 Re sum_l omega_l S(zeta_l)^{-1} Y          (eq. (3.5))
//   filter_interface():  block Krylov basis with rank-revealing QR       (Alg. 3.1)
//   solve_interior(), rayleigh_ritz(): interior.hip
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dense.hpp"
#include "engine_impl.hpp"
#include "orth.hpp"
#include "sparse.hpp"

namespace rfd {

// Z = X_re + X_im (rows x cols per item).
__global__ void k_plane_sum(DMat<double> X, DMat<double> Z, int64_t rows, int64_t cols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e % rows, j = e / rows;
  const DMat<double> x = X.item(blockIdx.y), z = Z.item(blockIdx.y);
  z.re[i + j * z.ld] = x.re[i + j * x.ld] + x.im[i + j * x.ld];
}

// The rest of R -= S X in Gauss's form, with P1 = S_re X_re, P2 = S_im X_im
// and R_im already holding Y_im - (S_re + S_im)(X_re + X_im):
// R_re += P2 - P1, R_im += P1 + P2.
__global__ void k_gauss_combine(DMat<double> Rm, DMat<double> P1, DMat<double> P2, int64_t rows,
                                int64_t cols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e % rows, j = e / rows;
  const DMat<double> r = Rm.item(blockIdx.y), a = P1.item(blockIdx.y), c = P2.item(blockIdx.y);
  const double p1 = a.re[i + j * a.ld], p2 = c.re[i + j * c.ld];
  r.re[i + j * r.ld] += p2 - p1;
  r.im[i + j * r.ld] += p1 + p2;
}

template <typename T>
static void upload(DevBuf& b, const std::vector<T>& v) {
  b.alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (!v.empty()) RFD_HIP(hipMemcpy(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
}

static void upload_pair(DevPairGroup& g, const std::vector<const PairCsr*>& blocks) {
  std::vector<int64_t> roff(1, 0), ptr;
  std::vector<int32_t> idx;
  std::vector<double> a, m;
  for (const PairCsr* B : blocks) {
    const int64_t base = (int64_t)idx.size();
    for (int64_t r = 0; r <= B->rows; ++r) ptr.push_back(base + B->ptr[r]);
    roff.push_back((int64_t)ptr.size());
    idx.insert(idx.end(), B->idx.begin(), B->idx.end());
    a.insert(a.end(), B->a.begin(), B->a.end());
    m.insert(m.end(), B->m.begin(), B->m.end());
  }
  upload(g.roff, roff);
  upload(g.ptr, ptr);
  upload(g.idx, idx);
  upload(g.a, a);
  upload(g.m, m);
}

DevPairCsr DevPairGroup::view() const {
  DevPairCsr v;
  v.roff = roff.as<int64_t>();
  v.ptr = ptr.as<int64_t>();
  v.idx = idx.as<int32_t>();
  v.a = a.as<double>();
  v.m = m.as<double>();
  return v;
}

// ---------------------------------------------------------------------------
Engine::Engine(const Csr& A, const Csr& M, const Partition& P) : d_(new EngineImpl) {
  EngineImpl& e = *d_;
  RFD_HIP(hipGetDevice(&e.device));
  e.A = &A;
  e.M = &M;
  e.P = &P;
  e.n = A.n;
  e.p = P.p;
  e.s = (int64_t)P.iface.size();
  e.SP = round_up(e.s, NB);
  e.D = round_up(P.d_max, NB);
  e.SJ = round_up(std::max<int64_t>(P.sj_max, 1), NB);
  e.normA = abs_row_sum_max(A);
  std::vector<const PairCsr*> bl, el, etl;
  std::vector<int32_t> dj, sj, adj((size_t)e.p * e.SJ, 0);
  for (int j = 0; j < e.p; ++j) {
    bl.push_back(&P.Bloc[j]);
    el.push_back(&P.Eloc[j]);
    etl.push_back(&P.EtLoc[j]);
    dj.push_back((int32_t)P.interior[j].size());
    sj.push_back((int32_t)P.adj[j].size());
    for (size_t a = 0; a < P.adj[j].size(); ++a) adj[(size_t)j * e.SJ + a] = P.adj[j][a];
  }
  upload_pair(e.Bg, bl);
  upload_pair(e.Eg, el);
  upload_pair(e.Etg, etl);
  {
    // the blocks renumbered for the Schur solves on trailing blocks
    const SchurRenumber R = make_schur_renumber(P, e.D, NB);
    e.TS = R.TS;
    e.SJA = R.SJ;
    std::vector<const PairCsr*> b2p, e2p, et2p;
    for (int j = 0; j < e.p; ++j) {
      b2p.push_back(&R.B[j]);
      e2p.push_back(&R.E[j]);
      et2p.push_back(&R.Et[j]);
    }
    upload_pair(e.Bg2, b2p);
    upload_pair(e.Eg2, e2p);
    upload_pair(e.Etg2, et2p);
    upload(e.dj2, std::vector<int32_t>((size_t)e.p, (int32_t)e.D));
  }
  upload_pair(e.Cg, {&P.Cloc});
  upload(e.dj, dj);
  upload(e.sj, sj);
  upload(e.adj, adj);
  e.colors_d.resize(P.colors.size());
  for (size_t c = 0; c < P.colors.size(); ++c) upload(e.colors_d[c], P.colors[c]);
  // global CSR of A and M and the reordering (interiors, then interface)
  upload(e.Aptr, A.ptr);
  upload(e.Aidx, A.idx);
  upload(e.Aval, A.val);
  upload(e.Mptr, M.ptr);
  upload(e.Midx, M.idx);
  upload(e.Mval, M.val);
  std::vector<int32_t> order, ioff(1, 0);
  for (int j = 0; j < e.p; ++j) {
    order.insert(order.end(), P.interior[j].begin(), P.interior[j].end());
    ioff.push_back((int32_t)order.size());
  }
  order.insert(order.end(), P.iface.begin(), P.iface.end());
  upload(e.order, order);
  upload(e.ioff, ioff);
  e.emax = 0;
  for (int j = 0; j < e.p; ++j)
    for (size_t k = 0; k < P.Eloc[j].a.size(); ++k)
      e.emax = std::max(e.emax, std::fabs(P.Eloc[j].a[k]) + std::fabs(P.Eloc[j].m[k]));
  e.flags.alloc(sizeof(unsigned) * 4);
  e.scal.alloc(sizeof(double) * 8);
  RFD_HIP(hipMemset(e.flags.p, 0, sizeof(unsigned) * 4));
}

Engine::~Engine() {
  EngineImpl& e = *d_;
  try {
    e.join_prepare();
  } catch (...) {
  }
  if (e.h_stream) (void)hipStreamSynchronize(e.h_stream);
  for (hipStream_t ps : {e.prep_stream, e.prep_stream2, e.h_stream})
    if (ps) {
      release_stream_resources(ps);
      (void)hipStreamDestroy(ps);
    }
  for (hipEvent_t ev : {e.h_lvl, e.h_done})
    if (ev) (void)hipEventDestroy(ev);
}

void Engine::set_poles(const Poles& poles) {
  d_->join_prepare();
  EngineImpl& e = *d_;
  e.poles = poles;
  std::vector<double> z, w;
  for (int l = 0; l < poles.n_c; ++l) {
    z.push_back(poles.zeta[l].real());
    z.push_back(poles.zeta[l].imag());
    w.push_back(poles.omega[l].real());
    w.push_back(poles.omega[l].imag());
  }
  upload(e.zeta, z);
  upload(e.omega, w);
  e.factored = false;
}

void Engine::set_precision(int mode, double tol, int sweeps) {
  d_->join_prepare();
  EngineImpl& e = *d_;
  if (mode != e.mode) e.factored = false;
  e.mode = mode;
  e.tol = tol;
  e.sweeps = sweeps;
}

int64_t Engine::estimate_bytes(int mode, int n_c, int m, int steps, int nev_b, int psi) const {
  const EngineImpl& e = *d_;
  const bool b32 = e.b_fp32(mode);                                              // interior
  const bool f32 = e.s_precision(mode, std::min<int64_t>(e.s, (int64_t)steps * m)) == 1;  // S
  const int64_t es = f32 ? 4 : 8, D = e.D, SP = e.SP, SJ = e.SJ, p = e.p, n = e.n;
  const int64_t bs = b32 ? 4 : 8;
  const int64_t per_pole = p * (D * D * 2 * bs + (int64_t)NB * 2 * D * 2 * bs +
                                D * SJ * (b32 ? 16 + 16 + 8 + 8 : 16));
  const int64_t chunk = std::min<int64_t>(n_c, std::max<int64_t>(1, (int64_t(96) << 30) / per_pole));
  const int64_t MP = round_up(std::max(m, 1), NB);
  const int64_t mu = std::min<int64_t>(e.s, (int64_t)steps * m);
  const int64_t MUP = round_up(std::max<int64_t>(mu, 1), NB);
  const int64_t VB = nev_b + 16;
  const int64_t k = p * VB + (int64_t)psi * mu;
  int64_t b = chunk * per_pole;                                   // shifted blocks, Schur solves
  if (e.tree.L > 0) {
    b += n_c * e.tree_pole_bytes(MP, f32 ? 1 : 0);                 // two-level S, right-hand sides
  } else {
    b += SP * SP * n_c * 16 + (f32 ? SP * SP * n_c * 8 : 0);      // S (FP64, FP32 copy)
    if (f32 && SP * SP * n_c * 8 <= EngineImpl::GAUSS_MAX_BYTES)
      b += SP * SP * n_c * 8 + SP * round_up(std::max(m, 1), NB) * n_c * 24;  // S_re + S_im, P1 P2 X sum
    b += (int64_t)NB * 2 * SP * n_c * 2 * es;                     // S block inverses
    b += SP * MP * n_c * (f32 ? 16 + 16 + 8 : 16);                // filter right-hand sides
  }
  b += e.s * (mu + m) * 8 * 3;                                    // interface basis, orth work
  b += p * (D * VB + 3 * D * D + D * (int64_t)psi * MUP) * 8;     // V_j, B_sigma, levels
  b += p * (2 * 256 * D + 256 * MUP) * 8;                          // B_sigma wide leaves, their work
  b += n * (k * 3 + 4 * mu) * 8 + k * k * 8 * 2;                  // Z, A Z, H, level work
  if (e.interior_solver == 1)                                      // eigenvectors, work, F, F_zeta
    b += p * (2 * D * D + D * SJ * (1 + 2 * chunk) + D * MUP) * 8;
  return b + b / 10 + (int64_t(64) << 20);
}

int64_t Engine::device_bytes() const {
  d_->join_prepare();
  return d_->bytes_held();
}

void Engine::reset_caches(bool release) {
  d_->join_prepare();
  EngineImpl& e = *d_;
  e.factored = false;
  e.vcache_valid = false;
  e.bs_valid = false;
  e.interior_ready = false;
  // the projected matrix may still be assembling on the helper stream
  if (e.h_stream) RFD_HIP(hipStreamSynchronize(e.h_stream));
  e.h_ready = false;
  if (!release) return;
  e.spec_valid = e.spec_f_valid = false;
  e.spec_orth = 0;
  for (DevBuf* b : e.solve_buffers()) b->release();
  e.tw_v.cap = e.tw_h.cap = 0;
  e.ow.v_elems = 0;
  e.ow.m_cap = e.ow.mu_cap = 0;
  e.kz = 0;
}

void Engine::set_timing(bool on) {
  d_->join_prepare();
  d_->timer.enabled = on;
}

void Engine::set_pole_window(int w) {
  d_->join_prepare();
  if (d_->max_window != w) d_->factored = false;
  d_->max_window = w;
}

int Engine::set_interior_solver(int kind) {
  d_->join_prepare();
  EngineImpl& e = *d_;
  if (kind != 0 && kind != 1) throw Error(ST_EINVAL, "interior solver kind must be 0 or 1");
  const int prev = e.interior_solver;
  if (kind != prev) {
    e.factored = false;
    e.vcache_valid = false;
    e.bs_valid = false;
    e.interior_ready = false;
  }
  e.interior_solver = kind;
  return prev;
}

double Engine::spectral_orthogonality() const {
  d_->join_prepare();
  return d_->spec_orth;
}
void Engine::phase_times(double* ms16) {
  d_->join_prepare();
  d_->timer.collect(ms16);
}

// ---------------------------------------------------------------------------
void PhaseTimer::begin(hipStream_t s, int phase) {
  if (!enabled) return;
  Rec r;
  r.phase = phase;
  r.s = s;
  RFD_HIP(hipEventCreate(&r.a));
  RFD_HIP(hipEventCreate(&r.b));
  RFD_HIP(hipEventRecord(r.a, s));
  std::lock_guard<std::mutex> g(mu);
  open.push_back(r);
}
// closes the innermost open phase of stream s
void PhaseTimer::end(hipStream_t s) {
  if (!enabled) return;
  Rec r;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = open.rbegin();
    while (it != open.rend() && it->s != s) ++it;
    if (it == open.rend()) return;
    r = *it;
    open.erase(std::next(it).base());
  }
  RFD_HIP(hipEventRecord(r.b, s));
  std::lock_guard<std::mutex> g(mu);
  done.push_back(r);
}
void PhaseTimer::collect(double* ms16) {
  std::lock_guard<std::mutex> g(mu);
  for (auto& r : done) {
    RFD_HIP(hipEventSynchronize(r.b));
    float ms = 0;
    RFD_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    acc[r.phase] += ms;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  done.clear();
  for (int i = 0; i < 16; ++i) ms16[i] = acc[i];
  for (int i = 0; i < 16; ++i) acc[i] = 0;
  ms16[12] = sweeps_schur;
  ms16[13] = sweeps_filter;
}
PhaseTimer::~PhaseTimer() {
  for (auto& r : done) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto& r : open) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
}

std::vector<DevBuf*> EngineImpl::solve_buffers() {
  std::vector<DevBuf*> v{&K32, &K64, &Kinv32, &Kinv64, &X32, &X64, &R32, &R64, &S64, &S32,
                         &Ssum, &Xsum, &Pg,
                         &Sinv32, &Sinv64, &Swide, &Swork, &Yc, &Xf, &Rf, &Rf32, &W, &Qint, &Vb, &Bs, &Bsinv,
                         &Bspiv, &Bswide, &Bswork, &Lev, &Zt, &work1, &work2, &work3, &work4, &work5, &work6,
                         &ipiv_small, &iscal, &gwork, &work6b, &rr_az, &rr_h, &ow.V, &ow.T,
                         &ow.cn, &ow.used, &ow.piv, &ow.tau, &ow.scal, &ow.rank, &ow.wg, &ow.wt,
                         &ow.w1, &ow.w2, &Tgg64, &TgT64, &Ttt64, &Txc64, &Tgg32, &TgT32,
                         &Txc32, &Ttt32, &Tinvg, &Tinvt, &Twide, &Twork, &Tgt, &TRG, &TRT, &TXG,
                         &TXT, &TRG32, &TRT32, &TU, &TXTg, &Vs, &lam_s, &Fs, &Fz, &Ts, &Gsp,
                         &Mlu, &Mluinv, &mflag};
  for (TriWork* t : {&tw_v, &tw_h})
    for (DevBuf* b : {&t->d, &t->e, &t->tau, &t->pt, &t->acol, &t->vw, &t->red, &t->sq, &t->ptvp,
                      &t->wv, &t->wg, &t->wt, &t->w1, &t->w2})
      v.push_back(b);
  for (DevBuf& b : tmp) v.push_back(&b);
  return v;
}

// Buffers an interior preparation writes (see prepare_interior).
std::vector<DevBuf*> EngineImpl::prep_buffers() {
  std::vector<DevBuf*> v{&Vb, &work1, &work2, &work3, &kap_d, &Bs, &Bsinv, &Bspiv, &Bswide,
                         &Bswork, &prep_flags, &Mlu, &Mluinv, &mflag};
  for (DevBuf* b : {&tw_v.d, &tw_v.e, &tw_v.tau, &tw_v.pt, &tw_v.acol, &tw_v.vw, &tw_v.red,
                    &tw_v.sq, &tw_v.ptvp, &tw_v.wv, &tw_v.wg, &tw_v.wt, &tw_v.w1, &tw_v.w2})
    v.push_back(b);
  for (int i = 0; i <= 6; ++i) v.push_back(&tmp[i]);
  return v;
}

int64_t EngineImpl::bytes_held() const {
  EngineImpl* e = const_cast<EngineImpl*>(this);
  // while a preparation runs, its buffers change size under it: they are
  // left out (the estimate of what this pencil holds only gets smaller)
  std::vector<DevBuf*> skip;
  if (prep_running.load()) skip = e->prep_buffers();
  int64_t t = 0;
  for (DevBuf* b : e->solve_buffers())
    if (std::find(skip.begin(), skip.end(), b) == skip.end()) t += (int64_t)b->bytes;
  return t;
}

void EngineImpl::join_prepare() {
  if (prep.joinable()) prep.join();
  prep_running.store(false);
  if (prep_err) {
    std::exception_ptr e = prep_err;
    prep_err = nullptr;
    std::rethrow_exception(e);
  }
}

void Engine::prepare_interior(double sig, int nevb) {
  EngineImpl& e = *d_;
  e.join_prepare();
  // the spectral path's interior caches are a column window of the pencil's
  // eigendecomposition, which the filter's factorization makes first
  if (e.interior_solver == 1) return;
  if (e.vcache_valid && e.vcache_sigma == sig && e.vcache_nevb == nevb && e.bs_valid &&
      e.bs_sigma == sig)
    return;
  if (!e.prep_stream) RFD_HIP(hipStreamCreateWithFlags(&e.prep_stream, hipStreamNonBlocking));
  if (!e.prep_stream2) RFD_HIP(hipStreamCreateWithFlags(&e.prep_stream2, hipStreamNonBlocking));
  if (!e.prep_flags.p) {
    e.prep_flags.alloc(sizeof(unsigned));
    RFD_HIP(hipMemsetAsync(e.prep_flags.p, 0, sizeof(unsigned), e.prep_stream));
  }
  e.prep_running.store(true);
  e.prep = std::thread([&e, sig, nevb]() {
    try {
      RFD_HIP(hipSetDevice(e.device));
      // B_sigma's factorization (no host round trip until its flag check) is
      // enqueued on a second stream first, so that it runs beside the
      // subdomain eigensolver, whose steps wait on the host
      e.factor_bsigma(e.prep_stream2, sig, &e.prep_flags, false);
      e.interior_basis(e.prep_stream, sig, nevb);
      e.check_flags(e.prep_stream2, "B_sigma factorization", &e.prep_flags);
      RFD_HIP(hipStreamSynchronize(e.prep_stream));
    } catch (...) {
      // nothing half-made is kept
      e.vcache_valid = false;
      e.bs_valid = false;
      e.prep_err = std::current_exception();
    }
  });
}

double EngineImpl::read_scalar(hipStream_t s, int i) {
  double v = 0;
  RFD_HIP(hipMemcpyAsync(&v, scal.as<double>() + i, sizeof(double), hipMemcpyDeviceToHost, s));
  RFD_HIP(hipStreamSynchronize(s));
  return v;
}

void EngineImpl::zero_scalar(hipStream_t s, int i) {
  RFD_HIP(hipMemsetAsync(scal.as<double>() + i, 0, sizeof(double), s));
}

void EngineImpl::check_flags(hipStream_t s, const char* what, DevBuf* fb) {
  DevBuf& fw = fb ? *fb : flags;
  unsigned f = 0;
  RFD_HIP(hipMemcpyAsync(&f, fw.as<unsigned>(), sizeof(unsigned), hipMemcpyDeviceToHost, s));
  RFD_HIP(hipStreamSynchronize(s));
  if (f) {
    RFD_HIP(hipMemsetAsync(fw.p, 0, sizeof(unsigned), s));
    throw Error(ST_EBREAKDOWN, std::string(what) + ": pivot below the breakdown threshold" +
                                   ((f & 2) ? " (non-finite value)" : ""));
  }
}

// Precision of S's factors (see rfd_set_precision): FP32 pays when the LU
// work it saves, (4/3) sum N^3 FP64-equivalent flops over the factored
// blocks, exceeds what the refinement adds to c filtered columns, about
// 16 sum N^2 per column (two FP64 residuals and two FP32 solves against one
// FP64 solve).
int EngineImpl::s_precision(int md, int64_t c) const {
  if (md != 2) return md == 1 ? 1 : 0;
  double n3 = 0.0, n2 = 0.0;
  auto add = [&](double N, double count) {
    n3 += count * N * N * N;
    n2 += count * N * N;
  };
  if (tree.L > 0) {
    add((double)tree.NGP, (double)tree.L);
    add((double)tree.TP, 1.0);
  } else {
    add((double)SP, 1.0);
  }
  return n3 > 12.0 * (double)std::max<int64_t>(c, 1) * n2 ? 1 : 0;
}

// Poles processed together for the interior part: as many as fit the budget.
int EngineImpl::pole_chunk() const {
  const int64_t items_bytes_per_pole =
      (int64_t)p * (D * D * (b_fp32(mode) ? 8 : 16) + NB * 2 * D * (b_fp32(mode) ? 8 : 16) +
                    D * SJ * (b_fp32(mode) ? 16 + 16 + 8 + 8 : 16));
  const int64_t budget = int64_t(48) << 30;
  int c = (int)std::max<int64_t>(1, budget / std::max<int64_t>(items_bytes_per_pole, 1));
  return std::min(c, poles.n_c);
}

// ---------------------------------------------------------------------------
// Factorizations for every pole (Sec. 3.1).
// ---------------------------------------------------------------------------
// The filter solves with S stop their recursion at SLW-wide diagonal blocks
// (SLW = 256 or 128 when it divides SP): their inverses are merged once per
// factorization, so that each solve needs a few large products instead of
// SP / 64 small sequential ones.
template <typename T>
void EngineImpl::wide_inverses(hipStream_t st, DMat<T> LU, DMat<T> inv, int nc) {
  SLW = (SP % 256 == 0 && SP > 256) ? 256 : ((SP % 128 == 0 && SP > 128) ? 128 : 0);
  if (!SLW) return;
  const int64_t per = (int64_t)SLW * 2 * SP;  // elements per plane per pole
  Swide.alloc(2 * per * nc * sizeof(T));
  DMat<T> w2{Swide.as<T>(), Swide.as<T>() + per * nc, SLW, per};
  const int64_t mw = (int64_t)(SLW / 2) * (SLW / 2) * std::max<int64_t>(SP / SLW, nc);
  Swork.alloc(std::max<int64_t>(Swork.bytes, 2 * mw * sizeof(T)));
  DMat<T> wk{Swork.as<T>(), Swork.as<T>() + mw, SLW / 2, 0};
  merge_inverses<T>(st, LU, inv, SP, nc, w2, SLW, wk);
}

void EngineImpl::factor(hipStream_t st, int w0, int wn) {
  const int nc = wn;  // poles in the window; pole index = w0 + item
  Shifts z{zeta.as<double>()};
  const int chunk = std::min(pole_chunk(), wn);
  const int items_max = chunk * p;
  // Schur complements (FP64 planar), all poles
  const int64_t sbytes = SP * SP * (int64_t)nc * sizeof(double);
  const bool two_level = tree.L > 0;
  DMat<double> S, Tg, TgT, Tt;
  const int64_t TG_ = tree.NGP, TGT_ = tree.TGP, TP_ = tree.TP;
  const int tL = tree.L;
  if (!two_level) {
    S64.alloc(2 * sbytes);
    S = DMat<double>{S64.as<double>(), S64.as<double>() + SP * SP * nc, SP, SP * SP};
    fill<double>(st, S, SP, SP, nc, 0.0);
    schur_init(st, S, s, SP, nc, w0, Cg.view(), z);
  } else {
    // the two-level blocks of S (group blocks, their top couplings, the top block)
    const int64_t ni = (int64_t)nc * tL;
    Tgg64.alloc(2 * TG_ * TG_ * ni * sizeof(double));
    TgT64.alloc(2 * TG_ * TGT_ * ni * sizeof(double));
    Ttt64.alloc(2 * TP_ * TP_ * nc * sizeof(double));
    Tg = DMat<double>{Tgg64.as<double>(), Tgg64.as<double>() + TG_ * TG_ * ni, TG_, TG_ * TG_};
    TgT = DMat<double>{TgT64.as<double>(), TgT64.as<double>() + TG_ * TGT_ * ni, TG_, TG_ * TGT_};
    Tt = DMat<double>{Ttt64.as<double>(), Ttt64.as<double>() + TP_ * TP_ * nc, TP_, TP_ * TP_};
    fill<double>(st, Tg, TG_, TG_, (int)ni, 0.0);
    fill<double>(st, TgT, TG_, TGT_, (int)ni, 0.0);
    fill<double>(st, Tt, TP_, TP_, nc, 0.0);
    tree_init(st, Tg, TgT, Tt, nc, w0, Cg.view(), tree, z);
  }
  const int64_t kk = D * D * (int64_t)items_max, ki = (int64_t)NB * 2 * D * items_max,
                xs = D * SJ * (int64_t)items_max;
  const bool fp32 = b_fp32(mode);           // the interior blocks
  s_mode = s_precision(mode, cols_hint);    // S
  const bool spectral = interior_solver == 1;
  if (spectral) {
    spectral_decompose(st);
  } else if (fp32) {
    K32.alloc(2 * kk * sizeof(float));
    Kinv32.alloc(2 * ki * sizeof(float));
    X32.alloc(2 * xs * sizeof(float));
  } else {
    K64.alloc(2 * kk * sizeof(double));
    Kinv64.alloc(2 * ki * sizeof(double));
  }
  X64.alloc(2 * xs * sizeof(double));
  if (fp32 && !spectral) R64.alloc(2 * xs * sizeof(double));
  int max_sweeps_used = 0;
  for (int l0 = w0; l0 < w0 + nc; l0 += chunk) {
    const int np = std::min(chunk, w0 + nc - l0);
    const int items = np * p;
    DMat<double> X{X64.as<double>(), X64.as<double>() + xs, D, D * SJ};
    if (spectral) {
      // no shifted block is factored: X = V (Lambda - zeta)^{-1} V^T Ehat
      timer.begin(st, 1);
      spectral_schur(st, l0, np, X);
      timer.end(st);
    } else if (fp32) {
      timer.begin(st, 0);
      DMat<float> K{K32.as<float>(), K32.as<float>() + kk, D, D * D};
      DMat<float> Ki{Kinv32.as<float>(), Kinv32.as<float>() + ki, NB, (int64_t)NB * 2 * D};
      fill<float>(st, K, D, D, items, 0.f);
      expand_shifted<float>(st, K, D, p, np, l0, dj.as<int32_t>(), Bg.view(), z, false, 0.0);
      lu_nopiv<float>(st, K, D, items, Ki, flags.as<unsigned>(), 1e-30);
      timer.end(st);
      timer.begin(st, 1);
      DMat<float> X3{X32.as<float>(), X32.as<float>() + xs, D, D * SJ};
      fill<float>(st, X3, D, SJ, items, 0.f);
      expand_rhs<float>(st, X3, p, np, l0, dj.as<int32_t>(), Eg.view(), z);
      lu_solve<float>(st, K, Ki, nullptr, D, X3, SJ, items);
      convert<double, float>(st, X3, X, D, SJ, items);
      DMat<double> Rm{R64.as<double>(), R64.as<double>() + xs, D, D * SJ};
      int sw = 0;
      for (;; ++sw) {
        zero_scalar(st, 0);
        residual_shifted(st, X, Rm, D, SJ, p, np, l0, dj.as<int32_t>(), sj.as<int32_t>(),
                         Bg.view(), Eg.view(), z, scal.as<double>());
        const double r = read_scalar(st, 0);
        if (!(r == r)) throw Error(ST_EBREAKDOWN, "non-finite residual in the interior solves");
        if (r <= tol * emax) break;
        if (sw >= sweeps)
          throw Error(ST_ENOCONV, "interior refinement did not converge (residual " +
                                      std::to_string(r / emax) + ")");
        convert<float, double>(st, Rm, X3, D, SJ, items);
        lu_solve<float>(st, K, Ki, nullptr, D, X3, SJ, items);
        add_to<double, float>(st, X3, X, D, SJ, items);
      }
      max_sweeps_used = std::max(max_sweeps_used, sw);
      timer.end(st);
    } else {
      // renumbered blocks: Ehat_j touches only the last TS rows, so
      // Ehat_j^T K^{-1} Ehat_j = Ehat_t^T (L_tt U_tt)^{-1} Ehat_t with the
      // trailing TS x TS blocks of the factors (those of K^{-1} are the
      // inverses of theirs), and only those rows of X are solved for
      timer.begin(st, 0);
      DMat<double> K{K64.as<double>(), K64.as<double>() + kk, D, D * D};
      DMat<double> Ki{Kinv64.as<double>(), Kinv64.as<double>() + ki, NB, (int64_t)NB * 2 * D};
      fill<double>(st, K, D, D, items, 0.0);
      expand_shifted<double>(st, K, D, p, np, l0, dj2.as<int32_t>(), Bg2.view(), z, false, 0.0);
      lu_nopiv<double>(st, K, D, items, Ki, flags.as<unsigned>(), 1e-300);
      timer.end(st);
      timer.begin(st, 1);
      const int64_t t0 = D - TS;
      fill<double>(st, X.sub(t0, 0), TS, SJ, items, 0.0);
      expand_rhs<double>(st, X, p, np, l0, dj2.as<int32_t>(), Eg2.view(), z);
      lu_solve<double>(st, K.sub(t0, t0), Ki.sub(0, 2 * t0), nullptr, TS, X.sub(t0, 0), SJ,
                       items);
      timer.end(st);
    }
    timer.begin(st, 2);
    // (X in the renumbered rows on the FP64 path)
    const DevPairCsr et = (!spectral && !fp32) ? Etg2.view() : Etg.view();
    if (!two_level) {
      DMat<double> Sc = S.item(l0 - w0);
      for (size_t c = 0; c < colors_d.size(); ++c)
        schur_scatter(st, Sc, X, SJ, p, np, l0, colors_d[c].as<int32_t>(),
                      (int)P->colors[c].size(), sj.as<int32_t>(), adj.as<int32_t>(), et, z);
    } else {
      const int64_t i0 = (int64_t)(l0 - w0) * tL;
      for (size_t c = 0; c < colors_d.size(); ++c)
        tree_scatter(st, Tg.item(i0), TgT.item(i0), Tt.item(l0 - w0), X, SJ, p, np, l0,
                     colors_d[c].as<int32_t>(), (int)P->colors[c].size(), sj.as<int32_t>(), et,
                     tree, z);
    }
    timer.end(st);
  }
  check_flags(st, "interior factorization");
  timer.sweeps_schur = max_sweeps_used;
  // factor S(zeta_l), all poles in one batch
  timer.begin(st, 3);
  if (two_level) {
    tree_factor(st, nc);
  } else if (s_mode == 1) {
    S32.alloc(2 * SP * SP * (int64_t)nc * sizeof(float));
    Sinv32.alloc(2 * (int64_t)NB * 2 * SP * nc * sizeof(float));
    DMat<float> S3{S32.as<float>(), S32.as<float>() + SP * SP * nc, SP, SP * SP};
    DMat<float> Si{Sinv32.as<float>(), Sinv32.as<float>() + (int64_t)NB * 2 * SP * nc, NB,
                   (int64_t)NB * 2 * SP};
    convert<float, double>(st, S, S3, SP, SP, nc);
    // the refinement residual takes three real products instead of four
    // when S_re + S_im fits in GAUSS_MAX_BYTES
    gauss3 = sbytes <= GAUSS_MAX_BYTES;
    if (gauss3) {
      Ssum.alloc(sbytes);
      DMat<double> Sz{Ssum.as<double>(), nullptr, SP, SP * SP};
      k_plane_sum<<<dim3(grid1(SP * SP), nc), 256, 0, st>>>(S, Sz, SP, SP);
      RFD_CHECK_LAUNCH();
    } else {
      Ssum.release();
    }
    lu_nopiv<float>(st, S3, SP, nc, Si, flags.as<unsigned>(), 1e-30);
    wide_inverses<float>(st, S3, Si, nc);
  } else {
    Sinv64.alloc(2 * (int64_t)NB * 2 * SP * nc * sizeof(double));
    DMat<double> Si{Sinv64.as<double>(), Sinv64.as<double>() + (int64_t)NB * 2 * SP * nc, NB,
                    (int64_t)NB * 2 * SP};
    lu_nopiv<double>(st, S, SP, nc, Si, flags.as<unsigned>(), 1e-300);
    wide_inverses<double>(st, S, Si, nc);
  }
  // the interior factors are no longer needed; large ones are released (a
  // release synchronises the device, small ones stay for the next solve)
  if (!keep_interior && K32.bytes + K64.bytes + X32.bytes + R64.bytes > (size_t(16) << 30)) {
    K32.release();
    Kinv32.release();
    X32.release();
    R64.release();
    K64.release();
    Kinv64.release();
  }
  if (X64.bytes > (size_t(8) << 30)) X64.release();
  timer.end(st);
  check_flags(st, "Schur complement factorization");
  win0 = w0;
  winn = wn;
  factored = (w0 == 0 && wn == poles.n_c);
}

// Poles whose factors fit together in the device memory: all of them when
// they fit, else the largest window that does (at least one pole).  Counts
// the FP64 Schur complements (and the FP32 copies), their block inverses, the
// filter's right-hand sides for a block of m columns, and the interior
// factors of the poles processed together.
int EngineImpl::pole_window(int m) const {
  const int nc = poles.n_c;
  const bool f32 = s_precision(mode, cols_hint) == 1;  // S
  const bool b32 = b_fp32(mode);                        // the interior blocks
  const int64_t MP = round_up(std::max(m, 1), NB);
  const int64_t per_pole = tree.L > 0 ? tree_pole_bytes(MP, f32 ? 1 : 0)
                                       : 2 * SP * SP * (f32 ? 8 + 4 : 8) +
                                             2 * (int64_t)NB * 2 * SP * (f32 ? 4 : 8) +
                                             2 * SP * MP * (f32 ? 8 + 8 + 4 : 8);
  const int64_t per_chunk_pole =
      (int64_t)p * (D * D * (b32 ? 8 : 16) + (int64_t)NB * 2 * D * (b32 ? 8 : 16) +
                    D * SJ * (b32 ? 48 : 16));
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return nc;
  }
  // what this pencil already holds counts as available
  const double avail = 0.8 * ((double)fr + (double)bytes_held());
  int w = (max_window > 0) ? std::min(max_window, nc) : nc;
  auto need = [&](int wn) {
    double b = (double)wn * per_pole + (double)std::min(pole_chunk(), wn) * per_chunk_pole;
    // S_re + S_im and the three-product work of the FP32 refinement
    if (tree.L == 0 && f32 && SP * SP * (int64_t)wn * 8 <= GAUSS_MAX_BYTES)
      b += (double)wn * (SP * SP * 8 + SP * MP * 24);
    return b;
  };
  while (w > 1 && need(w) > avail) --w;
  return w;
}

void EngineImpl::run_filter(hipStream_t st, const double* Y, int64_t ldy, int m, double* W,
                            int64_t ldw) {
  const int nc = poles.n_c;
  if (factored) {
    apply_filter(st, Y, ldy, m, W, ldw, false);
    return;
  }
  const int w = pole_window(m);
  if (w >= nc) {
    factor(st, 0, nc);
    apply_filter(st, Y, ldy, m, W, ldw, false);
    return;
  }
  for (int l = 0; l < nc; l += w) {
    factor(st, l, std::min(w, nc - l));
    apply_filter(st, Y, ldy, m, W, ldw, l > 0);
  }
  // only the last window's factors would remain: they are released, making
  // room for the interior part (the next application factors again)
  RFD_HIP(hipStreamSynchronize(st));
  for (DevBuf* b : {&K32, &K64, &Kinv32, &Kinv64, &X32, &X64, &R32, &R64, &S64, &S32, &Ssum,
                    &Xsum, &Pg, &Sinv32, &Sinv64, &Swide, &Swork, &Yc, &Xf, &Rf, &Rf32, &Tgg64,
                    &TgT64, &Ttt64, &Txc64, &Tgg32, &TgT32, &Txc32, &Ttt32, &Tinvg, &Tinvt, &Twide,
                    &Twork, &Tgt, &TRG, &TRT, &TXG, &TXT, &TRG32, &TRT32, &TU, &TXTg})
    b->release();
  factored = false;
}

// W = 2 Re sum_l omega_l S(zeta_l)^{-1} Y  (eq. (3.5)); Y real s x m (ld ldy),
// W real (ld ldw).  With FP32 factors every pole's solve is refined against S_64.
void EngineImpl::apply_filter(hipStream_t st, const double* Y, int64_t ldy, int m, double* Wout,
                              int64_t ldw, bool add) {
  if (tree.L > 0) {
    tree_apply(st, Y, ldy, m, Wout, ldw, add);
    return;
  }
  const int nc = winn;
  const double* om = omega.as<double>() + 2 * (int64_t)win0;
  const int64_t MP = round_up(m, NB);
  const int64_t ys = SP * MP * (int64_t)nc;
  Yc.alloc(2 * ys * sizeof(double));
  DMat<double> Ycm{Yc.as<double>(), Yc.as<double>() + ys, SP, SP * MP};
  DMat<double> S{S64.as<double>(), S64.as<double>() + SP * SP * nc, SP, SP * SP};
  timer.begin(st, 4);
  if (s_mode == 1) {
    Xf.alloc(2 * ys * sizeof(double));
    Rf32.alloc(2 * ys * sizeof(float));
    DMat<double> X{Xf.as<double>(), Xf.as<double>() + ys, SP, SP * MP};
    DMat<float> R3{Rf32.as<float>(), Rf32.as<float>() + ys, SP, SP * MP};
    DMat<float> S3{S32.as<float>(), S32.as<float>() + SP * SP * nc, SP, SP * SP};
    DMat<float> Si{Sinv32.as<float>(), Sinv32.as<float>() + (int64_t)NB * 2 * SP * nc, NB,
                   (int64_t)NB * 2 * SP};
    // |Y| for the stopping test
    zero_scalar(st, 1);
    DMat<double> Ym{const_cast<double*>(Y), nullptr, ldy, 0};
    absmax<double>(st, Ym, s, m, 1, scal.as<double>() + 1);
    const double ymax = read_scalar(st, 1);
    broadcast_rhs(st, Y, ldy, s, m, Ycm, SP, MP, nc);   // R = Y - S 0
    fill<double>(st, X, SP, MP, nc, 0.0);
    int sw = 0;
    for (;; ++sw) {
      convert<float, double>(st, Ycm, R3, SP, MP, nc);
      lu_solve<float>(st, S3, Si, nullptr, SP, R3, MP, nc, 3, wide<float>(nc), SLW,
                      solve_work<float>(MP, nc));
      add_to<double, float>(st, R3, X, SP, MP, nc);
      broadcast_rhs(st, Y, ldy, s, m, Ycm, SP, MP, nc);
      // R = Y - S_64 X as real products on the planes (large real FP64
      // products on the 128-wide tile): three in Gauss's form when S_re + S_im is
      // kept, else four
      {
        auto re = [](DMat<double> a) { a.im = nullptr; return a; };
        auto im = [](DMat<double> a) { a.re = a.im; a.im = nullptr; return a; };
        if (gauss3) {
          Xsum.alloc(ys * sizeof(double));
          Pg.alloc(2 * ys * sizeof(double));
          DMat<double> Sz{Ssum.as<double>(), nullptr, SP, SP * SP};
          DMat<double> Xz{Xsum.as<double>(), nullptr, SP, SP * MP};
          DMat<double> P1{Pg.as<double>(), nullptr, SP, SP * MP};
          DMat<double> P2{Pg.as<double>() + ys, nullptr, SP, SP * MP};
          k_plane_sum<<<dim3(grid1(SP * MP), nc), 256, 0, st>>>(X, Xz, SP, MP);
          RFD_CHECK_LAUNCH();
          gemm<double>(st, false, false, SP, MP, SP, 1.0, re(S), re(X), 0.0, P1, nc);
          gemm<double>(st, false, false, SP, MP, SP, 1.0, im(S), im(X), 0.0, P2, nc);
          gemm<double>(st, false, false, SP, MP, SP, -1.0, Sz, Xz, 1.0, im(Ycm), nc);
          k_gauss_combine<<<dim3(grid1(SP * MP), nc), 256, 0, st>>>(Ycm, P1, P2, SP, MP);
          RFD_CHECK_LAUNCH();
        } else {
          gemm<double>(st, false, false, SP, MP, SP, -1.0, re(S), re(X), 1.0, re(Ycm), nc);
          gemm<double>(st, false, false, SP, MP, SP, 1.0, im(S), im(X), 1.0, re(Ycm), nc);
          gemm<double>(st, false, false, SP, MP, SP, -1.0, re(S), im(X), 1.0, im(Ycm), nc);
          gemm<double>(st, false, false, SP, MP, SP, -1.0, im(S), re(X), 1.0, im(Ycm), nc);
        }
      }
      zero_scalar(st, 0);
      absmax<double>(st, Ycm, SP, MP, nc, scal.as<double>());
      const double r = read_scalar(st, 0);
      if (!(r == r)) throw Error(ST_EBREAKDOWN, "non-finite residual in the filter solves");
      if (r <= tol * ymax) break;
      if (sw + 1 >= sweeps)
        throw Error(ST_ENOCONV, "filter refinement did not converge (residual " +
                                    std::to_string(r / ymax) + ")");
    }
    timer.sweeps_filter = std::max(timer.sweeps_filter, sw + 1);
    filter_accumulate(st, X, om, nc, Wout, ldw, s, m, add);
  } else {
    DMat<double> Si{Sinv64.as<double>(), Sinv64.as<double>() + (int64_t)NB * 2 * SP * nc, NB,
                    (int64_t)NB * 2 * SP};
    broadcast_rhs(st, Y, ldy, s, m, Ycm, SP, MP, nc);
    lu_solve<double>(st, S, Si, nullptr, SP, Ycm, MP, nc, 3, wide<double>(nc), SLW,
                     solve_work<double>(MP, nc));
    filter_accumulate(st, Ycm, om, nc, Wout, ldw, s, m, add);
  }
  timer.end(st);
}

void Engine::filter_interface(hipStream_t st, int m, const double* Y0, int steps, double* Q,
                              int64_t ldq_cols, int* mu) {
  EngineImpl& e = *d_;
  if (!e.poles.set) throw Error(ST_ESTATE, "poles not set");
  const int64_t s = e.s;
  const int64_t cap = std::min<int64_t>(ldq_cols, std::min<int64_t>(s, (int64_t)steps * m));
  e.cols_hint = std::min<int64_t>(s, (int64_t)steps * m);
  e.W.alloc(sizeof(double) * s * (int64_t)m);
  double* W = e.W.as<double>();
  int total = 0, prev0 = 0, prevw = 0;
  for (int t = 1; t <= steps; ++t) {
    if (t == 1) {
      e.run_filter(st, Y0, s, m, W, s);
    } else {
      if (prevw == 0 || total >= cap) break;
      e.run_filter(st, Q + (int64_t)prev0 * s, s, prevw, W, s);
    }
    const int width = (t == 1) ? m : prevw;
    const int room = (int)(cap - total);
    e.timer.begin(st, 5);
    int r = orth_block(st, W, s, s, width, Q, s, total, Q + (int64_t)total * s, s, 1e-13,
                       room, e.ow);
    e.timer.end(st);
    r = std::min(r, room);
    prev0 = total;
    prevw = r;
    total += r;
  }
  *mu = total;
  // keep Q for the interior part
  e.mu = total;
  e.Qint.alloc(sizeof(double) * std::max<int64_t>(s * total, 1));
  if (total > 0)
    RFD_HIP(hipMemcpyAsync(e.Qint.p, Q, sizeof(double) * s * total, hipMemcpyDeviceToDevice, st));
  e.interior_ready = false;
}

// Alg. 3.1 taken on a block (Sec. 3.2): Q_1 = orth(Y0); for t = 1, 2, ..:
// W = F Q_t, the trace of A_t = Q_t^T W is added to tr(T_t) (the sum of its
// eigenvalues, line 13), and every `every` vectors the relative change of
// tr(T_t) since the previous test is compared with tol; Q_{t+1} = orth(W)
// against Q_1..Q_t (twice, lines 4-12).  Q = [Q_1 .. Q_t] at the stop.
void Engine::filter_lanczos(hipStream_t st, int m, const double* Y0, double tol, int max_steps,
                            int every, double* Q, int64_t ldq_cols, int* mu, int* steps,
                            double* traces, int* converged) {
  EngineImpl& e = *d_;
  if (!e.poles.set) throw Error(ST_ESTATE, "poles not set");
  const int64_t s = e.s;
  const int64_t cap = std::min<int64_t>(ldq_cols, s);
  e.cols_hint = std::min<int64_t>(s, (int64_t)max_steps * m);
  e.W.alloc(sizeof(double) * s * (int64_t)m);
  double* W = e.W.as<double>();
  RFD_HIP(hipMemcpyAsync(W, Y0, sizeof(double) * s * m, hipMemcpyDeviceToDevice, st));
  e.timer.begin(st, 5);
  int total = std::min<int>(orth_block(st, W, s, s, m, Q, s, 0, Q, s, 1e-13, (int)cap, e.ow),
                            (int)cap);
  e.timer.end(st);
  int prev0 = 0, prevw = total, t = 0;
  const int test_blocks = std::max(1, (every + m - 1) / m);
  double tr = 0.0, tr_test = 0.0;
  bool have_test = false;
  *converged = 0;
  DevBuf& dots = e.tmp[23];
  dots.alloc(sizeof(double) * std::max(m, 1));
  std::vector<double> hd(std::max(m, 1));
  while (prevw > 0) {
    ++t;
    e.run_filter(st, Q + (int64_t)prev0 * s, s, prevw, W, s);
    col_dots(st, Q + (int64_t)prev0 * s, s, W, s, s, prevw, dots.as<double>());
    RFD_HIP(hipMemcpyAsync(hd.data(), dots.p, sizeof(double) * prevw, hipMemcpyDeviceToHost, st));
    RFD_HIP(hipStreamSynchronize(st));
    double a = 0.0;
    for (int i = 0; i < prevw; ++i) a += hd[i];
    tr += a;
    if (traces && t <= max_steps) traces[t - 1] = tr;
    if (t % test_blocks == 0) {
      if (have_test && std::fabs(tr - tr_test) <= tol * std::fabs(tr)) {
        *converged = 1;
        break;
      }
      tr_test = tr;
      have_test = true;
    }
    if (t >= max_steps || total >= cap) break;
    e.timer.begin(st, 5);
    int r = orth_block(st, W, s, s, prevw, Q, s, total, Q + (int64_t)total * s, s, 1e-13,
                       (int)(cap - total), e.ow);
    e.timer.end(st);
    r = std::min<int>(r, (int)(cap - total));
    if (r <= 0) break;
    prev0 = total;
    prevw = r;
    total += r;
  }
  *mu = total;
  *steps = t;
  e.mu = total;
  e.Qint.alloc(sizeof(double) * std::max<int64_t>(s * total, 1));
  if (total > 0)
    RFD_HIP(hipMemcpyAsync(e.Qint.p, Q, sizeof(double) * s * total, hipMemcpyDeviceToDevice, st));
  e.interior_ready = false;
}

// Negative real parts among the first act[b] (or act0 when act is null)
// diagonal entries of the n x n items b of LU (the pivots of the LU without
// pivoting of a real symmetric matrix stored as complex with zero imaginary
// part), added to *count.
__global__ void k_count_negative_pivots(DMat<double> LU, const int32_t* act, int64_t act0,
                                        int64_t n, int per, unsigned long long* count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  const int64_t na = act ? act[b % per] : act0;
  if (i >= n || i >= na) return;
  const DMat<double> x = LU.item(b);
  if (x.re[i + i * x.ld] < 0.0) atomicAdd(count, 1ull);
}

int64_t Engine::inertia(hipStream_t st, double tau) {
  d_->join_prepare();
  EngineImpl& e = *d_;
  const Poles saved = e.poles;
  const int saved_mode = e.mode;
  Poles q;
  q.alpha = q.beta = tau;
  q.n_c = 1;
  q.zeta = {std::complex<double>(tau, 0.0)};
  q.omega = {std::complex<double>(0.0, 0.0)};
  q.set = true;
  set_poles(q);
  e.mode = 0;
  int64_t neg = 0;
  try {
    e.keep_interior = true;
    e.factor(st, 0, 1);
    e.keep_interior = false;
    DevBuf& cnt = e.tmp[22];
    cnt.alloc(sizeof(unsigned long long));
    RFD_HIP(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), st));
    auto* c = cnt.as<unsigned long long>();
    int64_t below = 0;
    if (e.interior_solver == 1) {
      // subdomain blocks: eigenvalues of (B_j, M_Bj) below tau
      for (int j = 0; j < e.p; ++j) {
        const int d = (int)e.P->interior[j].size();
        for (int i = 0; i < d; ++i) below += e.lam_h[(size_t)j * e.DE + i] < tau ? 1 : 0;
      }
    } else {
      // subdomain blocks: items j of the single pole, d_j active rows each
      DMat<double> K{e.K64.as<double>(), e.K64.as<double>() + e.D * e.D * (int64_t)e.p, e.D,
                     e.D * e.D};
      if (!e.K64.p) throw Error(ST_ESTATE, "inertia: interior factors were released");
      // (renumbered items: the pad rows' unit pivots add nothing)
      k_count_negative_pivots<<<dim3(grid1(e.D), e.p), 256, 0, st>>>(K, e.dj2.as<int32_t>(), 0,
                                                                     e.D, e.p, c);
      RFD_CHECK_LAUNCH();
    }
    if (e.tree.L > 0) {
      const TreeDev& t = e.tree;
      DMat<double> G{e.Tgg64.as<double>(), e.Tgg64.as<double>() + t.NGP * t.NGP * t.L, t.NGP,
                     t.NGP * t.NGP};
      DMat<double> T{e.Ttt64.as<double>(), e.Ttt64.as<double>() + t.TP * t.TP, t.TP, t.TP * t.TP};
      k_count_negative_pivots<<<dim3(grid1(t.NGP), t.L), 256, 0, st>>>(G, t.ngd.as<int32_t>(), 0,
                                                                       t.NGP, t.L, c);
      RFD_CHECK_LAUNCH();
      k_count_negative_pivots<<<dim3(grid1(t.TP), 1), 256, 0, st>>>(T, nullptr, t.t, t.TP, 1, c);
      RFD_CHECK_LAUNCH();
    } else {
      DMat<double> S{e.S64.as<double>(), e.S64.as<double>() + e.SP * e.SP, e.SP, e.SP * e.SP};
      k_count_negative_pivots<<<dim3(grid1(e.SP), 1), 256, 0, st>>>(S, nullptr, e.s, e.SP, 1, c);
      RFD_CHECK_LAUNCH();
    }
    unsigned long long h = 0;
    RFD_HIP(hipMemcpyAsync(&h, c, sizeof(h), hipMemcpyDeviceToHost, st));
    RFD_HIP(hipStreamSynchronize(st));
    neg = (int64_t)h + below;
  } catch (...) {
    e.keep_interior = false;
    e.mode = saved_mode;
    e.factored = false;
    if (saved.set) set_poles(saved);
    throw;
  }
  e.mode = saved_mode;
  e.factored = false;
  if (saved.set) set_poles(saved);
  else e.poles = saved;
  return neg;
}

void Engine::filter_apply(hipStream_t st, int m, const double* Y, double* W) {
  EngineImpl& e = *d_;
  if (!e.poles.set) throw Error(ST_ESTATE, "poles not set");
  e.cols_hint = m;
  e.run_filter(st, Y, e.s, m, W, e.s);
}

}  // namespace rfd
