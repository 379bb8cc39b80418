// Internal state of an Engine (see engine.hpp): device copies of the pencil
// and its reordering maps, factor buffers, the interface basis and the
// interior / Rayleigh-Ritz workspaces.
#pragma once

#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

#include "engine.hpp"
#include "eig.hpp"
#include "nested.hpp"
#include "orth.hpp"
#include "sparse.hpp"

namespace rfd {

struct DevPairGroup {
  DevBuf roff, ptr, idx, a, m;
  DevPairCsr view() const;
};

struct PhaseTimer {
  struct Rec {
    int phase;
    hipStream_t s;
    hipEvent_t a, b;
  };
  std::mutex mu;  // phases may run on two host threads (interior preparation)
  bool enabled = false;
  std::vector<Rec> open, done;
  double acc[16] = {0};
  int sweeps_schur = 0, sweeps_filter = 0;
  void begin(hipStream_t s, int phase);
  void end(hipStream_t s);
  void collect(double* ms16);
  ~PhaseTimer();
};

struct EngineImpl {
  const Csr* A = nullptr;
  const Csr* M = nullptr;
  const Partition* P = nullptr;
  int64_t n = 0, s = 0, SP = 0, D = 0, SJ = 0;
  int p = 0;
  double normA = 0, emax = 0;
  // pencil and maps
  DevPairGroup Bg, Eg, Etg, Cg;
  DevBuf dj, sj, adj, order, ioff;
  // The subdomain blocks with rows renumbered for the FP64 Schur solves:
  // padding first (unit diagonal), then the rows that Ehat_j does not touch,
  // then the TS-row trailing part that holds every row it touches, so that
  // Ehat_j^T K_j^{-1} Ehat_j needs only the trailing blocks of K_j's factors.
  // Items are D x D with all D rows active (dj2 = D).
  DevPairGroup Bg2, Eg2, Etg2;
  DevBuf dj2;
  int64_t TS = 0;
  int64_t SJA = 0;  // largest interface adjacency of a subdomain (columns of Ehat_j)
  // FP64 factors with Schur solves on the trailing blocks cost, per item and
  // in complex multiply-adds, D^3 / 3 + TS^2 SJ; FP32 factors (half the
  // time on the matrix cores) with refinement, whose solves need the full
  // solution, about (D^3 / 3 + 2 D^2 SJ) / 2 (one correcting solve).  FP64
  // pays when D^3 / 6 < SJ (D^2 - TS^2).
  bool trailing_pays() const {
    const double d = (double)D, t = (double)TS, c = (double)SJA;
    return d * d * d / 6.0 < c * (d * d - t * t);
  }
  // FP32 factors of the shifted interior blocks for precision mode md: always
  // with md = 1; with md = 2 unless FP64 with trailing solves costs less
  bool b_fp32(int md) const { return md == 1 || (md == 2 && !trailing_pays()); }
  std::vector<DevBuf> colors_d;
  DevBuf Aptr, Aidx, Aval, Mptr, Midx, Mval;      // original numbering
  DevBuf Arptr, Aridx, Arval, Mrptr, Mridx, Mrval;  // reordered numbering (lazy)
  DevBuf Mrdiag;                                   // diag(M), reordered (diagonal M)
  // poles and precision
  Poles poles;
  DevBuf zeta, omega;
  int mode = 0;           // 0: FP64, 1: FP32 factors + FP64 refinement, 2: FP32 where it pays
  int s_mode = 0;         // precision of S's factors in the current factorization (0 / 1)
  int64_t cols_hint = 0;  // columns the coming filter applications carry in all
  // 1 when the factors of S are FP32 for precision mode md and c columns
  int s_precision(int md, int64_t c) const;
  double tol = 1e-13;
  int sweeps = 8;
  bool factored = false;
  bool keep_interior = false;  // factor() keeps the interior factors (inertia counts)
  // factor buffers
  DevBuf K32, K64, Kinv32, Kinv64, X32, X64, R32, R64;
  DevBuf S64, S32, Sinv32, Sinv64;
  DevBuf Swide, Swork;  // inverses of the SLW-wide diagonal blocks of S's factors, workspace
  int SLW = 0;
  DevBuf Yc, Xf, Rf, Rf32, W;
  // FP32 mode: S_re + S_im per pole, for the refinement residual in Gauss's
  // three-product form (kept when it takes at most GAUSS_MAX_BYTES)
  DevBuf Ssum, Xsum, Pg;
  bool gauss3 = false;
  static constexpr int64_t GAUSS_MAX_BYTES = int64_t(4) << 30;
  OrthWork ow;
  // Two-level interface (set_interface_groups; tree.L = 0: dense S).  Blocks
  // of S per pole (FP64: Tgg64, TgT64, Ttt64, kept unfactored in FP32 mode for
  // the refinement residual), their FP32 copies and factors, X_g = S_gg^{-1}
  // S_gT (Txc), the top complement's block inverses and wide leaves, and the
  // blocked right-hand sides of the filter solves.
  TreeDev tree;
  DevBuf Tgg64, TgT64, Ttt64, Txc64, Tgg32, TgT32, Txc32, Ttt32, Tinvg, Tinvt, Twide, Twork, Tgt;
  DevBuf TRG, TRT, TXG, TXT, TRG32, TRT32, TU, TXTg;
  int TLW = 0;
  // factors the window's blocks (assembled by factor()); nc poles
  void tree_factor(hipStream_t st, int nc);
  // R <- S^{-1} R in the blocked layout with the current factors
  template <typename T>
  void tree_solve(hipStream_t st, DMat<T> RG, DMat<T> RT, int64_t MP, int nc);
  void tree_apply(hipStream_t st, const double* Y, int64_t ldy, int m, double* W, int64_t ldw,
                  bool add);
  // device bytes of one pole's blocks and of its filter right-hand sides
  int64_t tree_pole_bytes(int64_t MP, int md) const;
  // interface basis
  DevBuf Qint;
  int mu = 0;
  // interior part
  bool interior_ready = false;
  double sigma = 0;
  int nev_b = 0, psi = 0;
  std::vector<int> kappa;                 // per subdomain
  int kappa_tot = 0;
  bool vcache_valid = false;
  double vcache_sigma = 0;
  int vcache_nevb = -1;
  DevBuf Vb;                              // per subdomain D x VB (M_B-orthonormal)
  int64_t VB = 0;                         // padded column capacity per subdomain
  DevBuf kap_d, delta_d;
  DevBuf Mlu, Mluinv, mflag;              // non-diagonal M: M_Bj = L U (no pivoting), flags
  DevBuf Bs, Bsinv, Bspiv;                // B_sigma LU (FP64, pivoted)
  DevBuf Bswide, Bswork;                  // its BLW-wide diagonal inverses, leaf workspace
  int BLW = 0;
  bool bs_valid = false;
  double bs_sigma = 0;
  // spectral interior path: one eigendecomposition of every (B_j, M_Bj)
  // serves all shifts (poles, sigma) of the pencil
  int interior_solver = 0;                // 0: LU per shift, 1: spectral
  bool spec_valid = false, spec_f_valid = false;
  int64_t DE = 0;                         // rows the eigensolver runs on (max d_j)
  DevBuf Vs;                              // per subdomain D x D, M_B-orthonormal eigenvectors
  DevBuf lam_s;                           // per subdomain DE eigenvalues, ascending
  std::vector<double> lam_h;              // host copy of lam_s
  DevBuf Fs, Fz, Ts;                      // V^T Ehat (D x SJ), scaled copies, level work
  DevBuf Gsp;                             // decomposition work (Gram blocks, Ehat)
  double spec_orth = 0;                   // max |U^T U - I| after the orthonormalisation
  void spectral_decompose(hipStream_t st);
  void spectral_select(hipStream_t st, double sigma, int nev_b);
  void spectral_schur(hipStream_t st, int pole0, int np, DMat<double> X);
  void spectral_level(hipStream_t st, DMat<double> X, int64_t cols, double sigma);
  DevBuf Lev;                             // levels: per subdomain D x (psi * MUP)
  int64_t MUP = 0;
  DevBuf Zt;                              // M-orthonormal basis of range(Z), n x k (reordered)
  int64_t kz = 0;                         // columns of Zt
  DevBuf work1, work2, work3, work4, work5, work6;
  DevBuf ipiv_small, iscal, gwork, work6b;
  DevBuf rr_az, rr_h;   // Rayleigh-Ritz: A Z and the projected matrix
  // H = Z^T A Z assembled on a helper stream while Z is built: each finished
  // block of columns adds its rows (lower triangle, ld h_ld); h_ready marks
  // an H for the current basis of h_k columns (the eigensolver overwrites it)
  hipStream_t h_stream = nullptr;
  hipEvent_t h_lvl = nullptr, h_done = nullptr;
  bool h_ready = false, h_use = false;
  int64_t h_ld = 0, h_k = 0;
  void h_begin(bool use);
  void h_add_block(hipStream_t st, int64_t c0, int64_t r);
  DevBuf tmp[24];       // small per-call buffers, kept to avoid device-wide frees
  TriWork tw_v, tw_h;   // eigensolver work: subdomain blocks, projected matrix
  PhaseTimer timer;
  // every buffer that a solve grows (released by reset_caches(true))
  std::vector<DevBuf*> solve_buffers();
  DevBuf flags, scal;
  // interior preparation (V_j and the B_sigma factors) running on a thread
  // and stream of its own, concurrently with the filter
  int device = 0;
  std::thread prep;
  std::atomic<bool> prep_running{false};
  std::exception_ptr prep_err;
  hipStream_t prep_stream = nullptr, prep_stream2 = nullptr;
  DevBuf prep_flags;
  std::vector<DevBuf*> prep_buffers();
  void join_prepare();

  int64_t bytes_held() const;
  int64_t interior_bytes() const;
  double read_scalar(hipStream_t s, int i);
  void zero_scalar(hipStream_t s, int i);
  void check_flags(hipStream_t s, const char* what, DevBuf* f = nullptr);
  int pole_chunk() const;
  // Factors poles [w0, w0 + wn) (the "window": S buffers hold wn poles)
  void factor(hipStream_t st, int w0, int wn);
  template <typename T>
  void wide_inverses(hipStream_t st, DMat<T> LU, DMat<T> inv, int nc);
  // views of the wide inverses of S and of a leaf workspace for r columns
  template <typename T>
  DMat<T> wide(int nc) {
    const int64_t per = (int64_t)SLW * 2 * SP;
    if (!SLW) return DMat<T>{};
    return DMat<T>{Swide.as<T>(), Swide.as<T>() + per * nc, SLW, per};
  }
  template <typename T>
  DMat<T> solve_work(int64_t r, int nc) {
    if (!SLW) return DMat<T>{};
    const int64_t per = (int64_t)SLW * r;
    Swork.alloc(std::max<int64_t>(Swork.bytes, 2 * per * nc * sizeof(T)));
    return DMat<T>{Swork.as<T>(), Swork.as<T>() + per * nc, SLW, per};
  }
  // W (=, or += when add) 2 Re sum over the window of omega_l S_l^{-1} Y
  void apply_filter(hipStream_t st, const double* Y, int64_t ldy, int m, double* W, int64_t ldw,
                    bool add);
  // The filter over every pole: factored once when all poles fit the device
  // memory, else window by window (factors dropped after their window)
  void run_filter(hipStream_t st, const double* Y, int64_t ldy, int m, double* W, int64_t ldw);
  int pole_window(int m) const;  // poles whose factors fit together (n_c when all do)
  int win0 = 0, winn = 0;
  int max_window = 0;  // caller's cap on the pole window (0: by free memory)
  void ensure_reordered(hipStream_t st);
  // Y = M X in the reordered numbering (a row scaling when M is diagonal)
  void apply_m(hipStream_t st, const double* X, int64_t ldx, double* Y, int64_t ldy,
               int64_t cols);
  void col_mnorms(hipStream_t st, const double* X, int64_t cols, double* MX, double* out);
  void interior_basis(hipStream_t st, double sigma, int nev_b);
  double mb_standard_form(hipStream_t st, DMat<double> C, double* sq, double* isq, double sigma);
  void factor_bsigma(hipStream_t st, double sigma, DevBuf* fl = nullptr, bool check = true);
  int gram_orth(hipStream_t st, const double* B, int ncol, double* MB, double* Out,
                double droptol);
  void project_out(hipStream_t st, double* X, int ncols, double* MX, const double* Zp,
                   int64_t kprev, int passes);
};

}  // namespace rfd
