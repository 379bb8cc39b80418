// Device-side execution of the RF-DDES path for one pencil: buffers, the
// per-pole factorizations, the interface filter, the interior part and the
// Rayleigh-Ritz step.  Owned by a pencil handle (capi.cpp).
#pragma once

#include <memory>

#include "pencil.hpp"

namespace rfd {

struct EngineImpl;

class Engine {
 public:
  Engine(const Csr& A, const Csr& M, const Partition& P);
  ~Engine();
  void set_poles(const Poles& poles);
  void set_precision(int mode, double tol, int sweeps);
  void filter_interface(hipStream_t s, int m, const double* Y0, int steps, double* Q,
                        int64_t ldq_cols, int* mu);
  void filter_apply(hipStream_t s, int m, const double* Y, double* W);
  // Number of eigenvalues of (A, M) below the real shift tau: the negative
  // pivots of the FP64 LU without pivoting of every B_j - tau M_Bj and of
  // S(tau) (Sylvester's law of inertia with Haynsworth's additivity).
  int64_t inertia(hipStream_t s, double tau);
  // Alg. 3.1 on a block of m vectors with the trace stopping test (see
  // rfd_filter_lanczos); traces: host, max_steps entries or null.
  void filter_lanczos(hipStream_t s, int m, const double* Y0, double tol, int max_steps,
                      int every, double* Q, int64_t ldq_cols, int* mu, int* steps,
                      double* traces, int* converged);
  // Starts the sigma-dependent interior caches (V_j, the B_sigma factors) on
  // an internal thread and stream; every call below except filter_interface
  // and filter_apply first waits for it (and reports its error).
  void prepare_interior(double sigma, int nev_b);
  void solve_interior(hipStream_t s, double sigma, int nev_b, int psi, int64_t* k);
  void rayleigh_ritz(hipStream_t s, int max_out, double* evals, double* evecs, double* resid,
                     int* nfound);
  int64_t device_bytes() const;
  // Upper estimate of the device memory one solve with these parameters holds.
  int64_t estimate_bytes(int mode, int n_c, int m, int steps, int nev_b, int psi) const;
  void reset_caches(bool release);
  void copy_basis(hipStream_t s, double* dst, int64_t cap, int64_t* k);
  void set_timing(bool on);
  void set_pole_window(int w);
  // Two-level factorization of S(zeta) over L interface groups (group[a] per
  // interface position, -1 = top set); L = 0 returns to the dense S.
  void set_interface_groups(int L, const int32_t* group);
  void phase_times(double* ms16);
  // 0: every shifted interior block B_j - z M_Bj is factored (LU); 1: the
  // spectral path, one eigendecomposition of every (B_j, M_Bj) per pencil
  // serving all poles and every sigma (Sec. 4.1).  Returns the previous kind.
  int set_interior_solver(int kind);
  // Largest |U^T U - I| of the last spectral decomposition (0 before one).
  double spectral_orthogonality() const;

 private:
  std::unique_ptr<EngineImpl> d_;
};

}  // namespace rfd
