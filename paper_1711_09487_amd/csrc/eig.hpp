// Dense FP64 symmetric eigensolver for selected eigenpairs (batched):
// Householder tridiagonalization, Sturm-count bisection, inverse iteration
// with reorthogonalisation inside clusters, back-transformation.  Plus a
// pivoted Cholesky factorization with triangular inverse (rank-revealing
// Gram reduction).
#pragma once

#include <vector>

#include "rfd_common.hpp"

namespace rfd {

constexpr int TRI_NB = 32;  // panel width of the blocked tridiagonalization

struct TriWork {
  DevBuf d, e, tau, pvec, acol, vw, red, sq;
  int64_t cap = 0;
  void reserve(int64_t n, int batch);
};

// A: batch of n x n symmetric matrices (ld, item stride).  On return the
// tridiagonal T = Q^T A Q is in (d, e) and A holds the Householder vectors:
// column j, rows j+2..n-1 with the implicit 1 at row j+1, and tau[j].
void sy_tridiag(hipStream_t s, DMat<double> A, int64_t n, int batch, TriWork& w);

// Number of eigenvalues of T (item b) below x[b * nx + i] -> cnt[b * nx + i].
void sturm_counts(hipStream_t s, const TriWork& w, int64_t n, int batch, const double* x, int nx,
                  int* cnt);

// Eigenvalues with indices lo[b] .. lo[b] + num[b] - 1 (ascending, 0-based) of
// item b by bisection -> lam[b * ld_lam + i].
void bisect(hipStream_t s, const TriWork& w, int64_t n, int batch, const int* lo, const int* num,
            int maxnum, double* lam, int64_t ld_lam);

// Eigenvectors of T for lam[b * ld_lam + i], i < num[b], into Y (n x ld_lam
// columns per item, ld n) by inverse iteration.  clus[b * ld_lam + i] = index
// of the first member of i's cluster (vectors of one cluster are
// orthogonalised against each other).
void inverse_iteration(hipStream_t s, const TriWork& w, int64_t n, int batch, const double* lam,
                       const int* num, const int* clus, int64_t ld_lam, DMat<double> Y,
                       DevBuf& scratch);

// Y <- Q Y with Q the product of the Householder reflectors left in A by
// sy_tridiag (cols columns per item; only the first num[b] are used).
void back_transform(hipStream_t s, DMat<double> A, const TriWork& w, int64_t n, int batch,
                    DMat<double> Y, const int* num, int maxcols);

// Pivoted Cholesky of the m x m SPD item G (in place, lower triangle):
// P^T G P = L L^T for the first r pivots, stopping when the largest remaining
// diagonal is <= tol * (largest initial diagonal).  piv[i] = original index of
// the i-th pivot, *rank = r.  Linv (m x m, ld m) receives L^{-1} (r x r).
void pivoted_cholesky(hipStream_t s, double* G, int64_t ldg, int64_t m, double tol, int* piv,
                      int* rank, double* Linv, int64_t ldl);

}  // namespace rfd
