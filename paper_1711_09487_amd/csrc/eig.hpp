// Dense FP64 symmetric eigensolver for selected eigenpairs (batched):
// Householder tridiagonalization, Sturm-count bisection, inverse iteration
// with reorthogonalisation inside clusters, back-transformation.
#pragma once

#include <vector>

#include "rfd_common.hpp"

namespace rfd {

constexpr int TRI_NB = 32;  // panel width of the blocked tridiagonalization
constexpr int TRI_TB = 64;  // tile of its symmetric mat-vec

// Tile blocks (plus one) of the mat-vec over an n x n matrix.
inline int64_t tri_blocks(int64_t n) { return (n + TRI_TB - 1) / TRI_TB + 1; }

// Work space of the eigensolver (kept by the caller so that repeated solves
// of one shape reuse it).
struct TriWork {
  DevBuf d, e, tau, pt, acol, vw, red, sq, ptvp;
  DevBuf wv, wg, wt, w1, w2;  // back-transformation panels
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

// Reflectors per compact-WY block (I - V T V^T).
constexpr int WY_NB = 128;

// T (WY_NB x WY_NB, upper triangular, per item) of the compact-WY form
// H_i0 .. H_{i0+nbp-1} = I - V T V^T, from G = V^T V (WY_NB x WY_NB per item,
// finite; its rows and columns beyond nbp are not used) and the scalars
// tau[b * ld_tau + i0 + k], k < nbp.  Rows and columns of T beyond nbp are 0.
void wy_triangle(hipStream_t s, const double* G, const double* tau, int64_t ld_tau, int64_t i0,
                 int nbp, double* T, int batch);

// Y <- Q Y with Q the product of the Householder reflectors left in A by
// sy_tridiag (cols columns per item; columns beyond num[b] must be zero or
// are transformed along).
void back_transform(hipStream_t s, DMat<double> A, TriWork& w, int64_t n, int batch,
                    DMat<double> Y, const int* num, int maxcols);

}  // namespace rfd
