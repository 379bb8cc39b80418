// Rank-revealing orthonormalisation of a tall FP64 block (see orth.hip).
#pragma once

#include "rfd_common.hpp"

namespace rfd {

struct OrthWork {
  DevBuf V, T, cn, used, piv, tau, scal, rank;
  DevBuf wg, wt, w1, w2;  // compact-WY formation of Q
  int64_t v_elems = 0;
  int m_cap = 0, mu_cap = 0;
  void reserve(int64_t rows, int m, int mu_max);
};

// W (rows x m, ld ldw) is projected twice against K (rows x mu0, ld ldk,
// orthonormal columns; mu0 may be 0), then factored by Householder QR with
// column pivoting; directions with residual norm <= rel_tol times the largest
// column norm of the unprojected W are dropped.  The r orthonormal columns
// are written to Qout (ld ldq); returns r (synchronises the stream).
// W is overwritten.
// At most max_r columns are produced.
int orth_block(hipStream_t s, double* W, int64_t ldw, int64_t rows, int m, const double* K,
               int64_t ldk, int mu0, double* Qout, int64_t ldq, double rel_tol, int max_r,
               OrthWork& w);

// out[j] = A[:, j]^T B[:, j] for j < cols (rows x cols, FP64), one workgroup
// per column with a fixed-order reduction.
void col_dots(hipStream_t s, const double* A, int64_t lda, const double* B, int64_t ldb,
              int64_t rows, int cols, double* out);

}  // namespace rfd
