// Rank-revealing orthonormalisation of a tall block (Alg. 3.1, lines 3-12,
// taken blockwise): projection against an existing orthonormal basis (twice),
// then Householder QR with column pivoting.  A direction is dropped once the
// largest remaining column norm falls to tol_abs.
//
// One launch per elimination step; one workgroup per column.  Every
// workgroup selects the pivot from the same read-only state (column norms and
// the consumed mask of the current step), so all agree without a grid
// barrier; each workgroup writes only its own column and its own entries of
// the next step's state (double-buffered by step parity).  The explicit
// factor Q = H_0 .. H_{r-1} [I_r; 0] is formed column by column in one more
// launch: column c needs only H_0 .. H_c.
#include <algorithm>

#include "dense.hpp"
#include "orth.hpp"

namespace rfd {

__device__ inline double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Column norms (one workgroup per column); optionally tol = factor * max.
__global__ void k_colnorms(const double* W, int64_t ldw, int64_t rows, double* out) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0;
  for (int64_t i = threadIdx.x; i < rows; i += blockDim.x) {
    const double v = W[i + c * ldw];
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[c] = sqrt(s);
}

__global__ void k_scaled_max(const double* v, int m, double factor, double* out) {
  __shared__ double red[256];
  double mx = 0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) mx = fmax(mx, v[i]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = factor * red[0];
}

__global__ void k_hqr_init(int m, int* used, int* rank) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < m) used[c] = 0;
  if (c == 0) *rank = -1;
}

__global__ __launch_bounds__(256) void k_hqr_step(double* A, int64_t lda, int64_t rows, int m,
                                                  int j, const double* tol_abs, double* cn,
                                                  int* used, int* piv, double* tau, double* V,
                                                  int64_t ldv, int* rank) {
  __shared__ double red[256];
  __shared__ int ired[256];
  __shared__ double sv[256];
  const int c = blockIdx.x, t = threadIdx.x;
  const int cur = j & 1, nxt = cur ^ 1;
  const double* cnc = cn + (int64_t)cur * m;
  double* cnn = cn + (int64_t)nxt * m;
  const int* usc = used + (int64_t)cur * m;
  int* usn = used + (int64_t)nxt * m;
  // pivot: the unconsumed column of largest norm (lowest index on ties)
  double best = -1.0;
  int bi = m;
  for (int q = t; q < m; q += blockDim.x)
    if (!usc[q] && cnc[q] > best) { best = cnc[q]; bi = q; }
  sv[t] = best;
  ired[t] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      if (sv[t + w] > sv[t] || (sv[t + w] == sv[t] && ired[t + w] < ired[t])) {
        sv[t] = sv[t + w];
        ired[t] = ired[t + w];
      }
    }
    __syncthreads();
  }
  const int P = ired[0];
  const double cmax = sv[0];
  __syncthreads();
  const bool stop = (P >= m) || !(cmax > *tol_abs) || (j >= rows);
  if (stop || usc[c]) {
    if (t == 0) {
      cnn[c] = cnc[c];
      usn[c] = usc[c];
      if (stop && c == 0 && *rank < 0) *rank = j;
    }
    return;
  }
  // Householder vector of column P below row j (beta = -sign(x0) ||x||)
  const double* ap = A + (int64_t)P * lda;
  double s2 = 0;
  for (int64_t i = j + t; i < rows; i += blockDim.x) s2 += ap[i] * ap[i];
  s2 = block_sum(s2, red);
  const double x0 = ap[j];
  const double nrm = sqrt(s2);
  const double beta = x0 >= 0 ? -nrm : nrm;
  const double tj = (beta - x0) / beta;
  const double scal = 1.0 / (x0 - beta);
  if (c == P) {
    double* v = V + (int64_t)j * ldv;
    for (int64_t i = t; i < rows; i += blockDim.x)
      v[i] = (i < j) ? 0.0 : (i == j ? 1.0 : ap[i] * scal);
    if (t == 0) {
      piv[j] = P;
      tau[j] = tj;
      cnn[c] = 0.0;
      usn[c] = 1;
    }
    return;
  }
  double* ac = A + (int64_t)c * lda;
  double d = 0;
  for (int64_t i = j + t; i < rows; i += blockDim.x) d += (i == j ? 1.0 : ap[i] * scal) * ac[i];
  d = block_sum(d, red);
  const double f = tj * d;
  double s3 = 0;
  for (int64_t i = j + t; i < rows; i += blockDim.x) {
    const double nv = ac[i] - f * (i == j ? 1.0 : ap[i] * scal);
    ac[i] = nv;
    if (i > j) s3 += nv * nv;
  }
  s3 = block_sum(s3, red);
  if (t == 0) {
    cnn[c] = sqrt(s3);
    usn[c] = 0;
  }
}

__global__ void k_hqr_finish_rank(int* rank, int steps) {
  if (*rank < 0) *rank = steps;
}

// Column c of Q = H_0 H_1 .. H_c e_c, c < rank.
__global__ __launch_bounds__(256) void k_hqr_formq(const double* V, int64_t ldv, const double* tau,
                                                   const int* rank, int64_t rows, double* Q,
                                                   int64_t ldq) {
  __shared__ double red[256];
  const int c = blockIdx.x, t = threadIdx.x;
  if (c >= *rank) return;
  double* q = Q + (int64_t)c * ldq;
  for (int64_t i = t; i < rows; i += blockDim.x) q[i] = (i == c) ? 1.0 : 0.0;
  __syncthreads();
  for (int jj = c; jj >= 0; --jj) {
    const double* v = V + (int64_t)jj * ldv;
    double d = 0;
    for (int64_t i = jj + t; i < rows; i += blockDim.x) d += v[i] * q[i];
    d = block_sum(d, red);
    const double f = tau[jj] * d;
    for (int64_t i = jj + t; i < rows; i += blockDim.x) q[i] -= f * v[i];
    __syncthreads();
  }
}

void OrthWork::reserve(int64_t rows_, int m_, int mu_max) {
  const int64_t need_v = rows_ * (int64_t)m_;
  if (need_v > v_elems || m_ > m_cap || mu_max > mu_cap) {
    v_elems = std::max(v_elems, need_v);
    m_cap = std::max(m_cap, m_);
    mu_cap = std::max(mu_cap, mu_max);
    V.alloc(sizeof(double) * v_elems);
    T.alloc(sizeof(double) * (int64_t)mu_cap * m_cap);
    cn.alloc(sizeof(double) * 2 * (int64_t)m_cap);
    used.alloc(sizeof(int) * 2 * (int64_t)m_cap);
    piv.alloc(sizeof(int) * (int64_t)m_cap);
    tau.alloc(sizeof(double) * (int64_t)m_cap);
    scal.alloc(sizeof(double) * 2);
    rank.alloc(sizeof(int));
  }
}

int orth_block(hipStream_t s, double* W, int64_t ldw, int64_t rows, int m, const double* K,
               int64_t ldk, int mu0, double* Qout, int64_t ldq, double rel_tol, int max_r,
               OrthWork& w) {
  w.reserve(rows, m, std::max(mu0, 1));
  double* cn = w.cn.as<double>();
  double* tol = w.scal.as<double>();
  // tolerance from the unprojected block
  k_colnorms<<<m, 256, 0, s>>>(W, ldw, rows, cn);
  RFD_CHECK_LAUNCH();
  k_scaled_max<<<1, 256, 0, s>>>(cn, m, rel_tol, tol);
  RFD_CHECK_LAUNCH();
  if (mu0 > 0) {
    DMat<double> Km{const_cast<double*>(K), nullptr, ldk, 0};
    DMat<double> Wm{W, nullptr, ldw, 0};
    DMat<double> Tm{w.T.as<double>(), nullptr, mu0, 0};
    for (int pass = 0; pass < 2; ++pass) {
      gemm<double>(s, true, false, mu0, m, rows, 1.0, Km, Wm, 0.0, Tm, 1);
      gemm<double>(s, false, false, rows, m, mu0, -1.0, Km, Tm, 1.0, Wm, 1);
    }
    k_colnorms<<<m, 256, 0, s>>>(W, ldw, rows, cn);
    RFD_CHECK_LAUNCH();
  }
  k_hqr_init<<<grid1(m), 256, 0, s>>>(m, w.used.as<int>(), w.rank.as<int>());
  RFD_CHECK_LAUNCH();
  const int steps = (int)std::min<int64_t>(std::min<int64_t>(rows, m), max_r);
  if (steps <= 0) return 0;
  for (int j = 0; j < steps; ++j) {
    k_hqr_step<<<m, 256, 0, s>>>(W, ldw, rows, m, j, tol, cn, w.used.as<int>(), w.piv.as<int>(),
                                 w.tau.as<double>(), w.V.as<double>(), rows, w.rank.as<int>());
    RFD_CHECK_LAUNCH();
  }
  k_hqr_finish_rank<<<1, 1, 0, s>>>(w.rank.as<int>(), steps);
  RFD_CHECK_LAUNCH();
  k_hqr_formq<<<steps, 256, 0, s>>>(w.V.as<double>(), rows, w.tau.as<double>(), w.rank.as<int>(),
                                    rows, Qout, ldq);
  RFD_CHECK_LAUNCH();
  int r = 0;
  RFD_HIP(hipMemcpyAsync(&r, w.rank.as<int>(), sizeof(int), hipMemcpyDeviceToHost, s));
  RFD_HIP(hipStreamSynchronize(s));
  return r;
}

}  // namespace rfd
