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
// factor Q = H_0 .. H_{r-1} [I_r; 0] is formed in compact-WY blocks of
// reflectors (I - V T V^T), last block first, with matrix products.
#include <algorithm>

#include "dense.hpp"
#include "eig.hpp"
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

// Sums over a workgroup of exactly 256 threads (four wavefronts): shuffles
// within each wavefront, then the four partial sums in a fixed order.
__device__ inline double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline void block_sum256x2(double& a, double& b, double* red) {
  a = wave_sum64(a);
  b = wave_sum64(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w] = a;
    red[4 + w] = b;
  }
  __syncthreads();
  a = (red[0] + red[1]) + (red[2] + red[3]);
  b = (red[4] + red[5]) + (red[6] + red[7]);
  __syncthreads();
}
__device__ inline double block_sum256(double a, double* red) {
  double b = 0.0;
  block_sum256x2(a, b, red);
  return a;
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
  __shared__ double red[8];  // two sums of four wavefront partials
  __shared__ int ired[4];    // pivot candidates of the four wavefronts
  __shared__ double sv[4];
  const int c = blockIdx.x, t = threadIdx.x;
  const int cur = j & 1, nxt = cur ^ 1;
  const double* cnc = cn + (int64_t)cur * m;
  double* cnn = cn + (int64_t)nxt * m;
  const int* usc = used + (int64_t)cur * m;
  int* usn = used + (int64_t)nxt * m;
  // pivot: the unconsumed column of largest norm (lowest index on ties),
  // per thread, then across each wavefront by shuffles, then the four
  // wavefronts in order
  // (loads in rounds of four per thread, all issued before the first is
  // used, from clamped indices: a load per iteration would wait each time)
  double best = -1.0;
  int bi = m;
  for (int q0 = t; q0 < m; q0 += 4 * 256) {
    double cv[4];
    int uv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + 256 * u, qc = q < m ? q : m - 1;
      cv[u] = cnc[qc];
      uv[u] = usc[qc];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + 256 * u;
      if (q < m && !uv[u] && cv[u] > best) {
        best = cv[u];
        bi = q;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if ((t & 63) == 0) {
    sv[t >> 6] = best;
    ired[t >> 6] = bi;
  }
  __syncthreads();
  double cmax = sv[0];
  int P = ired[0];
  for (int w = 1; w < 4; ++w)
    if (sv[w] > cmax || (sv[w] == cmax && ired[w] < P)) {
      cmax = sv[w];
      P = ired[w];
    }
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
  // Householder vector of column P below row j (beta = -sign(x0) ||x||),
  // v = [1; x[1:] / (x0 - beta)].  The other columns take, in the same pass,
  // e = x[1:]^T a[j+1:], so that v^T a = a[j] + e / (x0 - beta).
  const double* ap = A + (int64_t)P * lda;
  double* ac = A + (int64_t)c * lda;
  const bool piv_col = c == P;
  const double x0 = ap[j];
  const double acj = piv_col ? 0.0 : ac[j];
  // (rounds of U16 rows per thread, loads from clamped indices all issued
  // before the first is used)
  constexpr int U16 = 16;
  double s2 = 0, e = 0;
  for (int64_t i0 = j + t; i0 < rows; i0 += 256 * U16) {
    double xv[U16], av[U16];
#pragma unroll
    for (int u = 0; u < U16; ++u) {
      const int64_t i = i0 + 256 * u, ic = i < rows ? i : j;
      xv[u] = ap[ic];
      av[u] = piv_col ? 0.0 : ac[ic];
    }
#pragma unroll
    for (int u = 0; u < U16; ++u) {
      const int64_t i = i0 + 256 * u;
      if (i < rows) {
        s2 += xv[u] * xv[u];
        if (i > j) e += xv[u] * av[u];
      }
    }
  }
  block_sum256x2(s2, e, red);
  const double nrm = sqrt(s2);
  const double beta = x0 >= 0 ? -nrm : nrm;
  const double tj = (beta - x0) / beta;
  const double scal = 1.0 / (x0 - beta);
  // (loops below load eight of the thread's rows before storing any: the
  // compiler cannot tell the columns apart, so a load after a store would
  // wait for it)
  constexpr int U8 = 8;
  if (piv_col) {
    double* v = V + (int64_t)j * ldv;
    for (int64_t i0 = t; i0 < rows; i0 += 256 * U8) {
      double xv[U8];
#pragma unroll
      for (int u = 0; u < U8; ++u) {
        const int64_t i = i0 + 256 * u;
        xv[u] = (i < rows && i > j) ? ap[i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U8; ++u) {
        const int64_t i = i0 + 256 * u;
        if (i < rows) v[i] = (i < j) ? 0.0 : (i == j ? 1.0 : xv[u] * scal);
      }
    }
    if (t == 0) {
      piv[j] = P;
      tau[j] = tj;
      cnn[c] = 0.0;
      usn[c] = 1;
    }
    return;
  }
  const double d = acj + scal * e;
  const double f = tj * d;
  double s3 = 0;
  for (int64_t i0 = j + t; i0 < rows; i0 += 256 * U8) {
    double av[U8], pv[U8];
#pragma unroll
    for (int u = 0; u < U8; ++u) {
      const int64_t i = i0 + 256 * u;
      const bool ok = i < rows;
      av[u] = ok ? ac[i] : 0.0;
      pv[u] = ok ? ap[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U8; ++u) {
      const int64_t i = i0 + 256 * u;
      if (i < rows) {
        const double nv = av[u] - f * (i == j ? 1.0 : pv[u] * scal);
        ac[i] = nv;
        if (i > j) s3 += nv * nv;
      }
    }
  }
  s3 = block_sum256(s3, red);
  if (t == 0) {
    cnn[c] = sqrt(s3);
    usn[c] = 0;
  }
}

__global__ void k_hqr_finish_rank(int* rank, int steps) {
  if (*rank < 0) *rank = steps;
}

// Column c of Q = H_0 H_1 .. H_c e_c, c < rank.
// Q = H_0 .. H_{r-1} [I_r; 0] (rows x r, ld ldq) from the reflectors in V
// (column j zero above row j, 1 at row j) and tau: blocks of WY_NB
// reflectors, last block first, Q <- Q - V_k T_k (V_k^T Q), where the rows
// above the block's first reflector are untouched.
static void form_q(hipStream_t s, OrthWork& w, int64_t rows, int r, double* Q, int64_t ldq) {
  DMat<double> Qm{Q, nullptr, ldq, 0};
  fill<double>(s, Qm, rows, r, 1, 0.0);
  pad_identity<double>(s, Qm, 0, r, 1);
  w.wg.alloc(sizeof(double) * WY_NB * WY_NB);
  w.wt.alloc(sizeof(double) * WY_NB * WY_NB);
  w.w1.alloc(sizeof(double) * WY_NB * (int64_t)r);
  w.w2.alloc(sizeof(double) * WY_NB * (int64_t)r);
  DMat<double> Gm{w.wg.as<double>(), nullptr, WY_NB, 0}, Tm{w.wt.as<double>(), nullptr, WY_NB, 0};
  DMat<double> W1m{w.w1.as<double>(), nullptr, WY_NB, 0}, W2m{w.w2.as<double>(), nullptr, WY_NB, 0};
  for (int64_t k0 = ((int64_t)(r - 1) / WY_NB) * WY_NB; k0 >= 0; k0 -= WY_NB) {
    const int nbp = (int)std::min<int64_t>(WY_NB, r - k0);
    const int64_t m = rows - k0;
    DMat<double> Vk{w.V.as<double>() + k0 + k0 * rows, nullptr, rows, 0};
    DMat<double> Qk = Qm.sub(k0, 0);
    fill<double>(s, Gm, WY_NB, WY_NB, 1, 0.0);
    gemm<double>(s, true, false, nbp, nbp, m, 1.0, Vk, Vk, 0.0, Gm, 1);
    wy_triangle(s, w.wg.as<double>(), w.tau.as<double>(), 0, k0, nbp, w.wt.as<double>(), 1);
    gemm<double>(s, true, false, nbp, r, m, 1.0, Vk, Qk, 0.0, W1m, 1);
    gemm<double>(s, false, false, nbp, r, nbp, 1.0, Tm, W1m, 0.0, W2m, 1);
    gemm<double>(s, false, false, m, r, nbp, -1.0, Vk, W2m, 1.0, Qk, 1);
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
  int r = 0;
  RFD_HIP(hipMemcpyAsync(&r, w.rank.as<int>(), sizeof(int), hipMemcpyDeviceToHost, s));
  RFD_HIP(hipStreamSynchronize(s));
  if (r < 0 || r > steps) throw Error(ST_EDEVICE, "orth_block: rank out of range");
  if (r > 0) form_q(s, w, rows, r, Qout, ldq);
  RFD_HIP(hipStreamSynchronize(s));
  return r;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pair_dots(const double* A, int64_t lda, const double* B,
                                                  int64_t ldb, int64_t rows, double* out) {
  __shared__ double red[8];
  const int j = blockIdx.x;
  const double* a = A + (int64_t)j * lda;
  const double* b = B + (int64_t)j * ldb;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) acc += a[i] * b[i];
  acc = block_sum256(acc, red);
  if (threadIdx.x == 0) out[j] = acc;
}

void col_dots(hipStream_t s, const double* A, int64_t lda, const double* B, int64_t ldb,
              int64_t rows, int cols, double* out) {
  if (cols <= 0) return;
  k_pair_dots<<<cols, 256, 0, s>>>(A, lda, B, ldb, rows, out);
  RFD_CHECK_LAUNCH();
}

}  // namespace rfd
