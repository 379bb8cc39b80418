// Dense FP64 symmetric eigensolver for selected eigenpairs (see eig.hpp).
//
// Tridiagonalization: one Householder reflector per step, two launches per
// step.  k_tri_a forms p = tau A v over the trailing block, one wavefront per
// column (A is kept fully symmetric, so column i of A is row i); k_tri_b
// applies the rank-2 update A -= v w^T + w v^T with w = p - (tau/2)(p^T v) v,
// each workgroup owning a block of columns and recomputing p^T v itself.  The
// reflector of step j stays unscaled in column j until step j+1 has read it
// and is scaled into v (implicit leading 1) by the first workgroup of step
// j+1 (or by the closing kernel).
#include <algorithm>
#include <cmath>

#include "eig.hpp"

namespace rfd {

constexpr double EPS = 2.220446049250313e-16;
constexpr double SAFMIN = 2.2250738585072014e-308;

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double block_sum256(double v, double* red) {
  const int t = threadIdx.x;
  v = wave_sum(v);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double r = 0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) r += red[i];
  __syncthreads();
  return r;
}

void TriWork::reserve(int64_t n, int batch) {
  const int64_t need = n * (int64_t)batch;
  if (need <= cap) return;
  cap = need;
  d.alloc(sizeof(double) * need);
  e.alloc(sizeof(double) * need);
  tau.alloc(sizeof(double) * need);
  scl.alloc(sizeof(double) * need);
  pvec.alloc(sizeof(double) * need);
}

// p[i] = tau * sum_c A[c, i] v[c], i, c in [j+1, n); v[j+1] = 1, v[c] = A[c, j] * scale.
__global__ __launch_bounds__(256) void k_tri_a(DMat<double> A, int64_t n, int64_t j, double* dv,
                                               double* ev, double* tauv, double* sclv, double* pv) {
  __shared__ double red[8];
  __shared__ double hh[4];
  const int b = blockIdx.y;
  DMat<double> a = A.item(b);
  const int t = threadIdx.x;
  // Householder data of column j (every workgroup computes it)
  double s2 = 0;
  for (int64_t i = j + 2 + t; i < n; i += blockDim.x) {
    const double x = a.re[i + j * a.ld];
    s2 += x * x;
  }
  s2 = block_sum256(s2, red);
  if (t == 0) {
    const double alpha = a.re[(j + 1) + j * a.ld];
    double tau = 0, beta = alpha, scale = 0;
    if (s2 > 0) {
      const double nrm = sqrt(alpha * alpha + s2);
      beta = alpha >= 0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    hh[0] = tau;
    hh[1] = beta;
    hh[2] = scale;
  }
  __syncthreads();
  const double tau = hh[0], scale = hh[2];
  if (blockIdx.x == 0 && t == 0) {
    dv[b * n + j] = a.re[j + j * a.ld];
    ev[b * n + j] = hh[1];
    tauv[b * n + j] = tau;
    sclv[b * n + j] = scale;
  }
  // the previous step's reflector: scale its column into v (nobody reads it now)
  if (blockIdx.x == 0 && j >= 1) {
    const double sp = sclv[b * n + j - 1];
    for (int64_t i = j + 1 + t; i < n; i += blockDim.x) a.re[i + (j - 1) * a.ld] *= sp;
  }
  // one wavefront per column i
  const int lane = t & 63, wv = t >> 6;
  const int64_t i = j + 1 + (int64_t)blockIdx.x * 4 + wv;
  if (i >= n) return;
  double acc = 0;
  const double* col = a.re + i * a.ld;
  const double* vj = a.re + j * a.ld;
  for (int64_t c = j + 1 + lane; c < n; c += 64) {
    const double v = (c == j + 1) ? 1.0 : vj[c] * scale;
    acc += col[c] * v;
  }
  acc = wave_sum(acc);
  if (lane == 0) pv[b * n + i] = tau * acc;
}

// A[r, c] -= v[r] w[c] + w[r] v[c] for r, c in [j+1, n); columns in blocks of 8.
__global__ __launch_bounds__(256) void k_tri_b(DMat<double> A, int64_t n, int64_t j,
                                               const double* tauv, const double* sclv,
                                               const double* pv) {
  __shared__ double red[8];
  const int b = blockIdx.y;
  DMat<double> a = A.item(b);
  const int t = threadIdx.x;
  const double tau = tauv[b * n + j], scale = sclv[b * n + j];
  if (tau == 0.0) return;
  const double* vj = a.re + j * a.ld;
  const double* p = pv + b * n;
  double dot = 0;
  for (int64_t c = j + 1 + t; c < n; c += blockDim.x) dot += p[c] * ((c == j + 1) ? 1.0 : vj[c] * scale);
  dot = block_sum256(dot, red);
  const double h = 0.5 * tau * dot;
  const int64_t c0 = j + 1 + (int64_t)blockIdx.x * 8;
  for (int64_t c = c0; c < c0 + 8 && c < n; ++c) {
    const double vc = (c == j + 1) ? 1.0 : vj[c] * scale;
    const double wc = p[c] - h * vc;
    double* col = a.re + c * a.ld;
    for (int64_t r = j + 1 + t; r < n; r += blockDim.x) {
      const double vr = (r == j + 1) ? 1.0 : vj[r] * scale;
      const double wr = p[r] - h * vr;
      col[r] -= vr * wc + wr * vc;
    }
  }
}

__global__ void k_tri_fin(DMat<double> A, int64_t n, double* dv, double* ev, double* sclv) {
  const int b = blockIdx.x;
  DMat<double> a = A.item(b);
  const int t = threadIdx.x;
  if (n >= 3) {
    const int64_t j = n - 3;
    const double sp = sclv[b * n + j];
    for (int64_t i = j + 2 + t; i < n; i += blockDim.x) a.re[i + j * a.ld] *= sp;
  }
  if (t == 0) {
    if (n >= 2) {
      dv[b * n + n - 2] = a.re[(n - 2) + (n - 2) * a.ld];
      ev[b * n + n - 2] = a.re[(n - 1) + (n - 2) * a.ld];
    }
    dv[b * n + n - 1] = a.re[(n - 1) + (n - 1) * a.ld];
    ev[b * n + n - 1] = 0.0;
  }
}

void sy_tridiag(hipStream_t s, DMat<double> A, int64_t n, int batch, TriWork& w) {
  w.reserve(n, batch);
  for (int64_t j = 0; j + 2 < n; ++j) {
    const int64_t L = n - j - 1;
    dim3 ga((unsigned)((L + 3) / 4), batch);
    k_tri_a<<<ga, 256, 0, s>>>(A, n, j, w.d.as<double>(), w.e.as<double>(), w.tau.as<double>(),
                               w.scl.as<double>(), w.pvec.as<double>());
    RFD_CHECK_LAUNCH();
    dim3 gb((unsigned)((L + 7) / 8), batch);
    k_tri_b<<<gb, 256, 0, s>>>(A, n, j, w.tau.as<double>(), w.scl.as<double>(),
                               w.pvec.as<double>());
    RFD_CHECK_LAUNCH();
  }
  k_tri_fin<<<batch, 256, 0, s>>>(A, n, w.d.as<double>(), w.e.as<double>(), w.scl.as<double>());
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Sturm counts and bisection.
// ---------------------------------------------------------------------------
__device__ inline int sturm(const double* d, const double* e, int64_t n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
  for (int64_t i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
  }
  return cnt;
}

__device__ inline double pivmin_of(const double* e, int64_t n) {
  double m = 1.0;
  for (int64_t i = 0; i + 1 < n; ++i) m = fmax(m, e[i] * e[i]);
  return SAFMIN * m / EPS;
}

__global__ void k_sturm(const double* dv, const double* ev, int64_t n, int batch, const double* x,
                        int nx, int* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch * nx) return;
  const int b = i / nx;
  const double* d = dv + (int64_t)b * n;
  const double* e = ev + (int64_t)b * n;
  cnt[i] = sturm(d, e, n, x[i], pivmin_of(e, n));
}

void sturm_counts(hipStream_t s, const TriWork& w, int64_t n, int batch, const double* x, int nx,
                  int* cnt) {
  k_sturm<<<grid1((int64_t)batch * nx), 256, 0, s>>>(w.d.as<double>(), w.e.as<double>(), n, batch,
                                                     x, nx, cnt);
  RFD_CHECK_LAUNCH();
}

__global__ void k_bisect(const double* dv, const double* ev, int64_t n, int batch, const int* lo,
                         const int* num, int maxnum, double* lam, int64_t ld_lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= maxnum || i >= num[b]) return;
  const double* d = dv + (int64_t)b * n;
  const double* e = ev + (int64_t)b * n;
  double gl = d[0], gu = d[0];
  for (int64_t r = 0; r < n; ++r) {
    const double off = (r > 0 ? fabs(e[r - 1]) : 0.0) + (r + 1 < n ? fabs(e[r]) : 0.0);
    gl = fmin(gl, d[r] - off);
    gu = fmax(gu, d[r] + off);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  gl -= 2.0 * EPS * tnorm * n + 1e-300;
  gu += 2.0 * EPS * tnorm * n + 1e-300;
  const double pivmin = pivmin_of(e, n);
  const int k = lo[b] + i;  // want the k-th smallest (0-based): count(x) <= k < count(y)
  double l = gl, u = gu;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (l + u);
    if (u - l <= 2.0 * EPS * fmax(fabs(l), fabs(u)) + 4.0 * pivmin) break;
    if (mid <= l || mid >= u) break;
    if (sturm(d, e, n, mid, pivmin) <= k) l = mid;
    else u = mid;
  }
  lam[(int64_t)b * ld_lam + i] = 0.5 * (l + u);
}

void bisect(hipStream_t s, const TriWork& w, int64_t n, int batch, const int* lo, const int* num,
            int maxnum, double* lam, int64_t ld_lam) {
  if (maxnum <= 0) return;
  dim3 g(grid1(maxnum, 64), batch);
  k_bisect<<<g, 64, 0, s>>>(w.d.as<double>(), w.e.as<double>(), n, batch, lo, num, maxnum, lam,
                            ld_lam);
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Inverse iteration: one thread per cluster head, members in order.
// ---------------------------------------------------------------------------
__device__ inline double hash_unit(uint64_t a, uint64_t b) {
  uint64_t x = a * 0x9E3779B97F4A7C15ull ^ (b + 0x632BE59BD9B4E019ull);
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

__global__ void k_invit(const double* dv, const double* ev, int64_t n, const double* lam,
                        const int* num, const int* clus, int64_t ld_lam, DMat<double> Y,
                        double* scratch) {
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i0 >= num[b] || i0 >= ld_lam) return;
  if (clus[(int64_t)b * ld_lam + i0] != i0) return;  // not a cluster head
  const double* d = dv + (int64_t)b * n;
  const double* e = ev + (int64_t)b * n;
  double* W = scratch + ((int64_t)b * ld_lam + i0) * 6 * n;
  double *dl = W, *dd = W + n, *du = W + 2 * n, *du2 = W + 3 * n, *x = W + 4 * n;
  int* ip = reinterpret_cast<int*>(W + 5 * n);
  DMat<double> y = Y.item(b);
  double tnorm = 0;
  for (int64_t r = 0; r < n; ++r)
    tnorm = fmax(tnorm, fabs(d[r]) + (r > 0 ? fabs(e[r - 1]) : 0.0) + (r + 1 < n ? fabs(e[r]) : 0.0));
  const double pert = 10.0 * EPS * fmax(tnorm, 1e-300);
  double prev = -INFINITY;
  for (int i = i0; i < num[b] && clus[(int64_t)b * ld_lam + i] == i0; ++i) {
    double lm = lam[(int64_t)b * ld_lam + i];
    if (lm - prev < pert) lm = prev + pert;
    prev = lm;
    // LU with partial pivoting of T - lm I (dgttrf)
    for (int64_t r = 0; r < n; ++r) dd[r] = d[r] - lm;
    for (int64_t r = 0; r + 1 < n; ++r) {
      dl[r] = e[r];
      du[r] = e[r];
    }
    for (int64_t r = 0; r + 2 < n; ++r) du2[r] = 0.0;
    for (int64_t r = 0; r + 1 < n; ++r) {
      if (fabs(dd[r]) >= fabs(dl[r])) {
        ip[r] = (int)r;
        const double f = (dd[r] != 0.0) ? dl[r] / dd[r] : 0.0;
        dl[r] = f;
        dd[r + 1] -= f * du[r];
      } else {
        ip[r] = (int)r + 1;
        const double f = dd[r] / dl[r];
        dd[r] = dl[r];
        dl[r] = f;
        const double tmp = du[r];
        du[r] = dd[r + 1];
        dd[r + 1] = tmp - f * dd[r + 1];
        if (r + 2 < n) {
          du2[r] = du[r + 1];
          du[r + 1] = -f * du[r + 1];
        }
      }
    }
    for (int64_t r = 0; r < n; ++r)
      if (fabs(dd[r]) < EPS * tnorm) dd[r] = (dd[r] < 0 ? -1.0 : 1.0) * EPS * fmax(tnorm, 1e-300);
    for (int64_t r = 0; r < n; ++r) x[r] = hash_unit((uint64_t)r + 1, (uint64_t)i + 7919ull * b);
    for (int it = 0; it < 4; ++it) {
      // solve L U x = P b in place
      for (int64_t r = 0; r + 1 < n; ++r) {
        if (ip[r] == r) {
          x[r + 1] -= dl[r] * x[r];
        } else {
          const double tmp = x[r];
          x[r] = x[r + 1];
          x[r + 1] = tmp - dl[r] * x[r];
        }
      }
      x[n - 1] /= dd[n - 1];
      if (n > 1) x[n - 2] = (x[n - 2] - du[n - 2] * x[n - 1]) / dd[n - 2];
      for (int64_t r = n - 3; r >= 0; --r) x[r] = (x[r] - du[r] * x[r + 1] - du2[r] * x[r + 2]) / dd[r];
      // orthogonalise against the previous members of the cluster (twice)
      for (int pass = 0; pass < 2; ++pass)
        for (int q = i0; q < i; ++q) {
          const double* yq = y.re + (int64_t)q * y.ld;
          double dt = 0;
          for (int64_t r = 0; r < n; ++r) dt += yq[r] * x[r];
          for (int64_t r = 0; r < n; ++r) x[r] -= dt * yq[r];
        }
      double nrm = 0;
      for (int64_t r = 0; r < n; ++r) nrm += x[r] * x[r];
      nrm = sqrt(nrm);
      const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
      for (int64_t r = 0; r < n; ++r) x[r] *= inv;
    }
    // sign convention: largest-magnitude component positive
    int64_t am = 0;
    for (int64_t r = 1; r < n; ++r)
      if (fabs(x[r]) > fabs(x[am])) am = r;
    const double sg = x[am] < 0 ? -1.0 : 1.0;
    double* yi = y.re + (int64_t)i * y.ld;
    for (int64_t r = 0; r < n; ++r) yi[r] = sg * x[r];
  }
}

void inverse_iteration(hipStream_t s, const TriWork& w, int64_t n, int batch, const double* lam,
                       const int* num, const int* clus, int64_t ld_lam, DMat<double> Y,
                       DevBuf& scratch) {
  if (ld_lam <= 0) return;
  scratch.alloc(sizeof(double) * 6 * n * ld_lam * (int64_t)batch);
  dim3 g(grid1(ld_lam, 64), batch);
  k_invit<<<g, 64, 0, s>>>(w.d.as<double>(), w.e.as<double>(), n, lam, num, clus, ld_lam, Y,
                           scratch.as<double>());
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Back-transformation: one workgroup per column of Y.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_backtr(DMat<double> A, const double* tauv, int64_t n,
                                                DMat<double> Y, const int* num) {
  __shared__ double red[8];
  const int c = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  if (c >= num[b]) return;
  DMat<double> a = A.item(b);
  double* y = Y.item(b).re + (int64_t)c * Y.ld;
  for (int64_t j = n - 3; j >= 0; --j) {
    const double tau = tauv[(int64_t)b * n + j];
    if (tau == 0.0) continue;
    const double* v = a.re + j * a.ld;
    double dt = 0;
    for (int64_t r = j + 1 + t; r < n; r += blockDim.x) dt += ((r == j + 1) ? 1.0 : v[r]) * y[r];
    dt = block_sum256(dt, red);
    const double f = tau * dt;
    for (int64_t r = j + 1 + t; r < n; r += blockDim.x) y[r] -= f * ((r == j + 1) ? 1.0 : v[r]);
    __syncthreads();
  }
}

void back_transform(hipStream_t s, DMat<double> A, const TriWork& w, int64_t n, int batch,
                    DMat<double> Y, const int* num, int maxcols) {
  if (maxcols <= 0) return;
  dim3 g(maxcols, batch);
  k_backtr<<<g, 256, 0, s>>>(A, w.tau.as<double>(), n, Y, num);
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Pivoted Cholesky (right-looking on the unselected index set, no physical
// swaps) and the inverse of the pivot-ordered factor.  One workgroup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_pchol(double* G, int64_t ldg, int64_t m, double tol,
                                                int* piv, int* rank, double* Lp, double* Linv,
                                                int64_t ldl, int* sel) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  __shared__ double d0;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int64_t i = t; i < m; i += nt) sel[i] = -1;
  double mx = 0;
  for (int64_t i = t; i < m; i += nt) mx = fmax(mx, G[i + i * ldg]);
  sv[t] = mx;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (t < w) sv[t] = fmax(sv[t], sv[t + w]);
    __syncthreads();
  }
  if (t == 0) d0 = sv[0];
  __syncthreads();
  const double thr = tol * d0;
  int r = 0;
  for (int64_t k = 0; k < m; ++k) {
    double best = -1;
    int bi = -1;
    for (int64_t i = t; i < m; i += nt)
      if (sel[i] < 0 && G[i + i * ldg] > best) { best = G[i + i * ldg]; bi = (int)i; }
    sv[t] = best;
    si[t] = bi;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (t < w && (sv[t + w] > sv[t] || (sv[t + w] == sv[t] && si[t + w] >= 0 &&
                                          (si[t] < 0 || si[t + w] < si[t])))) {
        sv[t] = sv[t + w];
        si[t] = si[t + w];
      }
      __syncthreads();
    }
    const int pk = si[0];
    const double dk = sv[0];
    __syncthreads();
    if (pk < 0 || !(dk > thr)) break;
    const double lkk = sqrt(dk);
    // column k of L (original indexing) into Lp[:, k]
    for (int64_t i = t; i < m; i += nt) {
      double v = 0;
      if (i == pk) v = lkk;
      else if (sel[i] < 0) v = G[i + (int64_t)pk * ldg] / lkk;
      Lp[i + k * ldl] = v;
    }
    __syncthreads();
    if (t == 0) {
      sel[pk] = (int)k;
      piv[k] = pk;
    }
    __syncthreads();
    // trailing update over unselected rows/cols
    for (int64_t e = t; e < m * m; e += nt) {
      const int64_t i = e % m, c = e / m;
      if (sel[i] < 0 && sel[c] < 0) G[i + c * ldg] -= Lp[i + k * ldl] * Lp[c + k * ldl];
    }
    __syncthreads();
    ++r;
  }
  if (t == 0) *rank = r;
  __syncthreads();
  // pivot-ordered L (r x r) back into G's leading block: L[a, b] = Lp[piv[a], b]
  for (int64_t e = t; e < (int64_t)r * r; e += nt) {
    const int64_t a = e % r, bcol = e / r;
    G[a + bcol * ldg] = (a >= bcol) ? Lp[piv[a] + bcol * ldl] : 0.0;
  }
  __syncthreads();
  // Linv: column c by one thread, forward substitution
  for (int64_t c = t; c < r; c += nt) {
    for (int64_t i = 0; i < r; ++i) {
      double v = 0;
      if (i == c) v = 1.0 / G[c + c * ldg];
      else if (i > c) {
        double sacc = 0;
        for (int64_t q = c; q < i; ++q) sacc += G[i + q * ldg] * Linv[q + c * ldl];
        v = -sacc / G[i + i * ldg];
      }
      Linv[i + c * ldl] = v;
    }
  }
}

void pivoted_cholesky(hipStream_t s, double* G, int64_t ldg, int64_t m, double tol, int* piv,
                      int* rank, double* Linv, int64_t ldl) {
  // scratch: Lp (m x m) and sel (m) right after Linv's m x m block
  static thread_local DevBuf scratch;
  scratch.alloc(sizeof(double) * (m * m + m));
  double* Lp = scratch.as<double>();
  int* sel = reinterpret_cast<int*>(Lp + m * m);
  k_pchol<<<1, 1024, 0, s>>>(G, ldg, m, tol, piv, rank, Lp, Linv, ldl, sel);
  RFD_CHECK_LAUNCH();
}

}  // namespace rfd
