// Interior part and Rayleigh-Ritz (Sec. 4, Sec. 5 / Alg. 5.1 steps 3, 6-8).
//
//  interior_basis():  V_j = eigenvectors of (B_j, M_Bj) closest to sigma
//                     (M_Bj diagonal: eigenvectors of M^{-1/2} B M^{-1/2},
//                     batched over subdomains), M_Bj-orthonormal.
//  factor_bsigma():   LU with partial pivoting of B_sigma^(j) = B_j - sigma M_Bj.
//  solve_interior():  resolvent levels of eqs. (5.2)-(5.4), each made
//                     M_Bj-orthogonal to V_j (deflated recurrence), then an
//                     M-orthonormal basis of range(Z) (eq. (5.5)) built level by
//                     level with pivoted Cholesky QR.
//  rayleigh_ritz():   H = Z^T A Z on that basis, eigenpairs with theta in
//                     [alpha, beta], Ritz vectors in the original numbering and
//                     their residuals.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "dense.hpp"
#include "eig.hpp"
#include "engine_impl.hpp"

namespace rfd {

__device__ inline double bsum(double v, double* red) {
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

// diag(M_B^(j)) and 1/sqrt of it, per subdomain row (p x D).
__global__ void k_mdiag(int64_t D, const int32_t* dj, DevPairCsr B, double* md, double* mis) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= D) return;
  double m = 1.0;
  if (r < dj[j]) {
    const int64_t* ptr = B.ptr + B.roff[j];
    for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e)
      if (B.idx[e] == r) m = B.m[e];
  }
  md[(int64_t)j * D + r] = m;
  mis[(int64_t)j * D + r] = 1.0 / sqrt(m);
}

// C_j = M^{-1/2} B_j M^{-1/2} (dense, zero on entry), padding diagonal = big.
__global__ void k_expand_scaled(DMat<double> C, int64_t D, const int32_t* dj, DevPairCsr B,
                                const double* mis, double big) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= D) return;
  DMat<double> c = C.item(j);
  if (r >= dj[j]) {
    c.re[r + r * c.ld] = big;
    return;
  }
  const double* mj = mis + (int64_t)j * D;
  const int64_t* ptr = B.ptr + B.roff[j];
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const int64_t q = B.idx[e];
    c.re[r + q * c.ld] = B.a[e] * mj[r] * mj[q];
  }
}

// X_j[r, c] *= vec[j * D + r] for r < rows, c < cols.
__global__ void k_scale_rows(DMat<double> X, int64_t rows, int64_t cols, const double* vec,
                             int64_t D) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e % rows, c = e / rows;
  DMat<double> x = X.item(blockIdx.y);
  x.re[r + c * x.ld] *= vec[(int64_t)blockIdx.y * D + r];
}

// The elementwise kernels over tall column blocks below give each thread one
// row and CG consecutive columns (grid: row blocks x column groups [x items]),
// so that per-row data is read once and no index is split by division.
constexpr int CG = 4;

static unsigned col_groups(int64_t cols) {
  const int64_t g = (cols + CG - 1) / CG;
  if (g > 65535) throw Error(ST_EINVAL, "too many columns for one launch");
  return (unsigned)std::max<int64_t>(g, 1);
}

// Y_j[r, c] = vec[j * D + r] * X_j[r, c]  (items over the z grid dimension)
__global__ void k_scaled_copy(DMat<double> X, DMat<double> Y, int64_t rows, int64_t cols,
                              const double* vec, int64_t D) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t c0 = (int64_t)blockIdx.y * CG;
  DMat<double> x = X.item(blockIdx.z), y = Y.item(blockIdx.z);
  const double f = vec[(int64_t)blockIdx.z * D + r];
  double v[CG];
#pragma unroll
  for (int u = 0; u < CG; ++u) v[u] = c0 + u < cols ? x.re[r + (c0 + u) * x.ld] : 0.0;
#pragma unroll
  for (int u = 0; u < CG; ++u)
    if (c0 + u < cols) y.re[r + (c0 + u) * y.ld] = f * v[u];
}

// out[c] = || column c of the level over all subdomains ||_{M_B}, one workgroup per column.
__global__ void k_level_colnorm(DMat<double> X, int p, const int32_t* dj, const double* md,
                                int64_t D, double* out) {
  __shared__ double red[256];
  const int64_t c = blockIdx.x;
  double acc = 0;
  for (int j = 0; j < p; ++j) {
    DMat<double> x = X.item(j);
    const int64_t dr = dj[j];
    const double* xc = x.re + c * x.ld;
    const double* mj = md + (int64_t)j * D;
    for (int64_t r0 = threadIdx.x; r0 < dr; r0 += 4 * 256) {
      double v[4], m[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t r = r0 + 256 * u;
        v[u] = r < dr ? xc[r] : 0.0;
        m[u] = r < dr ? mj[r] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += m[u] * v[u] * v[u];
    }
  }
  acc = bsum(acc, red);
  if (threadIdx.x == 0) out[c] = sqrt(acc);
}

// Zeroes column c of every subdomain's level when post[c] <= thr * pre[c]:
// a level that lies inside span(V_j) up to rounding carries no direction.
__global__ void k_level_drop(DMat<double> X, int64_t D, int64_t cols, const double* pre,
                             const double* post, double thr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  const int64_t c0 = (int64_t)blockIdx.y * CG;
  DMat<double> x = X.item(blockIdx.z);
#pragma unroll
  for (int u = 0; u < CG; ++u) {
    const int64_t c = c0 + u;
    if (c < cols && !(post[c] > thr * pre[c])) x.re[r + c * x.ld] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// A non-diagonal M_Bj.  The blocks are brought to standard form through the
// factorization M_Bj = L_j U_j without pivoting (M_Bj is symmetric positive
// definite, so U_j = diag(u) L_j^T and G_j = L_j diag(u)^{1/2} is its
// Cholesky factor): C_j = G_j^{-1} B_j G_j^{-T} = diag(u)^{-1/2} L_j^{-1} B_j
// L_j^{-T} diag(u)^{-1/2}, and eigenvectors Y of C_j give the M_Bj-orthonormal
// eigenvectors V = G_j^{-T} Y = U_j^{-1} diag(u)^{1/2} Y of (B_j, M_Bj).
// ---------------------------------------------------------------------------

// Dense image of every subdomain block (A values when which == 0, M values
// otherwise; C zero on entry), diagonal `pad` on the padding rows.
__global__ void k_expand_block(DMat<double> C, int64_t D, const int32_t* dj, DevPairCsr B,
                               int which, double pad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= D) return;
  DMat<double> c = C.item(j);
  if (r >= dj[j]) {
    c.re[r + r * c.ld] = pad;
    return;
  }
  const int64_t* ptr = B.ptr + B.roff[j];
  const double* v = which ? B.m : B.a;
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) c.re[r + (int64_t)B.idx[e] * c.ld] = v[e];
}

// sq = sqrt(u_rr), isq = 1 / sqrt(u_rr) from the diagonal of the factors of
// M_Bj (p x D; 1 on the padding rows).  A pivot that is not positive (M_Bj not
// positive definite) sets bit 1 of *flags.
__global__ void k_lu_diag(DMat<double> LU, int64_t D, const int32_t* dj, double* sq, double* isq,
                          unsigned* flags) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= D) return;
  DMat<double> f = LU.item(j);
  double u = r < dj[j] ? f.re[r + r * f.ld] : 1.0;
  if (!(u > 0.0) || !isfinite(u)) {
    atomicOr(flags, 1u);
    u = 1.0;
  }
  sq[(int64_t)j * D + r] = sqrt(u);
  isq[(int64_t)j * D + r] = 1.0 / sqrt(u);
}

// 32 x 32 LDS tiles over the leading D x D block of every item (grid D/32 x
// D/32 x items, 256 threads).  sym == 0: Y = X^T.  sym == 1: Y = (X + X^T) / 2
// scaled by g[r] g[q] over the active d_j x d_j part (g: p x D), zero
// elsewhere.  Both reads and the write run along columns.
constexpr int TT = 32;
__global__ __launch_bounds__(256) void k_tile_transpose(DMat<double> X, DMat<double> Y, int64_t D,
                                                        const int32_t* dj, const double* g,
                                                        int sym) {
  __shared__ double t[TT][TT + 1];
  const int j = blockIdx.z;
  DMat<double> x = X.item(j), y = Y.item(j);
  const int64_t r0 = (int64_t)blockIdx.x * TT, q0 = (int64_t)blockIdx.y * TT;
  const int tx = threadIdx.x & (TT - 1), ty = threadIdx.x / TT;
  // t[c][a] = X[q0 + a, r0 + c]
  for (int c = ty; c < TT; c += 256 / TT) {
    const int64_t q = q0 + tx, r = r0 + c;
    t[c][tx] = (q < D && r < D) ? x.re[q + r * x.ld] : 0.0;
  }
  __syncthreads();
  const int64_t dact = dj ? dj[j] : D;
  for (int c = ty; c < TT; c += 256 / TT) {
    const int64_t r = r0 + tx, q = q0 + c;
    if (r >= D || q >= D) continue;
    const double tv = t[tx][c];  // X[q, r]
    if (!sym) {
      y.re[r + q * y.ld] = tv;
    } else {
      const bool act = r < dact && q < dact;
      const double* gj = g + (int64_t)j * D;
      y.re[r + q * y.ld] = act ? 0.5 * (x.re[r + q * x.ld] + tv) * gj[r] * gj[q] : 0.0;
    }
  }
}

// *out = max over the active rows of every item of sum_q |C_j[r, q]|
// (||C_j||_inf, a bound on its spectral radius), bitwise atomic max.
__global__ void k_row_absmax(DMat<double> C, int64_t D, const int32_t* dj,
                             unsigned long long* out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int64_t d = dj[j];
  if (r >= d) return;
  DMat<double> c = C.item(j);
  double acc = 0;
  for (int64_t q = 0; q < d; ++q) acc += fabs(c.re[r + q * c.ld]);
  atomicMax(out, (unsigned long long)__double_as_longlong(acc));
}

// C_j[r, r] = v on the padding rows d_j <= r < D.
__global__ void k_pad_diag(DMat<double> C, int64_t D, const int32_t* dj, double v) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= D || r < dj[j]) return;
  DMat<double> c = C.item(j);
  c.re[r + r * c.ld] = v;
}

// Y_j = M_Bj X_j on the active rows, zero on the padding rows (CG columns
// per thread, subdomains over grid z), from the M values of the subdomain
// CSR blocks.
__global__ void k_block_mb(DMat<double> X, DMat<double> Y, int64_t D, int64_t cols,
                           const int32_t* dj, DevPairCsr B) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  const int j = blockIdx.z;
  const int64_t c0 = (int64_t)blockIdx.y * CG;
  DMat<double> x = X.item(j), y = Y.item(j);
  double acc[CG] = {};
  if (r < dj[j]) {
    const int64_t* ptr = B.ptr + B.roff[j];
    for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
      const double m = B.m[e];
      const double* xc = x.re + (int64_t)B.idx[e] + c0 * x.ld;
#pragma unroll
      for (int u = 0; u < CG; ++u)
        if (c0 + u < cols) acc[u] += m * xc[u * x.ld];
    }
  }
#pragma unroll
  for (int u = 0; u < CG; ++u)
    if (c0 + u < cols) y.re[r + (c0 + u) * y.ld] = acc[u];
}

// out[c] = sqrt(sum_j x_j^T (M_Bj x_j)) for column c of a level, from the
// level X and MX = M_B X (one workgroup per column).
__global__ void k_level_coldot(DMat<double> X, DMat<double> MX, int p, const int32_t* dj,
                               double* out) {
  __shared__ double red[256];
  const int64_t c = blockIdx.x;
  double acc = 0;
  for (int j = 0; j < p; ++j) {
    DMat<double> x = X.item(j), mx = MX.item(j);
    const int64_t dr = dj[j];
    const double* xc = x.re + c * x.ld;
    const double* mc = mx.re + c * mx.ld;
    for (int64_t r = threadIdx.x; r < dr; r += 256) acc += xc[r] * mc[r];
  }
  acc = bsum(acc, red);
  if (threadIdx.x == 0) out[c] = sqrt(fmax(acc, 0.0));
}

// rhs_j[r, c] = ((ca Ehat_j + cm Mhat_E^(j)) Q[adj_j, :])[r, c].  With ca = -1,
// cm = sigma: Phi of eq. (5.2), negated so that the first level carries the
// sign of eq. (5.5); with ca = 0, cm = 1: Psi = Mhat_E Q of eq. (5.3).
__global__ void k_gather_phi(DMat<double> R, int64_t D, int64_t cols_pad, const int32_t* dj,
                             DevPairCsr E, double ca, double cm, const double* Q, int64_t ldq,
                             int mu, const int32_t* adj, int64_t SJ) {
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (e0 >= D * cols_pad) return;
  const int64_t r = e0 % D, c = e0 / D;
  DMat<double> x = R.item(j);
  double v = 0;
  if (r < dj[j] && c < mu) {
    const int64_t* ptr = E.ptr + E.roff[j];
    for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e)
      v += (ca * E.a[e] + cm * E.m[e]) * Q[adj[(int64_t)j * SJ + E.idx[e]] + c * ldq];
  }
  x.re[r + c * x.ld] = v;
}

// Zt[ioff[j] + r, koff[j] + c] = V_j[r, c]
__global__ void k_scatter_v(double* Z, int64_t ldz, DMat<double> V, const int32_t* ioff,
                            const int32_t* koff, const int32_t* kap, const int32_t* dj,
                            int64_t rows) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int64_t kj = kap[j];
  if (e >= rows * kj) return;
  const int64_t r = e % rows, c = e / rows;
  if (r >= dj[j]) return;
  DMat<double> v = V.item(j);
  Z[(ioff[j] + r) + (koff[j] + c) * ldz] = v.re[r + c * v.ld];
}

// level t of Z in the reordered numbering: interior rows from Lev, interface
// rows Q (t == 0) or 0.  The subdomain of a row is found by bisection over
// the interior offsets, held in shared memory when there are at most
// BL_MAXP + 1 of them.
constexpr int BL_MAXP = 4095;
__global__ void k_build_level(double* L, int64_t ldl, DMat<double> Lev, int t, int64_t MUP,
                              const int32_t* ioff, int p, int64_t n_int, int64_t n, const double* Q,
                              int64_t ldq, int mu) {
  __shared__ int32_t so[BL_MAXP + 1];
  const bool in_lds = p <= BL_MAXP;
  if (in_lds)
    for (int k = threadIdx.x; k <= p; k += blockDim.x) so[k] = ioff[k];
  __syncthreads();
  const int32_t* off = in_lds ? so : ioff;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t c0 = (int64_t)blockIdx.y * CG;
  // the source of row i: its subdomain's level rows, Q's row, or nothing
  const double* src = nullptr;
  int64_t lds = 0;
  if (i < n_int) {
    int lo = 0, hi = p;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (off[mid] <= i) lo = mid;
      else hi = mid;
    }
    DMat<double> x = Lev.item(lo);
    src = x.re + (i - off[lo]) + (t * MUP + c0) * x.ld;
    lds = x.ld;
  } else if (t == 0) {
    src = Q + (i - n_int) + c0 * ldq;
    lds = ldq;
  }
  double v[CG];
#pragma unroll
  for (int u = 0; u < CG; ++u) v[u] = (src && c0 + u < mu) ? src[u * lds] : 0.0;
#pragma unroll
  for (int u = 0; u < CG; ++u)
    if (c0 + u < mu) L[i + (c0 + u) * ldl] = v[u];
}

// Y = op X with op a CSR matrix (n x n) (Y, X dense n x cols).  One thread
// per row and group of four columns: the row's entries are read once for the
// four columns, eight at a time with all their loads in flight before the
// gathers of X that depend on them; the y grid dimension runs over column
// groups.
__global__ void k_csr_mm(const int64_t* ptr, const int32_t* idx, const double* val, int64_t n,
                         const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t cols) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t c0 = (int64_t)blockIdx.y * 4;
  const int nc = (int)((cols - c0) < 4 ? (cols - c0) : 4);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t q0 = ptr[r], q1 = ptr[r + 1];
  const double* xc = X + c0 * ldx;
  for (int64_t qb = q0; qb < q1; qb += 8) {
    int32_t ix[8];
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool ok = qb + k < q1;
      ix[k] = ok ? idx[qb + k] : 0;
      v[k] = ok ? val[qb + k] : 0.0;
    }
    double xv[8][4];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        xv[k][u] = (qb + k < q1 && u < nc) ? xc[ix[k] + u * ldx] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += v[k] * xv[k][u];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (u < nc) Y[r + (c0 + u) * ldy] = acc[u];
}

static void csr_mm(hipStream_t s, const DevBuf& ptr, const DevBuf& idx, const DevBuf& val,
                   int64_t n, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t cols) {
  if (cols <= 0 || n <= 0) return;
  for (int64_t c = 0; c < cols; c += 4 * 65535) {
    const int64_t cc = std::min<int64_t>(cols - c, 4 * 65535);
    dim3 g(grid1(n), (unsigned)((cc + 3) / 4));
    k_csr_mm<<<g, 256, 0, s>>>(ptr.as<int64_t>(), idx.as<int32_t>(), val.as<double>(), n,
                               X + c * ldx, ldx, Y + c * ldy, ldy, cc);
    RFD_CHECK_LAUNCH();
  }
}

// out[c] = sqrt(x_c^T Y_c) (M-norms with Y = M X), one workgroup of 256 per
// column, eight loads of each operand in flight per thread.
__global__ void k_col_dots(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n,
                           double* out) {
  __shared__ double red[256];
  const int64_t c = blockIdx.x;
  const double* x = X + c * ldx;
  const double* y = Y + c * ldy;
  double acc = 0;
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += 8 * 256) {
    double xv[8], yv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + 256 * u;
      xv[u] = i < n ? x[i] : 0.0;
      yv[u] = i < n ? y[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += xv[u] * yv[u];
  }
  acc = bsum(acc, red);
  if (threadIdx.x == 0) out[c] = sqrt(fmax(acc, 0.0));
}

// The same M-norms for a diagonal M = diag(dg), from X alone:
// out[c] = sqrt(sum_i x_i (dg_i x_i)).
__global__ void k_col_mnorm(const double* dg, const double* X, int64_t ldx, int64_t n,
                            double* out) {
  __shared__ double red[256];
  const int64_t c = blockIdx.x;
  const double* x = X + c * ldx;
  double acc = 0;
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += 8 * 256) {
    double xv[8], dv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + 256 * u;
      xv[u] = i < n ? x[i] : 0.0;
      dv[u] = i < n ? dg[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += xv[u] * (dv[u] * xv[u]);
  }
  acc = bsum(acc, red);
  if (threadIdx.x == 0) out[c] = sqrt(fmax(acc, 0.0));
}

// X_c *= 1 / nrm[c], or zero the column when nrm[c] <= floor_rel * ref[c].
__global__ void k_col_normalize(double* X, int64_t ldx, int64_t n, const double* nrm,
                                const double* ref, double floor_rel) {
  const int64_t c = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = nrm[c];
  const bool drop = !(v > 0) || (ref && v <= floor_rel * ref[c]);
  X[i + c * ldx] = drop ? 0.0 : X[i + c * ldx] / v;
}

// Y[:, c] = X[:, piv[c]]
__global__ void k_gather_cols(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t n,
                              const int* piv, const int* rank) {
  const int64_t c = blockIdx.y;
  if (c >= *rank) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Y[i + c * ldy] = X[i + (int64_t)piv[c] * ldx];
}

// H[j, i] = H[i, j] for i > j (the upper triangle mirrors the lower one)
__global__ void k_mirror_lower(double* H, int64_t ld, int64_t k) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const int64_t i = e % k, j = e / k;
  if (i <= j) return;
  H[j + i * ld] = H[i + j * ld];
}

// X[order[i], c] = Xr[i, c]
__global__ void k_unpermute(const double* Xr, int64_t ldr, const int32_t* order, int64_t n,
                            double* X, int64_t ldx, int64_t cols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * cols) return;
  const int64_t i = e % n, c = e / n;
  X[order[i] + c * ldx] = Xr[i + c * ldr];
}

// resid[c] = ||AX_c - theta_c MX_c|| / (normA ||X_c||)
__global__ void k_resid(const double* AX, const double* MX, const double* X, int64_t ld, int64_t n,
                        const double* theta, double normA, double* out) {
  __shared__ double red[256];
  const int64_t c = blockIdx.x;
  const double th = theta[c];
  double r2 = 0, x2 = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double rv = AX[i + c * ld] - th * MX[i + c * ld];
    r2 += rv * rv;
    x2 += X[i + c * ld] * X[i + c * ld];
  }
  r2 = bsum(r2, red);
  x2 = bsum(x2, red);
  if (threadIdx.x == 0) out[c] = sqrt(r2) / (normA * sqrt(x2));
}

// ---------------------------------------------------------------------------
// Stream-ordered upload (the host vector may be released on return).
template <typename T>
static void upload_v(hipStream_t st, DevBuf& b, const std::vector<T>& v) {
  b.alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (!v.empty()) {
    RFD_HIP(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
    RFD_HIP(hipStreamSynchronize(st));
  }
}

template <typename T>
static std::vector<T> download(hipStream_t s, const void* p, size_t n) {
  std::vector<T> v(n);
  if (n) {
    RFD_HIP(hipMemcpyAsync(v.data(), p, sizeof(T) * n, hipMemcpyDeviceToHost, s));
    RFD_HIP(hipStreamSynchronize(s));
  }
  return v;
}

void EngineImpl::ensure_reordered(hipStream_t st) {
  if (Arptr.p) return;
  std::vector<int32_t> ord;
  for (int j = 0; j < p; ++j) ord.insert(ord.end(), P->interior[j].begin(), P->interior[j].end());
  ord.insert(ord.end(), P->iface.begin(), P->iface.end());
  std::vector<int32_t> pos(n);
  for (int64_t i = 0; i < n; ++i) pos[ord[i]] = (int32_t)i;
  for (int w = 0; w < 2; ++w) {
    const Csr& X = w == 0 ? *A : *M;
    std::vector<int64_t> ptr(1, 0);
    std::vector<int32_t> idx;
    std::vector<double> val;
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = 0; i < n; ++i) {
      const int32_t g = ord[i];
      row.clear();
      for (int64_t e = X.ptr[g]; e < X.ptr[g + 1]; ++e) row.emplace_back(pos[X.idx[e]], X.val[e]);
      std::sort(row.begin(), row.end());
      for (auto& kv : row) {
        idx.push_back(kv.first);
        val.push_back(kv.second);
      }
      ptr.push_back((int64_t)idx.size());
    }
    upload_v(st, w == 0 ? Arptr : Mrptr, ptr);
    upload_v(st, w == 0 ? Aridx : Mridx, idx);
    upload_v(st, w == 0 ? Arval : Mrval, val);
    if (w == 1 && P->m_diag) {
      std::vector<double> dg(n, 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
          if (idx[e] == i) dg[i] += val[e];
      upload_v(st, Mrdiag, dg);
    }
  }
}

// Y[:, c] = dg .* X[:, c] for c < cols
__global__ void k_diag_scale(const double* dg, int64_t n, const double* X, int64_t ldx, double* Y,
                             int64_t ldy, int64_t cols) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t c0 = (int64_t)blockIdx.y * CG;
  const double f = dg[r];
  double v[CG];
#pragma unroll
  for (int u = 0; u < CG; ++u) v[u] = c0 + u < cols ? X[r + (c0 + u) * ldx] : 0.0;
#pragma unroll
  for (int u = 0; u < CG; ++u)
    if (c0 + u < cols) Y[r + (c0 + u) * ldy] = f * v[u];
}

void EngineImpl::apply_m(hipStream_t st, const double* X, int64_t ldx, double* Y, int64_t ldy,
                         int64_t cols) {
  if (cols <= 0 || n <= 0) return;
  if (!P->m_diag || !Mrdiag.p) {
    csr_mm(st, Mrptr, Mridx, Mrval, n, X, ldx, Y, ldy, cols);
    return;
  }
  for (int64_t c = 0; c < cols; c += (int64_t)CG * 65535) {
    const int64_t cc = std::min<int64_t>(cols - c, (int64_t)CG * 65535);
    k_diag_scale<<<dim3(grid1(n), col_groups(cc)), 256, 0, st>>>(
        Mrdiag.as<double>(), n, X + c * ldx, ldx, Y + c * ldy, ldy, cc);
    RFD_CHECK_LAUNCH();
  }
}

// out[c] = ||X[:, c]||_M for c < cols (MX: n x cols scratch, used only when M
// is not diagonal).
void EngineImpl::col_mnorms(hipStream_t st, const double* X, int64_t cols, double* MX,
                            double* out) {
  if (cols <= 0 || n <= 0) return;
  if (P->m_diag && Mrdiag.p) {
    k_col_mnorm<<<(unsigned)cols, 256, 0, st>>>(Mrdiag.as<double>(), X, n, n, out);
  } else {
    apply_m(st, X, n, MX, n, cols);
    k_col_dots<<<(unsigned)cols, 256, 0, st>>>(X, n, MX, n, n, out);
  }
  RFD_CHECK_LAUNCH();
}

int64_t EngineImpl::interior_bytes() const {
  int64_t t = 0;
  for (const DevBuf* b : {&Vb, &Bs, &Bsinv, &Bspiv, &Bswide, &Bswork, &Lev, &Zt, &work1, &work2,
                          &work3, &work4, &work5, &work6})
    t += (int64_t)b->bytes;
  return t;
}

// Clusters for inverse iteration: consecutive values closer than gap.  With
// shifts from bisection (absolute error a few eps ||T||) and four iterations,
// vectors of eigenvalues 1e-10 ||T|| apart already come out orthogonal to
// working precision, so only tighter groups share a thread and are
// orthogonalised against each other.
static std::vector<int> clusters(const std::vector<double>& lam, double gap) {
  std::vector<int> c(lam.size());
  for (size_t i = 0; i < lam.size(); ++i)
    c[i] = (i > 0 && lam[i] - lam[i - 1] <= gap) ? c[i - 1] : (int)i;
  return c;
}

// Standard form of the pencils (B_j, M_Bj) for a non-diagonal M: C_j =
// G_j^{-1} B_j G_j^{-T} (C zero on entry) with M_Bj = G_j G_j^T from the
// factorization M_Bj = L_j U_j kept in Mlu / Mluinv; sq, isq (p x D) receive
// sqrt(u) and 1 / sqrt(u).  Sets the padding diagonal of C and returns it: a
// value above ||C_j||_inf of every block and |sigma|.
double EngineImpl::mb_standard_form(hipStream_t st, DMat<double> C, double* sq, double* isq,
                                    double sig) {
  Mlu.alloc(sizeof(double) * D * D * p);
  Mluinv.alloc(sizeof(double) * NB * 2 * D * p);
  mflag.alloc(sizeof(unsigned long long) * 2);
  RFD_HIP(hipMemsetAsync(mflag.p, 0, sizeof(unsigned long long) * 2, st));
  unsigned* fl = mflag.as<unsigned>();
  unsigned long long* nrm = mflag.as<unsigned long long>() + 1;
  DMat<double> F{Mlu.as<double>(), nullptr, D, D * D};
  DMat<double> Fi{Mluinv.as<double>(), nullptr, NB, NB * 2 * D};
  fill<double>(st, F, D, D, p, 0.0);
  k_expand_block<<<dim3(grid1(D), p), 256, 0, st>>>(F, D, dj.as<int32_t>(), Bg.view(), 1, 1.0);
  RFD_CHECK_LAUNCH();
  lu_nopiv<double>(st, F, D, p, Fi, fl, 1e-300);
  k_lu_diag<<<dim3(grid1(D), p), 256, 0, st>>>(F, D, dj.as<int32_t>(), sq, isq, fl);
  RFD_CHECK_LAUNCH();
  // C = L^{-1} B, W = C^T = B L^{-T}, W = L^{-1} W, C = sym(W) scaled by
  // diag(u)^{-1/2} on both sides
  k_expand_block<<<dim3(grid1(D), p), 256, 0, st>>>(C, D, dj.as<int32_t>(), Bg.view(), 0, 0.0);
  RFD_CHECK_LAUNCH();
  lu_solve<double>(st, F, Fi, nullptr, D, C, D, p, 1);
  DevBuf& wb = tmp[6];
  wb.alloc(sizeof(double) * D * D * p);
  DMat<double> Wm{wb.as<double>(), nullptr, D, D * D};
  const dim3 tg((unsigned)((D + TT - 1) / TT), (unsigned)((D + TT - 1) / TT), (unsigned)p);
  k_tile_transpose<<<tg, 256, 0, st>>>(C, Wm, D, nullptr, nullptr, 0);
  RFD_CHECK_LAUNCH();
  lu_solve<double>(st, F, Fi, nullptr, D, Wm, D, p, 1);
  k_tile_transpose<<<tg, 256, 0, st>>>(Wm, C, D, dj.as<int32_t>(), isq, 1);
  RFD_CHECK_LAUNCH();
  k_row_absmax<<<dim3(grid1(D), p), 256, 0, st>>>(C, D, dj.as<int32_t>(), nrm);
  RFD_CHECK_LAUNCH();
  unsigned long long h[2] = {0, 0};
  RFD_HIP(hipMemcpyAsync(h, mflag.p, sizeof(h), hipMemcpyDeviceToHost, st));
  RFD_HIP(hipStreamSynchronize(st));
  if ((unsigned)h[0])
    throw Error(ST_EBREAKDOWN, "M_B factorization: a subdomain block of M is not positive definite");
  double cn = 0.0;
  std::memcpy(&cn, &h[1], sizeof(double));
  if (!std::isfinite(cn)) throw Error(ST_EBREAKDOWN, "M_B factorization: non-finite value");
  const double big = 2.0 * cn + 4.0 * std::fabs(sig) + 1.0;
  k_pad_diag<<<dim3(grid1(D), p), 256, 0, st>>>(C, D, dj.as<int32_t>(), big);
  RFD_CHECK_LAUNCH();
  return big;
}

void EngineImpl::interior_basis(hipStream_t st, double sig, int nevb) {
  if (vcache_valid && vcache_sigma == sig && vcache_nevb == nevb) return;
  if (interior_solver == 1) {
    spectral_select(st, sig, nevb);
    return;
  }
  kappa.assign(p, 0);
  kappa_tot = 0;
  VB = 0;
  if (nevb == 0) {
    vcache_valid = true;
    vcache_sigma = sig;
    vcache_nevb = nevb;
    return;
  }
  timer.begin(st, 6);
  // standard-form dense blocks: M^{-1/2} B M^{-1/2} (diagonal M) or
  // G^{-1} B G^{-T} with M_Bj = G G^T (otherwise); the padding rows get a
  // diagonal value above every eigenvalue of the blocks
  work1.alloc(sizeof(double) * 2 * p * D);
  double* md = work1.as<double>();   // diag(M_B), or sqrt(u) of M_B = L U
  double* mis = md + p * D;          // its inverse square roots, or 1 / sqrt(u)
  work2.alloc(sizeof(double) * D * D * p);
  DMat<double> C{work2.as<double>(), nullptr, D, D * D};
  fill<double>(st, C, D, D, p, 0.0);
  double big;
  if (P->m_diag) {
    k_mdiag<<<dim3(grid1(D), p), 256, 0, st>>>(D, dj.as<int32_t>(), Bg.view(), md, mis);
    RFD_CHECK_LAUNCH();
    double mmin = 1e300;
    for (double v : M->val) mmin = std::min(mmin, v > 0 ? v : 1e300);
    big = 4.0 * normA / std::max(mmin, 1e-300) + 4.0 * std::fabs(sig) + 1.0;
    k_expand_scaled<<<dim3(grid1(D), p), 256, 0, st>>>(C, D, dj.as<int32_t>(), Bg.view(), mis,
                                                       big);
    RFD_CHECK_LAUNCH();
  } else {
    big = mb_standard_form(st, C, md, mis, sig);
  }
  TriWork& tw = tw_v;
  // the eigensolver runs on the leading DE = max d_j rows and columns: beyond
  // them every block is the decoupled identity padding
  const int64_t DE = std::max<int64_t>(P->d_max, 1);
  sy_tridiag(st, C, DE, p, tw);
  // indices around sigma
  std::vector<double> xs(p, sig);
  work3.alloc(sizeof(double) * p + sizeof(int) * p);
  RFD_HIP(hipMemcpyAsync(work3.p, xs.data(), sizeof(double) * p, hipMemcpyHostToDevice, st));
  int* cnt_d = reinterpret_cast<int*>(work3.as<double>() + p);
  sturm_counts(st, tw, DE, p, work3.as<double>(), 1, cnt_d);
  auto cnt = download<int>(st, cnt_d, p);
  const int extra = 6;
  std::vector<int> lo(p), num(p);
  int maxnum = 0;
  for (int j = 0; j < p; ++j) {
    const int d = (int)P->interior[j].size();
    const int a = std::max(0, cnt[j] - nevb - extra), b = std::min(d, cnt[j] + nevb + extra);
    lo[j] = a;
    num[j] = b - a;
    maxnum = std::max(maxnum, num[j]);
  }
  DevBuf &lo_d = tmp[0], &num_d = tmp[1], &lam_d = tmp[2];
  upload_v(st, lo_d, lo);
  upload_v(st, num_d, num);
  lam_d.alloc(sizeof(double) * (size_t)p * maxnum);
  bisect(st, tw, DE, p, lo_d.as<int>(), num_d.as<int>(), maxnum, lam_d.as<double>(), maxnum);
  auto lam = download<double>(st, lam_d.p, (size_t)p * maxnum);
  // nev_b closest to sigma, whole clusters at the cut (ascending window)
  std::vector<int> w0(p), w1(p);
  int kmax = 0;
  for (int j = 0; j < p; ++j) {
    std::vector<int> ord(num[j]);
    std::iota(ord.begin(), ord.end(), 0);
    const double* lj = lam.data() + (size_t)j * maxnum;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
      return std::fabs(lj[x] - sig) < std::fabs(lj[y] - sig);
    });
    int k = std::min(nevb, num[j]);
    if (k > 0) {
      const double cut = std::fabs(lj[ord[k - 1]] - sig);
      while (k < num[j] && std::fabs(lj[ord[k]] - sig) <= cut * (1.0 + 1e-9) + 1e-300) ++k;
    }
    int a = num[j], b = 0;
    for (int q = 0; q < k; ++q) {
      a = std::min(a, ord[q]);
      b = std::max(b, ord[q] + 1);
    }
    if (k == 0) a = b = 0;
    w0[j] = a;
    w1[j] = b;
    kappa[j] = b - a;
    kmax = std::max(kmax, kappa[j]);
  }
  VB = std::max<int64_t>(kmax, 1);
  std::vector<double> sel((size_t)p * VB, 0.0);
  std::vector<int> cl((size_t)p * VB, 0), knum(p);
  const double tn = big;
  for (int j = 0; j < p; ++j) {
    std::vector<double> v(lam.begin() + (size_t)j * maxnum + w0[j],
                          lam.begin() + (size_t)j * maxnum + w1[j]);
    auto c = clusters(v, 1e-10 * tn);
    for (int q = 0; q < kappa[j]; ++q) {
      sel[(size_t)j * VB + q] = v[q];
      cl[(size_t)j * VB + q] = c[q];
    }
    knum[j] = kappa[j];
    kappa_tot += kappa[j];
  }
  DevBuf &sel_d = tmp[3], &cl_d = tmp[4], &kn_d = tmp[5], &scratch = tmp[6];
  upload_v(st, sel_d, sel);
  upload_v(st, cl_d, cl);
  upload_v(st, kn_d, knum);
  Vb.alloc(sizeof(double) * D * VB * p);
  DMat<double> Y{Vb.as<double>(), nullptr, D, D * VB};
  // columns kappa_j .. VB-1 of a subdomain are padding and must stay zero: the
  // deflation GEMMs run over all VB columns
  fill<double>(st, Y, D, VB, p, 0.0);
  inverse_iteration(st, tw, DE, p, sel_d.as<double>(), kn_d.as<int>(), cl_d.as<int>(), VB, Y,
                    scratch);
  back_transform(st, C, tw, DE, p, Y, kn_d.as<int>(), (int)VB);
  if (P->m_diag) {
    // V = M^{-1/2} Y
    k_scale_rows<<<dim3(grid1(D * VB), p), 256, 0, st>>>(Y, D, VB, mis, D);
    RFD_CHECK_LAUNCH();
  } else {
    // V = G^{-T} Y = U^{-1} diag(u)^{1/2} Y
    k_scale_rows<<<dim3(grid1(D * VB), p), 256, 0, st>>>(Y, D, VB, md, D);
    RFD_CHECK_LAUNCH();
    DMat<double> F{Mlu.as<double>(), nullptr, D, D * D};
    DMat<double> Fi{Mluinv.as<double>(), nullptr, NB, NB * 2 * D};
    lu_solve<double>(st, F, Fi, nullptr, D, Y, VB, p, 2);
  }
  upload_v(st, kap_d, kappa);
  timer.end(st);
  RFD_HIP(hipStreamSynchronize(st));
  vcache_valid = true;
  vcache_sigma = sig;
  vcache_nevb = nevb;
}

// ---------------------------------------------------------------------------
// Spectral interior path (Sec. 4.1, the expansion in the proof of Thm. 4.2).
// With B_j V_j = M_Bj V_j Lambda_j and V_j^T M_Bj V_j = I, every shifted
// block has (B_j - z M_Bj)^{-1} = V_j (Lambda_j - z I)^{-1} V_j^T.  One
// eigendecomposition per pencil then gives, for every pole zeta and every
// sigma, X_j = V_j (Lambda_j - zeta)^{-1} V_j^T Ehat_j (two real products per
// pole), the resolvent levels B_sigma^{-1} M_B X = V_j (Lambda_j - sigma)^{-1}
// V_j^T M_B X, and the deflation vectors V_j near sigma as a column window:
// no shifted block is factored.  For a non-diagonal M the decomposition runs
// on the standard form G^{-1} B_j G^{-T} (M_Bj = G G^T), and when M couples
// the interiors to the interface, Ehat_zeta = Ehat - zeta Mhat_E, so that
// V^T Ehat_zeta = V^T Ehat - zeta V^T Mhat_E from two products per pencil.
// ---------------------------------------------------------------------------

// C_j[r, c] = Ehat_j[r, c] (which == 0) or Mhat_E^(j)[r, c] (otherwise) on the
// active rows r < d_j (C zero on entry; D x SJ items).
__global__ void k_expand_e(DMat<double> C, const int32_t* dj, DevPairCsr E, int which) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= dj[j]) return;
  DMat<double> c = C.item(j);
  const int64_t* ptr = E.ptr + E.roff[j];
  const double* v = which ? E.m : E.a;
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) c.re[r + (int64_t)E.idx[e] * c.ld] = v[e];
}

// Fz_j = (Lambda_j - zeta_l)^{-1} (FA_j - zeta_l FM_j) for the pole l = pole0
// (FA = V^T Ehat, FM = V^T Mhat_E, real), planar complex; rows at or beyond DE
// are zero.  Subdomains j over grid z.
__global__ void k_spec_scale2(DMat<double> Fz, DMat<double> FA, DMat<double> FM, int64_t D,
                              int64_t DE, int64_t SJ, int pole0, const double* lam, Shifts z) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  const int j = blockIdx.z, l = pole0;
  const int64_t c0 = (int64_t)blockIdx.y * CG;
  DMat<double> fa = FA.item(j), fm = FM.item(j), o = Fz.item(j);
  const double zr = z.z[2 * l], zi = z.z[2 * l + 1];
  double wr = 0.0, wi = 0.0;
  if (r < DE) {
    const double dr = lam[(int64_t)j * DE + r] - zr;
    const double den = dr * dr + zi * zi;
    wr = dr / den;
    wi = zi / den;
  }
#pragma unroll
  for (int u = 0; u < CG; ++u) {
    const int64_t c = c0 + u;
    if (c < SJ) {
      // (wr + i wi) (a - i b) with a = FA - zr FM, b = zi FM
      const double m = fm.re[r + c * fm.ld];
      const double av = fa.re[r + c * fa.ld] - zr * m, bv = zi * m;
      o.re[r + c * o.ld] = wr * av + wi * bv;
      o.im[r + c * o.ld] = wi * av - wr * bv;
    }
  }
}

// Fz_j[r, c] = (1 / (lam_j[r] - zeta_l)) F_j[r, c] for the pole l = pole0,
// planar complex; rows at or beyond DE (no eigenpair) are zero.  Subdomains
// j over grid z.
__global__ void k_spec_scale(DMat<double> Fz, DMat<double> F, int64_t D, int64_t DE, int64_t SJ,
                             int p, int pole0, const double* lam, Shifts z) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  const int j = blockIdx.z, l = pole0;
  const int64_t c0 = (int64_t)blockIdx.y * CG;
  DMat<double> f = F.item(j), o = Fz.item(j);
  double wr = 0.0, wi = 0.0;
  if (r < DE) {
    const double dr = lam[(int64_t)j * DE + r] - z.z[2 * l], zi = z.z[2 * l + 1];
    const double den = dr * dr + zi * zi;
    wr = dr / den;
    wi = zi / den;
  }
#pragma unroll
  for (int u = 0; u < CG; ++u) {
    const int64_t c = c0 + u;
    if (c < SJ) {
      const double v = f.re[r + c * f.ld];
      o.re[r + c * o.ld] = wr * v;
      o.im[r + c * o.ld] = wi * v;
    }
  }
}

// T_j[r, c] /= (lam_j[r] - sigma) for r < DE, c < cols.
__global__ void k_spec_rowdiv(DMat<double> T, int64_t DE, int64_t cols, const double* lam,
                              double sig) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= DE) return;
  const int64_t c0 = (int64_t)blockIdx.y * CG;
  DMat<double> t = T.item(blockIdx.z);
  const double w = 1.0 / (lam[(int64_t)blockIdx.z * DE + r] - sig);
#pragma unroll
  for (int u = 0; u < CG; ++u)
    if (c0 + u < cols) t.re[r + (c0 + u) * t.ld] *= w;
}

// G_j[i, i] += v for i < n.
__global__ void k_add_diag(DMat<double> G, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  DMat<double> g = G.item(blockIdx.y);
  g.re[i + i * g.ld] += v;
}

// U_j += a T_j over the leading n x n block.
__global__ void k_axpy_block(DMat<double> U, DMat<double> T, int64_t n, double a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t r = e % n, c = e / n;
  DMat<double> u = U.item(blockIdx.y), t = T.item(blockIdx.y);
  u.re[r + c * u.ld] += a * t.re[r + c * t.ld];
}

// Every eigenpair of every (B_j, M_Bj), once per pencil: the batched
// eigensolver of the interior basis run over the whole spectrum (bisection
// for all DE values, inverse iteration, back-transformation), then the
// eigenvector blocks U_j of M^{-1/2} B_j M^{-1/2} are brought to orthonormal
// columns by Newton-Schulz steps U <- U - U (U^T U - I) / 2 (quadratic: a
// departure of 1e-8 leaves 1e-16), so that V_j = M^{-1/2} U_j is
// M_Bj-orthonormal to rounding and the expansion above holds to rounding.
void EngineImpl::spectral_decompose(hipStream_t st) {
  if (spec_valid) return;
  timer.begin(st, 6);
  spec_f_valid = false;
  work1.alloc(sizeof(double) * 2 * p * D);
  double* md = work1.as<double>();   // diag(M_B), or sqrt(u) of M_B = L U
  double* mis = md + p * D;          // its inverse square roots, or 1 / sqrt(u)
  work2.alloc(sizeof(double) * D * D * p);
  DMat<double> C{work2.as<double>(), nullptr, D, D * D};
  fill<double>(st, C, D, D, p, 0.0);
  double big;
  if (P->m_diag) {
    k_mdiag<<<dim3(grid1(D), p), 256, 0, st>>>(D, dj.as<int32_t>(), Bg.view(), md, mis);
    RFD_CHECK_LAUNCH();
    double mmin = 1e300;
    for (double v : M->val) mmin = std::min(mmin, v > 0 ? v : 1e300);
    // padding rows carry a value above the whole spectrum (||B|| / min M <= normA / mmin)
    big = 4.0 * normA / std::max(mmin, 1e-300) + 1.0;
    k_expand_scaled<<<dim3(grid1(D), p), 256, 0, st>>>(C, D, dj.as<int32_t>(), Bg.view(), mis,
                                                       big);
    RFD_CHECK_LAUNCH();
  } else {
    // standard form G^{-1} B G^{-T} with M_B = G G^T
    big = mb_standard_form(st, C, md, mis, 0.0);
  }
  DE = std::max<int64_t>(P->d_max, 1);
  sy_tridiag(st, C, DE, p, tw_v);
  std::vector<int> lo(p, 0), num(p, (int)DE);
  DevBuf &lo_d = tmp[0], &num_d = tmp[1], &cl_d = tmp[4];
  upload_v(st, lo_d, lo);
  upload_v(st, num_d, num);
  lam_s.alloc(sizeof(double) * (size_t)p * DE);
  bisect(st, tw_v, DE, p, lo_d.as<int>(), num_d.as<int>(), (int)DE, lam_s.as<double>(), DE);
  lam_h = download<double>(st, lam_s.p, (size_t)p * DE);
  std::vector<int> cl((size_t)p * DE);
  for (int j = 0; j < p; ++j) {
    std::vector<double> v(lam_h.begin() + (size_t)j * DE, lam_h.begin() + (size_t)(j + 1) * DE);
    auto c = clusters(v, 1e-10 * big);
    std::copy(c.begin(), c.end(), cl.begin() + (size_t)j * DE);
  }
  upload_v(st, cl_d, cl);
  Vs.alloc(sizeof(double) * D * D * p);
  DMat<double> U{Vs.as<double>(), nullptr, D, D * D};
  fill<double>(st, U, D, D, p, 0.0);
  inverse_iteration(st, tw_v, DE, p, lam_s.as<double>(), num_d.as<int>(), cl_d.as<int>(), DE, U,
                    tmp[6]);
  back_transform(st, C, tw_v, DE, p, U, num_d.as<int>(), (int)DE);
  RFD_HIP(hipStreamSynchronize(st));
  tmp[6].release();  // inverse-iteration scratch (7 DE^2 p doubles)
  // Newton-Schulz orthonormalisation (C's storage is free again: G and U G)
  DevBuf& gbuf = Gsp;
  gbuf.alloc(sizeof(double) * D * D * p);
  DMat<double> G{gbuf.as<double>(), nullptr, D, D * D};
  double dev = 0;
  for (int it = 0;; ++it) {
    gemm<double>(st, true, false, DE, DE, DE, 1.0, U, U, 0.0, G, p);
    k_add_diag<<<dim3(grid1(DE), p), 256, 0, st>>>(G, DE, -1.0);
    RFD_CHECK_LAUNCH();
    zero_scalar(st, 2);
    absmax<double>(st, G, DE, DE, p, scal.as<double>() + 2);
    dev = read_scalar(st, 2);
    if (!(dev == dev)) throw Error(ST_EBREAKDOWN, "non-finite subdomain eigenvectors");
    if (dev <= 1e-14) break;
    if (dev > 0.25 || it >= 6)
      throw Error(ST_EBREAKDOWN, "subdomain eigenvectors not orthonormal (max |U^T U - I| = " +
                                     std::to_string(dev) + ")");
    gemm<double>(st, false, false, DE, DE, DE, 1.0, U, G, 0.0, C, p);
    k_axpy_block<<<dim3(grid1(DE * DE), p), 256, 0, st>>>(U, C, DE, -0.5);
    RFD_CHECK_LAUNCH();
  }
  spec_orth = dev;
  gbuf.release();
  if (P->m_diag) {
    // V = M^{-1/2} U
    k_scale_rows<<<dim3(grid1(D * D), p), 256, 0, st>>>(U, D, D, mis, D);
    RFD_CHECK_LAUNCH();
  } else {
    // V = G^{-T} U = U_M^{-1} diag(u)^{1/2} U (U_M: the upper factor of M_B)
    k_scale_rows<<<dim3(grid1(D * D), p), 256, 0, st>>>(U, D, D, md, D);
    RFD_CHECK_LAUNCH();
    DMat<double> F{Mlu.as<double>(), nullptr, D, D * D};
    DMat<double> Fi{Mluinv.as<double>(), nullptr, NB, NB * 2 * D};
    lu_solve<double>(st, F, Fi, nullptr, D, U, D, p, 2);
  }
  timer.end(st);
  RFD_HIP(hipStreamSynchronize(st));
  spec_valid = true;
  vcache_valid = false;
}

// The nev_b eigenpairs of each (B_j, M_Bj) closest to sigma, whole clusters
// at the cut (the rule of interior_basis), as a column window of V_j.
void EngineImpl::spectral_select(hipStream_t st, double sig, int nevb) {
  spectral_decompose(st);
  timer.begin(st, 6);
  work1.alloc(sizeof(double) * 2 * p * D);
  k_mdiag<<<dim3(grid1(D), p), 256, 0, st>>>(D, dj.as<int32_t>(), Bg.view(), work1.as<double>(),
                                            work1.as<double>() + p * D);
  RFD_CHECK_LAUNCH();
  kappa.assign(p, 0);
  kappa_tot = 0;
  std::vector<int> w0(p, 0);
  int kmax = 0;
  for (int j = 0; j < p && nevb > 0; ++j) {
    const int d = (int)P->interior[j].size();
    const double* lj = lam_h.data() + (size_t)j * DE;
    std::vector<int> ord(d);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
      return std::fabs(lj[x] - sig) < std::fabs(lj[y] - sig);
    });
    int k = std::min(nevb, d);
    if (k > 0) {
      const double cut = std::fabs(lj[ord[k - 1]] - sig);
      while (k < d && std::fabs(lj[ord[k]] - sig) <= cut * (1.0 + 1e-9) + 1e-300) ++k;
    }
    int a = d, b = 0;
    for (int q = 0; q < k; ++q) {
      a = std::min(a, ord[q]);
      b = std::max(b, ord[q] + 1);
    }
    if (k == 0) a = b = 0;
    w0[j] = a;
    kappa[j] = b - a;
    kmax = std::max(kmax, kappa[j]);
    kappa_tot += kappa[j];
  }
  VB = std::max<int64_t>(kmax, 1);
  Vb.alloc(sizeof(double) * D * VB * p);
  DMat<double> Y{Vb.as<double>(), nullptr, D, D * VB};
  fill<double>(st, Y, D, VB, p, 0.0);
  for (int j = 0; j < p; ++j)
    if (kappa[j] > 0)
      RFD_HIP(hipMemcpyAsync(Vb.as<double>() + (int64_t)j * D * VB,
                             Vs.as<double>() + (int64_t)j * D * D + (int64_t)w0[j] * D,
                             sizeof(double) * D * kappa[j], hipMemcpyDeviceToDevice, st));
  upload_v(st, kap_d, kappa);
  timer.end(st);
  RFD_HIP(hipStreamSynchronize(st));
  vcache_valid = true;
  vcache_sigma = sig;
  vcache_nevb = nevb;
}

// Schur-contribution solves of poles pole0 .. pole0 + np - 1 by the
// expansion: X_(l,j) = V_j (Lambda_j - zeta_l)^{-1} F_j with F_j = V_j^T Ehat_j
// (formed once per decomposition).  X: planar complex, D x SJ per item.
void EngineImpl::spectral_schur(hipStream_t st, int pole0, int np, DMat<double> X) {
  spectral_decompose(st);
  Shifts z{zeta.as<double>()};
  DMat<double> V{Vs.as<double>(), nullptr, D, D * D};
  const int64_t fs = D * SJ * (int64_t)p;
  // F = V^T Ehat, and FM = V^T Mhat_E when M couples interiors to the
  // interface (then Ehat_zeta = Ehat - zeta Mhat_E, so V^T Ehat_zeta = F - zeta FM)
  const bool me = !P->m_e_zero;
  if (!spec_f_valid) {
    DevBuf& eb = Gsp;
    eb.alloc(sizeof(double) * fs);
    DMat<double> E{eb.as<double>(), nullptr, D, D * SJ};
    Fs.alloc(sizeof(double) * fs * (me ? 2 : 1));
    for (int w = 0; w < (me ? 2 : 1); ++w) {
      fill<double>(st, E, D, SJ, p, 0.0);
      k_expand_e<<<dim3(grid1(D), p), 256, 0, st>>>(E, dj.as<int32_t>(), Eg.view(), w);
      RFD_CHECK_LAUNCH();
      DMat<double> F{Fs.as<double>() + w * fs, nullptr, D, D * SJ};
      gemm<double>(st, true, false, D, SJ, D, 1.0, V, E, 0.0, F, p);
    }
    RFD_HIP(hipStreamSynchronize(st));
    eb.release();
    spec_f_valid = true;
  }
  // one pole at a time: F scaled by that pole's 1 / (lambda - zeta), then
  // X = V F_zeta for its p items (real and imaginary planes)
  Fz.alloc(2 * sizeof(double) * fs);
  DMat<double> Fzm{Fz.as<double>(), Fz.as<double>() + fs, D, D * SJ};
  DMat<double> F{Fs.as<double>(), nullptr, D, D * SJ};
  DMat<double> Br{Fzm.re, nullptr, D, D * SJ}, Bi{Fzm.im, nullptr, D, D * SJ};
  for (int q = 0; q < np; ++q) {
    if (me) {
      DMat<double> FM{Fs.as<double>() + fs, nullptr, D, D * SJ};
      k_spec_scale2<<<dim3(grid1(D), col_groups(SJ), (unsigned)p), 256, 0, st>>>(
          Fzm, F, FM, D, DE, SJ, pole0 + q, lam_s.as<double>(), z);
    } else {
      k_spec_scale<<<dim3(grid1(D), col_groups(SJ), (unsigned)p), 256, 0, st>>>(
          Fzm, F, D, DE, SJ, p, pole0 + q, lam_s.as<double>(), z);
    }
    RFD_CHECK_LAUNCH();
    const int64_t off = (int64_t)q * p * X.bs;
    DMat<double> Cr{X.re + off, nullptr, X.ld, X.bs}, Ci{X.im + off, nullptr, X.ld, X.bs};
    gemm<double>(st, false, false, D, SJ, DE, 1.0, V, Br, 0.0, Cr, p);
    gemm<double>(st, false, false, D, SJ, DE, 1.0, V, Bi, 0.0, Ci, p);
  }
}

// X_j <- B_sigma^{-1} X_j = V_j (Lambda_j - sigma)^{-1} V_j^T X_j (D x cols per item).
void EngineImpl::spectral_level(hipStream_t st, DMat<double> X, int64_t cols, double sig) {
  for (int j = 0; j < p; ++j) {
    const int d = (int)P->interior[j].size();
    for (int i = 0; i < d; ++i)
      if (!(std::fabs(lam_h[(size_t)j * DE + i] - sig) > 1e-300))
        throw Error(ST_EBREAKDOWN, "sigma is an eigenvalue of a subdomain block");
  }
  DMat<double> V{Vs.as<double>(), nullptr, D, D * D};
  Ts.alloc(std::max<size_t>(Ts.bytes, sizeof(double) * D * cols * p));
  DMat<double> T{Ts.as<double>(), nullptr, D, D * cols};
  gemm<double>(st, true, false, DE, cols, D, 1.0, V, X, 0.0, T, p);
  k_spec_rowdiv<<<dim3(grid1(DE), col_groups(cols), p), 256, 0, st>>>(T, DE, cols,
                                                                      lam_s.as<double>(), sig);
  RFD_CHECK_LAUNCH();
  gemm<double>(st, false, false, D, cols, DE, 1.0, V, T, 0.0, X, p);
}

void EngineImpl::factor_bsigma(hipStream_t st, double sig, DevBuf* fl, bool check) {
  DevBuf& fw = fl ? *fl : flags;
  if (bs_valid && bs_sigma == sig) return;
  if (interior_solver == 1) {  // the levels use the spectral expansion
    bs_valid = true;
    bs_sigma = sig;
    return;
  }
  timer.begin(st, 7);
  Bs.alloc(sizeof(double) * D * D * p);
  Bsinv.alloc(sizeof(double) * NB * 2 * D * p);
  Bspiv.alloc(sizeof(int32_t) * D * p);
  DMat<double> K{Bs.as<double>(), nullptr, D, D * D};
  DMat<double> Ki{Bsinv.as<double>(), nullptr, NB, NB * 2 * D};
  fill<double>(st, K, D, D, p, 0.0);
  Shifts z{zeta.as<double>()};
  expand_shifted<double>(st, K, D, p, 1, 0, dj.as<int32_t>(), Bg.view(), z, true, sig);
  lu_piv<double>(st, K, D, p, Ki, Bspiv.as<int32_t>(), fw.as<unsigned>(), 1e-300);
  // the level solves stop their recursion at BLW-wide diagonal blocks (256 or
  // 128 when it divides D): their inverses are merged here once
  BLW = (D % 256 == 0 && D > 256) ? 256 : ((D % 128 == 0 && D > 128) ? 128 : 0);
  if (BLW) {
    const int64_t per = (int64_t)BLW * 2 * D;
    Bswide.alloc(sizeof(double) * per * p);
    const int64_t mw = (int64_t)(BLW / 2) * (BLW / 2) * std::max<int64_t>(D / BLW, p);
    Bswork.alloc(std::max<int64_t>(Bswork.bytes, sizeof(double) * mw));
    merge_inverses<double>(st, K, Ki, D, p, DMat<double>{Bswide.as<double>(), nullptr, BLW, per},
                           BLW, DMat<double>{Bswork.as<double>(), nullptr, BLW / 2, 0});
  }
  timer.end(st);
  // (the caller checks the flags itself when check is false, after it has
  // enqueued its other work)
  if (check) check_flags(st, "B_sigma factorization", &fw);
  bs_valid = true;
  bs_sigma = sig;
}

// Scales column c of U^{-1} by sqrt(u_cc) (the LDL^T diagonal), or zeroes it
// when c is dropped or padding.
__global__ void k_scale_uinv(double* Ui, int64_t ld, const double* U, int64_t ldu, const int* drop,
                             int64_t ncol, int64_t np) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * np) return;
  const int64_t i = e % np, c = e / np;
  const double f = (c < ncol && !drop[c]) ? sqrt(U[c + c * ldu]) : 0.0;
  Ui[i + c * ld] *= f;
}

// M-orthonormal basis of the ncol columns of B (n x ncol, ld n): G = B^T M B
// (unit diagonal for normalised columns), G = L D L^T by the blocked
// semidefinite LU (pivots <= droptol drop their column), Q = B U^{-1} D^{1/2}
// over the kept columns, written to Out (ld n).  MB is n x ncol scratch.
// Returns the number of columns written.
int EngineImpl::gram_orth(hipStream_t st, const double* B, int ncol, double* MB, double* Out,
                          double droptol) {
  const int64_t np = round_up(ncol, NB);
  apply_m(st, B, n, MB, n, ncol);
  gwork.alloc(sizeof(double) * (3 * np * np + (int64_t)NB * 2 * np) + sizeof(int) * (2 * np + 2));
  double* G = gwork.as<double>();
  double* Ui = G + np * np;
  double* Tk = Ui + np * np;
  double* Gi = Tk + np * np;
  int* drop = reinterpret_cast<int*>(Gi + (int64_t)NB * 2 * np);
  int* keep = drop + np;
  DMat<double> Gm{G, nullptr, np, 0}, Uim{Ui, nullptr, np, 0}, Gim{Gi, nullptr, NB, 0};
  DMat<double> Bm{const_cast<double*>(B), nullptr, n, 0}, MBm{MB, nullptr, n, 0};
  fill<double>(st, Gm, np, np, 1, 0.0);
  gemm_lower<double>(st, true, false, ncol, n, 1.0, Bm, MBm, 0.0, Gm, 1);
  k_mirror_lower<<<grid1((int64_t)ncol * ncol), 256, 0, st>>>(G, np, ncol);
  RFD_CHECK_LAUNCH();
  pad_identity<double>(st, Gm, ncol, np, 1);
  RFD_HIP(hipMemsetAsync(drop, 0, sizeof(int) * np, st));
  lu_nopiv<double>(st, Gm, np, 1, Gim, flags.as<unsigned>(), 0.0, drop, droptol);
  fill<double>(st, Uim, np, np, 1, 0.0);
  pad_identity<double>(st, Uim, 0, np, 1);
  lu_solve<double>(st, Gm, Gim, nullptr, np, Uim, np, 1, 2);
  k_scale_uinv<<<grid1(np * np), 256, 0, st>>>(Ui, np, G, np, drop, ncol, np);
  RFD_CHECK_LAUNCH();
  std::vector<int> dh(ncol);
  RFD_HIP(hipMemcpyAsync(dh.data(), drop, sizeof(int) * ncol, hipMemcpyDeviceToHost, st));
  RFD_HIP(hipStreamSynchronize(st));
  std::vector<int> kept;
  for (int c = 0; c < ncol; ++c)
    if (!dh[c]) kept.push_back(c);
  const int r = (int)kept.size();
  if (r == 0) return 0;
  // Q = B U^{-1} D^{1/2} with U^{-1} D^{1/2} upper triangular (its dropped
  // columns zero): the product skips the zero half of K, straight into Out
  // when every column is kept, else into MB and the kept columns gathered
  DMat<double> Om{Out, nullptr, n, 0};
  if (r == ncol) {
    gemm_triu_b(st, n, ncol, ncol, 1.0, Bm, Uim, 0.0, Om, 1);
  } else {
    kept.push_back(r);  // device copy of the count follows the list
    RFD_HIP(hipMemcpyAsync(keep, kept.data(), sizeof(int) * (r + 1), hipMemcpyHostToDevice, st));
    gemm_triu_b(st, n, ncol, ncol, 1.0, Bm, Uim, 0.0, MBm, 1);
    k_gather_cols<<<dim3(grid1(n), r), 256, 0, st>>>(MB, n, Out, n, n, keep, keep + r);
    RFD_CHECK_LAUNCH();
  }
  RFD_HIP(hipStreamSynchronize(st));
  return r;
}

// X (n x ncols, reordered numbering) -= V (V^T M X) per subdomain and
// -= Zp (Zp^T M X) for the kprev previous level columns, `passes` times.
// MX is n x ncols scratch.
void EngineImpl::project_out(hipStream_t st, double* X, int ncols, double* MX, const double* Zp,
                             int64_t kprev, int passes) {
  if (ncols <= 0) return;
  DMat<double> Xm{X, nullptr, n, 0}, MXm{MX, nullptr, n, 0};
  for (int pass = 0; pass < passes; ++pass) {
    if (kappa_tot > 0) {
      apply_m(st, X, n, MX, n, ncols);
      work4.alloc(sizeof(double) * std::max<int64_t>(VB, 1) * std::max<int64_t>(MUP, ncols) * p);
      const int64_t ldt = std::max<int64_t>(VB, 1);
      bool uniform = true;
      for (int j = 1; j < p; ++j)
        if (P->interior[j].size() != P->interior[0].size()) uniform = false;
      if (uniform) {
        const int64_t d = (int64_t)P->interior[0].size();
        DMat<double> Vm{Vb.as<double>(), nullptr, D, D * VB};
        DMat<double> Xb{X, nullptr, n, d}, MXb{MX, nullptr, n, d};
        DMat<double> Tm{work4.as<double>(), nullptr, ldt, ldt * ncols};
        gemm<double>(st, true, false, VB, ncols, d, 1.0, Vm, MXb, 0.0, Tm, p);
        gemm<double>(st, false, false, d, ncols, VB, -1.0, Vm, Tm, 1.0, Xb, p);
      } else {
        int64_t off = 0;
        for (int j = 0; j < p; ++j) {
          const int64_t d = (int64_t)P->interior[j].size();
          DMat<double> Vm{Vb.as<double>() + (int64_t)j * D * VB, nullptr, D, 0};
          DMat<double> Xb{X + off, nullptr, n, 0}, MXb{MX + off, nullptr, n, 0};
          DMat<double> Tm{work4.as<double>(), nullptr, ldt, 0};
          gemm<double>(st, true, false, VB, ncols, d, 1.0, Vm, MXb, 0.0, Tm, 1);
          gemm<double>(st, false, false, d, ncols, VB, -1.0, Vm, Tm, 1.0, Xb, 1);
          off += d;
        }
      }
    }
    if (kprev > 0) {
      apply_m(st, X, n, MX, n, ncols);
      work6b.alloc(sizeof(double) * kprev * ncols);
      DMat<double> Zm{const_cast<double*>(Zp), nullptr, n, 0};
      DMat<double> Tq{work6b.as<double>(), nullptr, kprev, 0};
      gemm<double>(st, true, false, kprev, ncols, n, 1.0, Zm, MXm, 0.0, Tq, 1);
      gemm<double>(st, false, false, n, ncols, kprev, -1.0, Zm, Tq, 1.0, Xm, 1);
    }
  }
}

// The helper stream and its events (created on first use, on the caller's
// device); earlier work on it is finished before its buffers are reused.
// Small bases (A Z under 2^24 entries) form H in the Rayleigh-Ritz call
// instead: their blocks are too small to gain from the overlap, and a stream
// per engine would crowd the hardware queues that concurrent engines share.
void EngineImpl::h_begin(bool use) {
  h_ready = false;
  h_use = use;
  if (h_stream) RFD_HIP(hipStreamSynchronize(h_stream));
  if (!use) return;
  if (!h_stream) {
    RFD_HIP(hipStreamCreateWithFlags(&h_stream, hipStreamNonBlocking));
    RFD_HIP(hipEventCreateWithFlags(&h_lvl, hipEventDisableTiming));
    RFD_HIP(hipEventCreateWithFlags(&h_done, hipEventDisableTiming));
  }
}

// Columns [c0, c0 + r) of Z are final on st: on the helper stream, A Z for
// them and H's rows c0 .. c0 + r - 1 up to the block's diagonal.  The
// deflation columns (c0 = 0, r = kappa_tot) give the block-diagonal H_vv (one
// kappa_j block per subdomain, their interior rows only); a level block gives
// its rows against the deflation columns ((A Z_blk)^T Z_v, the subdomain's
// rows only, as interiors couple through the interface alone) and against the
// level columns so far (Z_blk^T A Z).
void EngineImpl::h_add_block(hipStream_t st, int64_t c0, int64_t r) {
  if (r <= 0 || !h_use) return;
  RFD_HIP(hipEventRecord(h_lvl, st));
  RFD_HIP(hipStreamWaitEvent(h_stream, h_lvl, 0));
  hipStream_t s2 = h_stream;
  double* Z = Zt.as<double>();
  double* AZ = rr_az.as<double>();
  double* H = rr_h.as<double>();
  const int64_t ld = h_ld, kv = kappa_tot;
  csr_mm(s2, Arptr, Aridx, Arval, n, Z + c0 * n, n, AZ + c0 * n, n, r);
  DMat<double> Zm{Z, nullptr, n, 0}, AZm{AZ, nullptr, n, 0}, Hm{H, nullptr, ld, 0};
  bool uniform = true;
  for (int j = 1; j < p && uniform; ++j)
    uniform = P->interior[j].size() == P->interior[0].size() && kappa[j] == kappa[0];
  if (c0 < kv) {
    fill<double>(s2, Hm, kv, kv, 1, 0.0);
    if (uniform) {
      const int64_t d = (int64_t)P->interior[0].size(), kj = kappa[0];
      DMat<double> Zb{Z, nullptr, n, d + kj * n}, AZb{AZ, nullptr, n, d + kj * n};
      DMat<double> Hvv{H, nullptr, ld, kj + kj * ld};
      gemm<double>(s2, true, false, kj, kj, d, 1.0, Zb, AZb, 0.0, Hvv, p);
    } else {
      int64_t off = 0, kof = 0;
      for (int j = 0; j < p; ++j) {
        const int64_t d = (int64_t)P->interior[j].size(), kj = kappa[j];
        if (kj > 0)
          gemm<double>(s2, true, false, kj, kj, d, 1.0, Zm.sub(off, kof), AZm.sub(off, kof), 0.0,
                       Hm.sub(kof, kof), 1);
        off += d;
        kof += kj;
      }
    }
    return;
  }
  if (kv > 0) {
    if (uniform) {
      const int64_t d = (int64_t)P->interior[0].size(), kj = kappa[0];
      DMat<double> Zb{Z, nullptr, n, d + kj * n};
      DMat<double> AZl{AZ + c0 * n, nullptr, n, d};
      DMat<double> Hlv{H + c0, nullptr, ld, kj * ld};
      gemm<double>(s2, true, false, r, kj, d, 1.0, AZl, Zb, 0.0, Hlv, p);
    } else {
      int64_t off = 0, kof = 0;
      for (int j = 0; j < p; ++j) {
        const int64_t d = (int64_t)P->interior[j].size(), kj = kappa[j];
        if (kj > 0)
          gemm<double>(s2, true, false, r, kj, d, 1.0, AZm.sub(off, c0), Zm.sub(off, kof), 0.0,
                       Hm.sub(c0, kof), 1);
        off += d;
        kof += kj;
      }
    }
  }
  gemm<double>(s2, true, false, r, c0 + r - kv, n, 1.0, Zm.sub(0, c0), AZm.sub(0, kv), 0.0,
               Hm.sub(c0, kv), 1);
}

void Engine::solve_interior(hipStream_t st, double sig, int nevb, int psi, int64_t* kout) {
  EngineImpl& e = *d_;
  e.join_prepare();
  if (e.Qint.p == nullptr) throw Error(ST_ESTATE, "rfd_filter_interface has not been called");
  e.ensure_reordered(st);
  e.interior_basis(st, sig, nevb);
  e.factor_bsigma(st, sig);
  const int p = e.p, mu = e.mu;
  const int64_t D = e.D, n = e.n, s = e.s;
  const int64_t n_int = n - s;
  e.sigma = sig;
  e.nev_b = nevb;
  e.psi = psi;
  e.MUP = round_up(std::max(mu, 1), NB);
  const int64_t MUP = e.MUP;
  // diag(M_B) per subdomain row, from interior_basis (read for a diagonal M only)
  const double* md = e.work1.as<double>();
  if (nevb == 0) {
    e.work1.alloc(sizeof(double) * 2 * p * D);
    k_mdiag<<<dim3(grid1(D), p), 256, 0, st>>>(D, e.dj.as<int32_t>(), e.Bg.view(),
                                              e.work1.as<double>(), e.work1.as<double>() + p * D);
    RFD_CHECK_LAUNCH();
    md = e.work1.as<double>();
  }
  // resolvent levels: Sigma (from Phi) and, when M_E != 0, Gamma (from Psi)
  const bool mdg = e.P->m_diag;
  const int ng = e.P->m_e_zero ? 1 : 2;
  const int nlev = psi * ng;
  e.timer.begin(st, 8);
  e.Lev.alloc(sizeof(double) * D * nlev * MUP * p);
  e.work3.alloc(sizeof(double) * D * MUP * p);            // right-hand side / M_B X
  e.work4.alloc(sizeof(double) * std::max<int64_t>(e.VB, 1) * MUP * p);  // V^T M X
  DMat<double> Lv{e.Lev.as<double>(), nullptr, D, D * nlev * MUP};
  DMat<double> Rh{e.work3.as<double>(), nullptr, D, D * MUP};
  DMat<double> Ki{e.Bsinv.as<double>(), nullptr, NB, NB * 2 * D};
  DMat<double> Bm{e.Bs.as<double>(), nullptr, D, D * D};
  DMat<double> Vm{e.Vb.as<double>(), nullptr, D, D * e.VB};
  DMat<double> Tm{e.work4.as<double>(), nullptr, std::max<int64_t>(e.VB, 1),
                  std::max<int64_t>(e.VB, 1) * MUP};
  const dim3 lg(grid1(D), col_groups(MUP), p);
  // Y = M_B X, per subdomain
  auto apply_mb = [&](DMat<double> X, DMat<double> Y) {
    if (mdg)
      k_scaled_copy<<<lg, 256, 0, st>>>(X, Y, D, MUP, md, D);
    else
      k_block_mb<<<lg, 256, 0, st>>>(X, Y, D, MUP, e.dj.as<int32_t>(), e.Bg.view());
    RFD_CHECK_LAUNCH();
  };
  // out[c] = M_B-norm of column c of a level (Rh is scratch for a general M)
  auto level_norms = [&](DMat<double> X, double* out) {
    if (mdg) {
      k_level_colnorm<<<MUP, 256, 0, st>>>(X, p, e.dj.as<int32_t>(), md, D, out);
    } else {
      apply_mb(X, Rh);
      k_level_coldot<<<MUP, 256, 0, st>>>(X, Rh, p, e.dj.as<int32_t>(), out);
    }
    RFD_CHECK_LAUNCH();
  };
  DevBuf& nrm = e.tmp[7];
  nrm.alloc(sizeof(double) * 2 * MUP);
  double* pre = nrm.as<double>();
  double* post = pre + MUP;
  for (int g = 0; g < ng; ++g) {
    k_gather_phi<<<dim3(grid1(D * MUP), p), 256, 0, st>>>(
        Rh, D, MUP, e.dj.as<int32_t>(), e.Eg.view(), g == 0 ? -1.0 : 0.0, g == 0 ? sig : 1.0,
        e.Qint.as<double>(), s, mu, e.adj.as<int32_t>(), e.SJ);
    RFD_CHECK_LAUNCH();
    for (int t = 0; t < psi; ++t) {
      DMat<double> X = Lv.sub(0, (g * psi + t) * MUP);
      convert<double, double>(st, Rh, X, D, MUP, p);
      if (e.interior_solver == 1) {
        e.spectral_level(st, X, MUP, sig);
      } else if (e.BLW) {
        const int64_t per = (int64_t)e.BLW * 2 * D;
        e.Bswork.alloc(std::max<int64_t>(e.Bswork.bytes, sizeof(double) * e.BLW * MUP * p));
        lu_solve<double>(st, Bm, Ki, e.Bspiv.as<int32_t>(), D, X, MUP, p, 3,
                         DMat<double>{e.Bswide.as<double>(), nullptr, e.BLW, per}, e.BLW,
                         DMat<double>{e.Bswork.as<double>(), nullptr, e.BLW, e.BLW * MUP});
      } else {
        lu_solve<double>(st, Bm, Ki, e.Bspiv.as<int32_t>(), D, X, MUP, p);
      }
      // make the level M_B-orthogonal to V_j (twice)
      if (e.kappa_tot > 0) {
        if (t > 0) level_norms(X, pre);
        for (int pass = 0; pass < 2; ++pass) {
          apply_mb(X, Rh);
          gemm<double>(st, true, false, e.VB, MUP, D, 1.0, Vm, Rh, 0.0, Tm, p);
          gemm<double>(st, false, false, D, MUP, e.VB, -1.0, Vm, Tm, 1.0, X, p);
        }
        if (t > 0) {
          level_norms(X, post);
          k_level_drop<<<lg, 256, 0, st>>>(X, D, MUP, pre, post, 1e-10);
          RFD_CHECK_LAUNCH();
        }
      }
      if (t + 1 < psi) apply_mb(X, Rh);
    }
  }
  e.timer.end(st);
  // M-orthonormal basis of range(Z): [V | levels orthonormalised level by level]
  e.timer.begin(st, 9);
  const int64_t kmax = e.kappa_tot + (int64_t)nlev * mu;
  e.h_begin(n * std::max<int64_t>(kmax, 1) >= (int64_t(1) << 24));
  e.Zt.alloc(sizeof(double) * n * std::max<int64_t>(kmax, 1));
  double* Z = e.Zt.as<double>();
  RFD_HIP(hipMemsetAsync(Z, 0, sizeof(double) * n * std::max<int64_t>(kmax, 1), st));
  if (e.h_use) {
    e.h_ld = std::max<int64_t>(kmax, 1);
    e.rr_az.alloc(sizeof(double) * n * e.h_ld);
    e.rr_h.alloc(sizeof(double) * e.h_ld * e.h_ld);
  }
  std::vector<int32_t> koff(p, 0), ioff(p + 1, 0);
  for (int j = 0; j < p; ++j) {
    koff[j] = (j ? koff[j - 1] + e.kappa[j - 1] : 0);
    ioff[j + 1] = ioff[j] + (int32_t)e.P->interior[j].size();
  }
  DevBuf &koff_d = e.tmp[8], &kap_d2 = e.tmp[9];
  upload_v(st, koff_d, koff);
  upload_v(st, kap_d2, e.kappa);
  if (e.kappa_tot > 0) {
    k_scatter_v<<<dim3(grid1(D * e.VB), p), 256, 0, st>>>(Z, n, Vm, e.ioff.as<int32_t>(),
                                                          koff_d.as<int32_t>(),
                                                          kap_d2.as<int32_t>(), e.dj.as<int32_t>(), D);
    RFD_CHECK_LAUNCH();
    e.h_add_block(st, 0, e.kappa_tot);
  }
  e.work5.alloc(sizeof(double) * n * (int64_t)mu * 2);
  double* Lb = e.work5.as<double>();             // current level block (n x mu)
  double* MLb = Lb + n * (int64_t)mu;            // M * block
  e.work6.alloc(sizeof(double) * (2 * mu + 8));
  double* n0 = e.work6.as<double>();             // column M-norms before / after projection
  double* n1 = n0 + mu;
  int64_t kz = e.kappa_tot;
  for (int t = 0; t < nlev && mu > 0; ++t) {
    k_build_level<<<dim3(grid1(n), col_groups(mu)), 256, 0, st>>>(
        Lb, n, Lv, t, MUP, e.ioff.as<int32_t>(), p, n_int, n, e.Qint.as<double>(), s, mu);
    RFD_CHECK_LAUNCH();
    // column M-norms before projection
    e.col_mnorms(st, Lb, mu, MLb, n0);
    // project against V and the previous level blocks (M-inner product)
    const int64_t kprev = kz - e.kappa_tot;
    e.project_out(st, Lb, mu, MLb, Z + e.kappa_tot * n, kprev, 1);
    e.col_mnorms(st, Lb, mu, MLb, n1);
    k_col_normalize<<<dim3(grid1(n), mu), 256, 0, st>>>(Lb, n, n, n1, n0, 1e-10);
    RFD_CHECK_LAUNCH();
    // block Gram-Schmidt twice with Cholesky QR through the semidefinite
    // LDL^T: the first pass drops the columns that depend on earlier ones; a
    // kept column with a small pivot amplifies rounding, so the result is
    // projected once more before the second pass restores orthonormality
    const int r = e.gram_orth(st, Lb, mu, MLb, Z + kz * n, 1e-13);
    if (r == 0) continue;
    e.project_out(st, Z + kz * n, r, MLb, Z + e.kappa_tot * n, kprev, 1);
    const int r2 = e.gram_orth(st, Z + kz * n, r, MLb, Lb, 1e-20);
    RFD_HIP(hipMemcpyAsync(Z + kz * n, Lb, sizeof(double) * n * r2, hipMemcpyDeviceToDevice, st));
    if (r2 < r)
      RFD_HIP(hipMemsetAsync(Z + (kz + r2) * n, 0, sizeof(double) * n * (r - r2), st));
    e.h_add_block(st, kz, r2);
    kz += r2;
  }
  e.kz = kz;
  if (e.h_use) {
    RFD_HIP(hipEventRecord(e.h_done, e.h_stream));
    e.h_ready = true;
    e.h_k = kz;
  }
  e.timer.end(st);
  RFD_HIP(hipStreamSynchronize(st));
  e.interior_ready = true;
  *kout = kz;
}

void Engine::copy_basis(hipStream_t st, double* dst, int64_t cap, int64_t* k) {
  EngineImpl& e = *d_;
  e.join_prepare();
  *k = e.interior_ready ? e.kz : 0;
  const int64_t c = std::min(cap, *k);
  if (c > 0)
    RFD_HIP(hipMemcpyAsync(dst, e.Zt.p, sizeof(double) * e.n * c, hipMemcpyDeviceToDevice, st));
  RFD_HIP(hipStreamSynchronize(st));
}

// Eigenpairs of H (lower triangle, k x k, overwritten) in [alpha, beta], the
// Ritz vectors Z G in the original numbering, their residuals.
static void rr_eigen(EngineImpl& e, hipStream_t st, DMat<double> Hm, DMat<double> Zm, int64_t k,
                     int max_out, double* evals, double* evecs, double* resid, int* nfound) {
  const int64_t n = e.n;
  // eigenpairs of H in [alpha, beta]
  e.timer.begin(st, 10);
  TriWork& tw = e.tw_h;
  sy_tridiag(st, Hm, k, 1, tw);
  DevBuf &xs = e.tmp[10], &cnt = e.tmp[11];
  std::vector<double> ab{e.poles.alpha, e.poles.beta};
  upload_v(st, xs, ab);
  cnt.alloc(sizeof(int) * 2);
  sturm_counts(st, tw, k, 1, xs.as<double>(), 2, cnt.as<int>());
  auto c = download<int>(st, cnt.p, 2);
  const int i0 = c[0], nf = c[1] - c[0];
  *nfound = nf;
  const int nout = std::min(nf, max_out);
  if (nout <= 0) {
    e.timer.end(st);
    return;
  }
  DevBuf &lo_d = e.tmp[12], &num_d = e.tmp[13], &lam_d = e.tmp[14];
  upload_v(st, lo_d, std::vector<int>{i0});
  upload_v(st, num_d, std::vector<int>{nout});
  lam_d.alloc(sizeof(double) * nout);
  bisect(st, tw, k, 1, lo_d.as<int>(), num_d.as<int>(), nout, lam_d.as<double>(), nout);
  auto lam = download<double>(st, lam_d.p, nout);
  double tn = 0;
  for (double v : lam) tn = std::max(tn, std::fabs(v));
  tn = std::max(tn, e.normA);
  auto cl = clusters(lam, 1e-10 * tn);
  DevBuf &cl_d = e.tmp[15], &Gv = e.tmp[16], &scratch = e.tmp[17];
  upload_v(st, cl_d, cl);
  Gv.alloc(sizeof(double) * k * nout);
  DMat<double> Gm{Gv.as<double>(), nullptr, k, 0};
  inverse_iteration(st, tw, k, 1, lam_d.as<double>(), num_d.as<int>(), cl_d.as<int>(), nout, Gm,
                    scratch);
  back_transform(st, Hm, tw, k, 1, Gm, num_d.as<int>(), nout);
  e.timer.end(st);
  // Ritz vectors, original numbering, residuals
  e.timer.begin(st, 11);
  RFD_HIP(hipMemcpyAsync(evals, lam_d.p, sizeof(double) * nout, hipMemcpyDeviceToDevice, st));
  DevBuf &Xr = e.tmp[18], &X2 = e.tmp[19], &AX = e.tmp[20], &MX = e.tmp[21];
  Xr.alloc(sizeof(double) * n * nout);
  DMat<double> Xm{Xr.as<double>(), nullptr, n, 0};
  gemm<double>(st, false, false, n, nout, k, 1.0, Zm, Gm, 0.0, Xm, 1);
  double* Xo = evecs;
  if (!Xo) {
    X2.alloc(sizeof(double) * n * nout);
    Xo = X2.as<double>();
  }
  k_unpermute<<<grid1(n * nout), 256, 0, st>>>(Xr.as<double>(), n, e.order.as<int32_t>(), n, Xo, n,
                                               nout);
  RFD_CHECK_LAUNCH();
  if (resid) {
    AX.alloc(sizeof(double) * n * nout);
    MX.alloc(sizeof(double) * n * nout);
    csr_mm(st, e.Aptr, e.Aidx, e.Aval, n, Xo, n, AX.as<double>(), n, nout);
    csr_mm(st, e.Mptr, e.Midx, e.Mval, n, Xo, n, MX.as<double>(), n, nout);
    k_resid<<<nout, 256, 0, st>>>(AX.as<double>(), MX.as<double>(), Xo, n, n, lam_d.as<double>(),
                                  e.normA, resid);
    RFD_CHECK_LAUNCH();
  }
  e.timer.end(st);
  RFD_HIP(hipStreamSynchronize(st));
}

void Engine::rayleigh_ritz(hipStream_t st, int max_out, double* evals, double* evecs,
                           double* resid, int* nfound) {
  EngineImpl& e = *d_;
  e.join_prepare();
  if (!e.interior_ready) throw Error(ST_ESTATE, "rfd_solve_interior has not been called");
  const int64_t n = e.n, k = e.kz;
  *nfound = 0;
  if (k == 0) return;
  double* Z = e.Zt.as<double>();
  // H = Z^T A Z, lower triangle (all the eigensolver reads).  Z = [Zv Zl]:
  // the kv deflation columns of subdomain j live on its interior rows only,
  // and interiors couple through the interface alone, so H_vv is block
  // diagonal (one kappa_j block per subdomain) and H_lv = (A Zl)^T Zv needs
  // each subdomain's interior rows only; H_ll = Zl^T (A Zl) is dense.
  DMat<double> Zm{Z, nullptr, n, 0};
  if (e.h_ready && e.h_k == k) {
    // assembled beside the construction of Z; used once (the eigensolver
    // overwrites it, a later call forms it again below)
    RFD_HIP(hipStreamWaitEvent(st, e.h_done, 0));
    e.h_ready = false;
    rr_eigen(e, st, DMat<double>{e.rr_h.as<double>(), nullptr, e.h_ld, 0}, Zm, k, max_out, evals,
             evecs, resid, nfound);
    return;
  }
  e.h_ready = false;
  e.timer.begin(st, 9);
  DevBuf& AZ = e.rr_az;
  DevBuf& Hb = e.rr_h;
  AZ.alloc(sizeof(double) * n * k);
  Hb.alloc(sizeof(double) * k * k);
  csr_mm(st, e.Arptr, e.Aridx, e.Arval, n, Z, n, AZ.as<double>(), n, k);
  DMat<double> AZm{AZ.as<double>(), nullptr, n, 0}, Hm{Hb.as<double>(), nullptr, k, 0};
  const int64_t kv = std::min<int64_t>(e.kappa_tot, k), kl = k - kv;
  bool uniform = kv > 0;
  for (int j = 1; j < e.p && uniform; ++j)
    uniform = e.P->interior[j].size() == e.P->interior[0].size() && e.kappa[j] == e.kappa[0];
  if (uniform) {
    // one batched product per block over the subdomains (item j: rows j d,
    // deflation columns j kj)
    fill<double>(st, Hm, kv, kv, 1, 0.0);
    const int64_t d = (int64_t)e.P->interior[0].size(), kj = e.kappa[0];
    DMat<double> Zb{Z, nullptr, n, d + kj * n}, AZb{AZ.as<double>(), nullptr, n, d + kj * n};
    DMat<double> Hvv{Hb.as<double>(), nullptr, k, kj + kj * k};
    gemm<double>(st, true, false, kj, kj, d, 1.0, Zb, AZb, 0.0, Hvv, e.p);
    if (kl > 0) {
      DMat<double> AZl{AZ.as<double>() + kv * n, nullptr, n, d};
      DMat<double> Hlv{Hb.as<double>() + kv, nullptr, k, kj * k};
      gemm<double>(st, true, false, kl, kj, d, 1.0, AZl, Zb, 0.0, Hlv, e.p);
    }
  } else if (kv > 0) {
    fill<double>(st, Hm, kv, kv, 1, 0.0);
    int64_t off = 0, kof = 0;
    for (int j = 0; j < e.p; ++j) {
      const int64_t d = (int64_t)e.P->interior[j].size(), kj = e.kappa[j];
      if (kj > 0) {
        DMat<double> Zj = Zm.sub(off, kof), AZj = AZm.sub(off, kof);
        gemm<double>(st, true, false, kj, kj, d, 1.0, Zj, AZj, 0.0, Hm.sub(kof, kof), 1);
        if (kl > 0)
          gemm<double>(st, true, false, kl, kj, d, 1.0, AZm.sub(off, kv), Zj, 0.0,
                       Hm.sub(kv, kof), 1);
      }
      off += d;
      kof += kj;
    }
  }
  if (kl > 0)
    gemm<double>(st, true, false, kl, kl, n, 1.0, Zm.sub(0, kv), AZm.sub(0, kv), 0.0,
                 Hm.sub(kv, kv), 1);
  e.timer.end(st);
  rr_eigen(e, st, Hm, Zm, k, max_out, evals, evecs, resid, nfound);
}

}  // namespace rfd
