// Dense FP64 symmetric eigensolver for selected eigenpairs (see eig.hpp):
// blocked Householder tridiagonalization, Sturm-count bisection, inverse
// iteration, back-transformation.
#include <algorithm>
#include <cmath>

#include <hip/hip_ext.h>

#include "dense.hpp"
#include "eig.hpp"

namespace rfd {

constexpr double EPS = 2.220446049250313e-16;
constexpr double SAFMIN = 2.2250738585072014e-308;

// v + (v moved across lanes by the DPP control CTRL, in the rows of 16 lanes
// that ROWS selects; other lanes add 0)
template <int CTRL, int ROWS>
__device__ inline double dpp_add(double v) {
  const uint64_t w = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)w, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(w >> 32), CTRL, ROWS, 0xf, false);
  return v + __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active), the same value in
// every lane: pairs and quads by quad permutations, 8 and 16 lanes by the
// half-row and row mirrors, then row sums carried into rows 1 and 3 and row
// 3 completed from lane 31; lane 63 holds the total.  Data-parallel moves
// only, no round trip through the LDS crossbar.
__device__ inline double wave_sum(double v) {
  v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
  v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
  const uint64_t w = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)w, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(w >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
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
  // each buffer grows on its own (DevBuf::alloc keeps a larger one): the
  // tile buffers grow with n^2, the others with n
  const int64_t need = n * (int64_t)batch;
  cap = std::max(cap, need);
  d.alloc(sizeof(double) * need);
  e.alloc(sizeof(double) * need);
  tau.alloc(sizeof(double) * need);
  acol.alloc(sizeof(double) * need);
  vw.alloc(sizeof(double) * need * 3 * TRI_NB);
  red.alloc(sizeof(double) * (2 * TRI_NB + 2) * batch);
  sq.alloc(sizeof(double) * ((n + 63) / 64) * batch);
  const int64_t nb = tri_blocks(n);
  pt.alloc(sizeof(double) * (nb + 1) * need);
  ptvp.alloc(sizeof(double) * (nb * (nb + 1) / 2) * batch);
}

// Blocked reduction (panels of TRI_NB columns).  Within a panel the trailing
// matrix is A - V W^T - W V^T with A as it was at the panel's start; V holds
// the reflectors (unit entry explicit, zero above it) and W the matching
// update vectors.  Only the lower triangle of A is read or updated.  For
// column j (panel position c):
//   k_tri_col   finishes W[:, c-1], forms the updated column j into acol and
//               the partial sums of squares below its subdiagonal;
//   k_tri_symv  makes the reflector v from acol (every workgroup), writes it
//               to V[:, c] and column j of A, and forms the pieces of
//               p = A v over the trailing block of the panel-start matrix,
//               64 x 64 lower tiles at a time (the next k_tri_col sums them);
//               2c extra workgroups of the same launch form W^T v and V^T v.
// After the panel, the lower triangle of the trailing block takes
// A -= [V W] [W V]^T as one product.
// w_c = tau (p - V (W^T v) - W (V^T v)) - (tau/2) (that^T v) v, i.e. the
// two-sided application of I - tau v v^T to the current trailing matrix.
// Both kernels issue all their global loads before their first barrier, so
// that each costs one round trip to memory.
//
// Work arrays per matrix: vw holds V, W and a second copy of V (n x TRI_NB
// each), so that [V W] and [W V] are both contiguous; pt holds the tile
// pieces of p, one row of n per slot; sq the partial sums of squares, one
// per 64 rows.
constexpr int COL_R = 64;  // rows per workgroup of k_tri_col (4 lanes per row)

// Four lanes per row r >= j: lane k of a row takes the V / W columns and the
// slots of p congruent to k mod 4.  c = panel position of column j; upd = 0
// only finishes W[:, c-1] (end of panel).  nslot / ntp: slots of p and
// partial sums of p^T v left by the previous column's k_tri_symv.
template <int LB>
__global__ __launch_bounds__(256) void k_tri_col(DMat<double> A, int64_t n, int64_t j, int c,
                                                 int upd, double* vw, const double* tauv,
                                                 const double* pt, int64_t pts, int nslot,
                                                 const double* red, double* acol, double* dv,
                                                 double* sq, int64_t sqs, const double* ptvp,
                                                 int64_t ptvs, int ntp) {
  constexpr int NQ = TRI_NB / 4;
  __shared__ double Vj[TRI_NB], Wj[TRI_NB], xs[TRI_NB], ys[TRI_NB], rs[8], pjs[1];
  const int b = blockIdx.y, t = threadIdx.x, k = t & 3, lane = t & 63, wave = t >> 6;
  DMat<double> a = A.item(b);
  double* V = vw + (int64_t)b * n * 3 * TRI_NB;
  double* W = V + n * TRI_NB;
  const double* rd = red + (int64_t)b * (2 * TRI_NB + 2);
  const double* p = pt + (int64_t)b * pts;
  const int64_t r = j + (int64_t)blockIdx.x * COL_R + (t >> 2);
  const bool act = r < n;
  // every global load first: this row of V and W, its slots of p, column j,
  // the partial sums of p^T v, p at row j, and the inputs of W[:, c-1]
  double vr[NQ], wr[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = 4 * i + k;
    vr[i] = (act && q < c) ? V[r + q * n] : 0.0;
    wr[i] = (act && q < c - 1) ? W[r + q * n] : 0.0;
  }
  double pr = 0.0, ps = 0.0, pjp = 0.0, tp = 0.0;
  if (c >= 1) {
    // (blocks of LB independent loads per lane, one wait each: up to 4 LB
    // slots and 256 LB partial sums per round; every round is a memory round
    // trip, so a single large matrix, whose few workgroups leave registers to
    // spare, takes LB = 32)
    if (act) {
      for (int s0 = k; s0 < nslot; s0 += 4 * LB) {
        double pv[LB];
#pragma unroll
        for (int i = 0; i < LB; ++i)
          pv[i] = s0 + 4 * i < nslot ? p[r + (int64_t)(s0 + 4 * i) * n] : 0.0;
#pragma unroll
        for (int i = 0; i < LB; ++i) pr += pv[i];
      }
    }
    const double* pp = ptvp + (int64_t)b * ptvs;
    for (int i0 = t; i0 < ntp; i0 += 256 * LB) {
      double pv[LB];
#pragma unroll
      for (int i = 0; i < LB; ++i) pv[i] = i0 + 256 * i < ntp ? pp[i0 + 256 * i] : 0.0;
#pragma unroll
      for (int i = 0; i < LB; ++i) ps += pv[i];
    }
    if (wave == 1)
      for (int s0 = lane; s0 < nslot; s0 += 256) {
        double pv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          pv[i] = s0 + 64 * i < nslot ? p[j + (int64_t)(s0 + 64 * i) * n] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) pjp += pv[i];
      }
    tp = tauv[(int64_t)b * n + j - 1];
  }
  const double ajr = (act && upd && k == 0) ? a.re[r + j * a.ld] : 0.0;
  if (t < c) {
    Vj[t] = V[j + (int64_t)t * n];
    if (t < c - 1) {
      Wj[t] = W[j + (int64_t)t * n];
      xs[t] = rd[2 + t];
      ys[t] = rd[2 + TRI_NB + t];
    }
  }
  if (c == 0 && act) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q = 4 * i + k;
      V[r + q * n] = 0.0;
      W[r + q * n] = 0.0;
      V[r + (2 * TRI_NB + q) * n] = 0.0;
    }
  }
  pr += __shfl_xor(pr, 1, 64);
  pr += __shfl_xor(pr, 2, 64);
  if (wave == 1) {
    pjp = wave_sum(pjp);
    if (lane == 0) pjs[0] = pjp;
  }
  __syncthreads();
  if (c >= 1) {
    const double ptv = block_sum256(ps, rs);
    double xy = 0;
#pragma unroll 8
    for (int q = 0; q < c - 1; ++q) xy += xs[q] * ys[q];
    const double al = -0.5 * tp * tp * (ptv - 2.0 * xy);
    if (t == 0) {
      double acc = pjs[0];
      for (int q = 0; q < c - 1; ++q) acc -= Vj[q] * xs[q] + Wj[q] * ys[q];
      Wj[c - 1] = tp * acc + al * Vj[c - 1];
    }
    // W[r, c-1]
    double part = 0.0, vl = 0.0;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q = 4 * i + k;
      if (q < c - 1) part += vr[i] * xs[q] + wr[i] * ys[q];
      if (q == c - 1) vl = vr[i];
    }
    part += __shfl_xor(part, 1, 64);
    part += __shfl_xor(part, 2, 64);
    vl = __shfl(vl, (lane & ~3) | ((c - 1) & 3), 64);
    const double wc = tp * (pr - part) + al * vl;
#pragma unroll
    for (int i = 0; i < NQ; ++i)
      if (4 * i + k == c - 1) wr[i] = wc;
    if (act && k == 0) W[r + (int64_t)(c - 1) * n] = wc;
    __syncthreads();
  }
  if (!upd) return;
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = 4 * i + k;
    if (q < c) part += vr[i] * Wj[q] + wr[i] * Vj[q];
  }
  part += __shfl_xor(part, 1, 64);
  part += __shfl_xor(part, 2, 64);
  const double ar = __shfl(ajr, lane & ~3, 64) - part;
  if (act && k == 0) {
    acol[(int64_t)b * n + r] = ar;
    if (r == j) dv[(int64_t)b * n + j] = ar;
  }
  const double s2 = block_sum256((act && k == 0 && r >= j + 2) ? ar * ar : 0.0, rs);
  if (t == 0) sq[(int64_t)b * sqs + blockIdx.x] = s2;
}

// Reflector of column j and the tile pieces of p = T v for the trailing
// block T = A[j1:n, j1:n] (j1 = j + 1) from its lower triangle.  Tiles of
// 64 x 64 are anchored at jb (j1, or j1 rounded down to even when the
// columns allow 16-byte loads; rows and columns below j1 are masked).
// Workgroup g < ntile owns lower tile (I, J), I >= J, of the nbt x nbt tile
// grid: it writes T_IJ v_J (rows of block I) to slot J and T_IJ^T v_I (rows
// of block J) to slot I + 1; a diagonal tile gives its strict lower part to
// slot I and its lower part with the diagonal to slot I + 1.  Every row of
// block R thus gets one value in each slot 0 .. nbt, and p = their sum.  The
// workgroup's share of p^T v goes to ptvp[g].  Tiles are numbered column by
// column, backwards for every other column j: a mat-vec starts on the tiles
// the previous one read last, which the caches still hold.  Within a tile,
// each wave owns 16 columns and each half-wave one column per step, two rows
// per lane.  The reflector is v = e_j1 + scale u with u the entries of column
// j below row j1, so the loads of u and of the tile do not wait for scale;
// every load of a workgroup is issued before its first wait.
template <bool VEC>
__global__ __launch_bounds__(256) void k_tri_symv(DMat<double> A, int64_t n, int64_t j, int c,
                                                  double* vw, double* ev, double* tauv,
                                                  const double* acol, const double* sq, int nsq,
                                                  int64_t sqs, int64_t jb, int ntile, double* red,
                                                  double* pt, int64_t pts, double* ptvp,
                                                  int64_t ptvs, int nbt, int rev) {
  __shared__ double hh[4];
  __shared__ double rsl[8][TRI_TB];
  __shared__ double cdl[TRI_TB];
  __shared__ double urow[TRI_TB], ucol[TRI_TB];
  __shared__ double rs[8];
  const int b = blockIdx.y, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = (int)blockIdx.x;
  DMat<double> a = A.item(b);
  const double* ac = acol + (int64_t)b * n;
  const int64_t j1 = j + 1;
  // tile coordinates: lower tiles numbered column by column (column J starts
  // at J nbt - J (J - 1) / 2), backwards when rev
  int I = 0, J = 0;
  const bool tile = g < ntile;
  if (tile) {
    const int gg = rev ? ntile - 1 - g : g;
    auto off = [&](int cj) { return cj * nbt - cj * (cj - 1) / 2; };
    const double q = 2.0 * nbt + 1.0;
    J = (int)((q - sqrt(q * q - 8.0 * (double)gg)) * 0.5);
    J = J < 0 ? 0 : (J > nbt - 1 ? nbt - 1 : J);
    while (J + 1 <= nbt - 1 && off(J + 1) <= gg) ++J;
    while (J > 0 && off(J) > gg) --J;
    I = J + (gg - off(J));
  }
  const int64_t rb = jb + (int64_t)TRI_TB * I, cb = jb + (int64_t)TRI_TB * J;
  const int h = lane >> 5;
  const int64_t r0 = rb + 2 * (lane & 31);
  // all global loads first, with no wait between them: the tile, the
  // entries of u at the tile's rows and columns, the partial sums of
  // squares (four per lane of wave 0; longer columns loop over the rest)
  double2 x[8];
  double dot = 0.0, y1 = 0.0;
  // u at row r: an unconditional load from a clamped index, then a select
  if (tile) {
    // a tile inside the trailing block and the matrix takes unmasked loads
    // at a fixed column stride; the others mask columns before j1 or past n
    // and rows past n
    const bool full = VEC && cb >= j1 && cb + TRI_TB <= n && rb + TRI_TB <= n;
    if (full) {
      const double* p0 = a.re + (cb + 16 * wave + h) * a.ld + r0;
      const int64_t cs = 2 * a.ld;
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = *reinterpret_cast<const double2*>(p0 + i * cs);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t q = cb + 16 * wave + 2 * i + h;
        const bool qok = q >= j1 && q < n;
        const double* colp = a.re + (qok ? q : j1) * a.ld;
        double2 v2 = make_double2(0.0, 0.0);
        if (VEC && qok && r0 + 1 < n) {
          v2 = *reinterpret_cast<const double2*>(colp + r0);
        } else {
          if (qok && r0 < n) v2.x = colp[r0];
          if (qok && r0 + 1 < n) v2.y = colp[r0 + 1];
        }
        x[i] = v2;
      }
    }
  } else {
    // W[:, e]^T u (e < c) or V[:, e - c]^T u, and the entries at row j1
    const int e = g - ntile;
    const double* V = vw + (int64_t)b * n * 3 * TRI_NB;
    const double* y = e < c ? V + n * TRI_NB + (int64_t)e * n : V + (int64_t)(e - c) * n;
    for (int64_t r0 = j1 + 1 + t; r0 < n; r0 += 8 * 256) {
      double yv[8], av[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t r = r0 + 256 * i;
        yv[i] = r < n ? y[r] : 0.0;
        av[i] = r < n ? ac[r] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) dot += yv[i] * av[i];
    }
    if (t == 0) y1 = y[j1];
  }
  // every lane loads (no branch, so no wait before the loads are all
  // issued); the masks are applied once the values are used
  const int64_t ru = rb + (t & (TRI_TB - 1)), cu = cb + (t & (TRI_TB - 1));
  const double ua = ac[ru < n ? ru : n - 1], ub = ac[cu < n ? cu : n - 1];
  const double* sqb = sq + (int64_t)b * sqs;
  double sqv[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) sqv[k] = sqb[min(lane + 64 * k, nsq - 1)];
  if (t < TRI_TB) {
    urow[t] = (ru > j1 && ru < n) ? ua : 0.0;
    ucol[t] = (cu > j1 && cu < n) ? ub : 0.0;
  }
  double s2 = 0.0;
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s2 += lane + 64 * k < nsq ? sqv[k] : 0.0;
    for (int i = lane + 256; i < nsq; i += 64) s2 += sqb[i];
  }
  const double alpha = ac[j1];
  if (wave == 0) {
    s2 = wave_sum(s2);
    if (lane == 0) {
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
  }
  __syncthreads();
  const double scale = hh[2];
  if (g == 0 && t == 0) {
    ev[(int64_t)b * n + j] = hh[1];
    tauv[(int64_t)b * n + j] = hh[0];
  }
  if (!tile) {
    const int e = g - ntile;
    dot = block_sum256(dot, rs);
    if (t == 0)
      red[(int64_t)b * (2 * TRI_NB + 2) + (e < c ? 2 + e : 2 + TRI_NB + e - c)] = scale * dot + y1;
    return;
  }
  auto vof = [&](int64_t r, double u) -> double { return r == j1 ? 1.0 : scale * u; };
  // 32-bit tile-local indices against uniform thresholds: local row lr is
  // row rb + lr, local column qc column cb + qc
  auto clampi = [](int64_t v) { return (int)(v < -1 ? -1 : (v > 2 * TRI_TB ? 2 * TRI_TB : v)); };
  const int lr = 2 * (lane & 31);
  const int rfirst = clampi(j1 - rb);       // local rows >= rfirst are >= j1
  const int cone = clampi(j1 - cb);         // local column of row / column j1
  const int dq = (int)(rb - cb);            // r > q  <=>  lr - qc > -dq
  const double vi0 = lr == rfirst ? 1.0 : scale * urow[lr];
  const double vi1 = lr + 1 == rfirst ? 1.0 : scale * urow[lr + 1];
  const double m0 = lr >= rfirst ? 1.0 : 0.0, m1 = lr + 1 >= rfirst ? 1.0 : 0.0;
  double rs0 = 0.0, rs1 = 0.0;
  double cp[8];  // this lane's part of the column sums of its 8 columns
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int qc = 16 * wave + 2 * i + h;
    const double vq = qc == cone ? 1.0 : scale * ucol[qc];
    // the strict lower part feeds the row sums, the lower part with the
    // diagonal the column sums; rows below j1 are masked
    const double x0 = m0 * x[i].x, x1 = m1 * x[i].y;
    const int d0 = lr - qc + dq;              // (rb + lr) - (cb + qc)
    rs0 += (d0 > 0 ? x0 : 0.0) * vq;
    rs1 += (d0 + 1 > 0 ? x1 : 0.0) * vq;
    cp[i] = (d0 >= 0 ? x0 : 0.0) * vi0 + (d0 + 1 >= 0 ? x1 : 0.0) * vi1;
  }
  // column sums over the 32 lanes of each half-wave by halving exchanges:
  // after the exchanges across lane bits 4, 3 and 2 a lane holds one column,
  // i = 4 b4 + 2 b3 + b2, summed over 8 lanes; bits 1 and 0 finish the sum
  {
    const int l = lane & 31;
    const bool b4 = l & 16, b3 = l & 8, b2 = l & 4;
    double d4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double snd = b4 ? cp[k] : cp[k + 4];
      d4[k] = (b4 ? cp[k + 4] : cp[k]) + __shfl_xor(snd, 16, 64);
    }
    double d2[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double snd = b3 ? d4[k] : d4[k + 2];
      d2[k] = (b3 ? d4[k + 2] : d4[k]) + __shfl_xor(snd, 8, 64);
    }
    double f = (b2 ? d2[1] : d2[0]) + __shfl_xor(b2 ? d2[0] : d2[1], 4, 64);
    f += __shfl_xor(f, 2, 64);
    f += __shfl_xor(f, 1, 64);
    if ((l & 3) == 0) cdl[16 * wave + 2 * (l >> 2) + h] = f;
  }
  rsl[2 * wave + h][2 * (lane & 31)] = rs0;
  rsl[2 * wave + h][2 * (lane & 31) + 1] = rs1;
  if (I == J && t < TRI_TB) {
    // the reflector: V[:, c] (both copies) and column j of A (rows >= j + 2)
    const int64_t r = rb + t;
    if (r >= j1 && r < n) {
      const double v = vof(r, urow[t]);
      double* V = vw + (int64_t)b * n * 3 * TRI_NB;
      V[r + (int64_t)c * n] = v;
      V[r + (int64_t)(2 * TRI_NB + c) * n] = v;
      if (r >= j + 2) a.re[r + j * a.ld] = v;
    }
  }
  __syncthreads();
  double share = 0.0;
  if (t < TRI_TB) {
    double rsum = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) rsum += rsl[k][t];
    const double cd = cdl[t];
    double* pb = pt + (int64_t)b * pts;
    const int64_t r = rb + t, q = cb + t;
    if (r < n) pb[(int64_t)J * n + r] = rsum;
    if (q < n) pb[(int64_t)(I + 1) * n + q] = cd;
    share = vof(r, urow[t]) * rsum + vof(q, ucol[t]) * cd;
  }
  if (wave == 0) {
    share = wave_sum(share);
    if (t == 0) ptvp[(int64_t)b * ptvs + g] = share;
  }
}

__global__ void k_tri_fin(DMat<double> A, int64_t n, double* dv, double* ev) {
  const int b = blockIdx.x;
  DMat<double> a = A.item(b);
  if (threadIdx.x == 0) {
    if (n >= 2) {
      dv[b * n + n - 2] = a.re[(n - 2) + (n - 2) * a.ld];
      ev[b * n + n - 2] = a.re[(n - 1) + (n - 2) * a.ld];
    }
    dv[b * n + n - 1] = a.re[(n - 1) + (n - 1) * a.ld];
    ev[b * n + n - 1] = 0.0;
  }
}

static void tridiag_launches(hipStream_t s, DMat<double> A, int64_t n, int batch, TriWork& w) {
  double* vw = w.vw.as<double>();
  const bool vec = A.ld % 2 == 0 && A.bs % 2 == 0 && ((uintptr_t)A.re & 15u) == 0;
  const int64_t nbmax = tri_blocks(n);
  const int64_t pts = (nbmax + 1) * n;                 // pt per matrix
  const int64_t ptvs = nbmax * (nbmax + 1) / 2;        // ptvp per matrix
  const int64_t sqs = (n + COL_R - 1) / COL_R;         // sq per matrix
  // tile anchor and counts of the mat-vec over the trailing block from row j1
  auto anchor = [&](int64_t j1) { return vec ? (j1 & ~(int64_t)1) : j1; };
  auto nblk = [&](int64_t j1) { return (int)((n - anchor(j1) + TRI_TB - 1) / TRI_TB); };
  auto col = [&](int64_t j, int c, int upd) {
    // the previous column's mat-vec covered rows from j
    const int nb = c >= 1 ? nblk(j) : 0;
    dim3 g1((unsigned)((n - j + COL_R - 1) / COL_R), batch);
    (batch == 1 ? k_tri_col<32> : k_tri_col<16>)<<<g1, 256, 0, s>>>(
        A, n, j, c, upd, vw, w.tau.as<double>(), w.pt.as<double>(), pts, nb + 1,
        w.red.as<double>(), w.acol.as<double>(), w.d.as<double>(), w.sq.as<double>(), sqs,
        w.ptvp.as<double>(), ptvs, nb * (nb + 1) / 2);
    RFD_CHECK_LAUNCH();
  };
  const int64_t nred = n - 2;  // columns that get a reflector
  for (int64_t i0 = 0; i0 < nred; i0 += TRI_NB) {
    const int nbp = (int)std::min<int64_t>(TRI_NB, nred - i0);
    for (int c = 0; c < nbp; ++c) {
      const int64_t j = i0 + c;
      col(j, c, 1);
      const int nb = nblk(j + 1);
      const int ntile = nb * (nb + 1) / 2;
      dim3 g2((unsigned)(ntile + 2 * c), batch);
      // algorithmic bytes: the lower triangle of the trailing block, the
      // column, p, V / W columns
      const double nt = (double)(n - j - 1);
      KernelAccount::Scope acct(s, KA_TRI_SYMV, 2.0 * nt * nt * batch,
                                8.0 * (0.5 * nt * (nt + 1.0) + 4.0 * nt + 4.0 * c * nt) * batch);
      hipExtLaunchKernelGGL(vec ? k_tri_symv<true> : k_tri_symv<false>, g2, dim3(256), 0, s,
                            acct.start(), acct.stop(), 0, A, n, j, c, vw, w.e.as<double>(),
                            w.tau.as<double>(), (const double*)w.acol.as<double>(),
                            (const double*)w.sq.as<double>(),
                            (int)((n - j + COL_R - 1) / COL_R), sqs, anchor(j + 1), ntile,
                            w.red.as<double>(), w.pt.as<double>(), pts, w.ptvp.as<double>(),
                            ptvs, nb, (int)(j & 1));
      RFD_CHECK_LAUNCH();
    }
    // finish W's last column, then the lower triangle of the trailing block
    // takes the panel's update A -= [V W] [W V]^T (columns beyond the panel
    // are zero)
    const int64_t i1 = i0 + nbp;
    col(i1, nbp, 0);
    const int64_t m = n - i1;
    DMat<double> VW{vw + i1, nullptr, n, n * 3 * TRI_NB};
    DMat<double> WV{vw + n * TRI_NB + i1, nullptr, n, n * 3 * TRI_NB};
    DMat<double> Cm = A.sub(i1, i1);
    gemm_lower<double>(s, false, true, m, 2 * TRI_NB, -1.0, VW, WV, 1.0, Cm, batch);
  }
  k_tri_fin<<<batch, 64, 0, s>>>(A, n, w.d.as<double>(), w.e.as<double>());
  RFD_CHECK_LAUNCH();
}

void sy_tridiag(hipStream_t s, DMat<double> A, int64_t n, int batch, TriWork& w) {
  if (n <= 0 || batch <= 0) return;
  w.reserve(n, batch);
  tridiag_launches(s, A, n, batch, w);
}

// ---------------------------------------------------------------------------
// Sturm counts and bisection.
// ---------------------------------------------------------------------------
// 1 / q from the hardware reciprocal estimate and two Newton steps (each
// r <- r + r (1 - q r) doubles the correct bits), about 1 ulp: the Sturm
// recurrence stays backward stable and its dependent chain is shorter than a
// correctly rounded division's.
__device__ inline double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

__device__ inline int sturm(const double* d, const double* e, int64_t n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
  for (int64_t i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] * rcp_nr(q);
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// The same count from d and the squares e2[i] = e[i]^2 (bitwise the same
// products as above), read from shared memory by the kernels below.
__device__ inline int sturm_sq(const double* d, const double* e2, int64_t n, double x,
                               double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
  for (int64_t i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] * rcp_nr(q);
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// Tridiagonals up to this order are staged in shared memory (d and e^2,
// 16 bytes a row) by the Sturm-count kernels: the recurrence then waits on
// no global load.
constexpr int64_t STURM_LDS_N = 4096;

// Copies d and e^2 of one item into shared memory (all threads of the
// workgroup; ends with a barrier).
__device__ inline void stage_tridiag(const double* d, const double* e, int64_t n, double* sd,
                                     double* se2) {
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    sd[r] = d[r];
    se2[r] = r + 1 < n ? e[r] * e[r] : 0.0;
  }
  __syncthreads();
}

// One wavefront per item: pivmin from the largest e^2 (a max, so the order
// of the reduction does not matter), then a count per shift, lanes over x.
__global__ __launch_bounds__(64) void k_sturm(const double* dv, const double* ev, int64_t n,
                                              int batch, const double* x, int nx, int* cnt) {
  extern __shared__ double st_sh[];
  const int b = blockIdx.x, lane = threadIdx.x;
  const double* d = dv + (int64_t)b * n;
  const double* e = ev + (int64_t)b * n;
  const bool staged = n <= STURM_LDS_N;
  if (staged) stage_tridiag(d, e, n, st_sh, st_sh + n);
  double m = 1.0;
  for (int64_t r = lane; r + 1 < n; r += 64) m = fmax(m, e[r] * e[r]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  const double pivmin = SAFMIN * m / EPS;
  for (int t = lane; t < nx; t += 64) {
    const double xv = x[(int64_t)b * nx + t];
    cnt[(int64_t)b * nx + t] =
        staged ? sturm_sq(st_sh, st_sh + n, n, xv, pivmin) : sturm(d, e, n, xv, pivmin);
  }
}

void sturm_counts(hipStream_t s, const TriWork& w, int64_t n, int batch, const double* x, int nx,
                  int* cnt) {
  if (batch <= 0 || nx <= 0 || n <= 0) return;
  const size_t sh = n <= STURM_LDS_N ? sizeof(double) * 2 * n : 0;
  k_sturm<<<batch, 64, sh, s>>>(w.d.as<double>(), w.e.as<double>(), n, batch, x, nx, cnt);
  RFD_CHECK_LAUNCH();
}

// Multisection: one wavefront per eigenvalue; each lane takes the Sturm
// count at one of 64 interior points of the current bracket, and the bracket
// shrinks to the two neighbouring points around the wanted index.
__global__ __launch_bounds__(256) void k_bisect(const double* dv, const double* ev, int64_t n,
                                                int batch, const int* lo, const int* num,
                                                int maxnum, double* lam, int64_t ld_lam) {
  extern __shared__ double bi_sh[];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.y;
  const double* d = dv + (int64_t)b * n;
  const double* e = ev + (int64_t)b * n;
  // the workgroup's four eigenvalues belong to one item: its d and e^2 go to
  // shared memory once
  const bool staged = n <= STURM_LDS_N;
  if (staged) stage_tridiag(d, e, n, bi_sh, bi_sh + n);
  if (i >= maxnum || i >= num[b]) return;
  double gl = INFINITY, gu = -INFINITY, em = 1.0;
  for (int64_t r = lane; r < n; r += 64) {
    const double off = (r > 0 ? fabs(e[r - 1]) : 0.0) + (r + 1 < n ? fabs(e[r]) : 0.0);
    gl = fmin(gl, d[r] - off);
    gu = fmax(gu, d[r] + off);
    if (r + 1 < n) em = fmax(em, e[r] * e[r]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, o, 64));
    gu = fmax(gu, __shfl_xor(gu, o, 64));
    em = fmax(em, __shfl_xor(em, o, 64));
  }
  const double pivmin = SAFMIN * em / EPS;
  const double tnorm = fmax(fabs(gl), fabs(gu));
  gl -= 2.0 * EPS * tnorm * n + 1e-300;
  gu += 2.0 * EPS * tnorm * n + 1e-300;
  const int k = lo[b] + i;  // want the k-th smallest (0-based): count(l) <= k < count(u)
  double l = gl, u = gu;
  for (int it = 0; it < 64; ++it) {
    if (u - l <= 2.0 * EPS * fmax(fabs(l), fabs(u)) + 4.0 * pivmin) break;
    const double x = l + (u - l) * ((double)(lane + 1) / 65.0);
    const int cnt = staged ? sturm_sq(bi_sh, bi_sh + n, n, x, pivmin) : sturm(d, e, n, x, pivmin);
    const unsigned long long m = __ballot(cnt > k);
    double nl = l, nu = u;
    if (m == 0ull) {
      nl = __shfl(x, 63, 64);
    } else {
      const int f = __ffsll((long long)m) - 1;
      nu = __shfl(x, f, 64);
      if (f > 0) nl = __shfl(x, f - 1, 64);
    }
    if (nl == l && nu == u) break;
    l = nl;
    u = nu;
  }
  if (lane == 0) lam[(int64_t)b * ld_lam + i] = 0.5 * (l + u);
}

void bisect(hipStream_t s, const TriWork& w, int64_t n, int batch, const int* lo, const int* num,
            int maxnum, double* lam, int64_t ld_lam) {
  if (maxnum <= 0) return;
  dim3 g((unsigned)((maxnum + 3) / 4), batch);
  const size_t sh = n <= STURM_LDS_N ? sizeof(double) * 2 * n : 0;
  k_bisect<<<g, 256, sh, s>>>(w.d.as<double>(), w.e.as<double>(), n, batch, lo, num, maxnum, lam,
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

// Scratch is interleaved over the threads (element r of slot g at r * S + g)
// so that a wavefront's accesses at one step are contiguous.  The
// elimination and the substitutions carry their running values in registers,
// and every loop reads one array and writes another (two vector buffers used
// in turn), so that loads can run ahead of the dependent arithmetic.
constexpr int IV = 32;  // rows per prefetched chunk in the inverse iteration

__global__ __launch_bounds__(64) void k_invit(const double* __restrict__ d0,
                                              const double* __restrict__ e0, int64_t n,
                                              const double* lam, const int* num, const int* clus,
                                              int64_t ld_lam, DMat<double> Y, double* scratch,
                                              int64_t S) {
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i0 >= num[b] || i0 >= ld_lam) return;
  if (clus[(int64_t)b * ld_lam + i0] != i0) return;  // not a cluster head
  const double* __restrict__ d = d0 + (int64_t)b * n;
  const double* __restrict__ e = e0 + (int64_t)b * n;
  const int64_t g = (int64_t)b * ld_lam + i0;
  double* __restrict__ dl = scratch + g;
  double* __restrict__ dd = scratch + n * S + g;
  double* __restrict__ du = scratch + 2 * n * S + g;
  double* __restrict__ du2 = scratch + 3 * n * S + g;
  double* xa = scratch + 4 * n * S + g;
  double* xb = scratch + 5 * n * S + g;
  int* __restrict__ ip = reinterpret_cast<int*>(scratch + 6 * n * S) + g;
  DMat<double> y = Y.item(b);
  double tnorm = 0;
#pragma unroll 8
  for (int64_t r = 0; r < n; ++r)
    tnorm = fmax(tnorm, fabs(d[r]) + (r > 0 ? fabs(e[r - 1]) : 0.0) + (r + 1 < n ? fabs(e[r]) : 0.0));
  const double pert = 10.0 * EPS * fmax(tnorm, 1e-300);
  const double tiny = EPS * fmax(tnorm, 1e-300);
  auto fix = [&](double v) { return fabs(v) < EPS * tnorm ? (v < 0 ? -tiny : tiny) : v; };
  double prev = -INFINITY;
  for (int i = i0; i < num[b] && clus[(int64_t)b * ld_lam + i] == i0; ++i) {
    double lm = lam[(int64_t)b * ld_lam + i];
    if (lm - prev < pert) lm = prev + pert;
    prev = lm;
    // LU with partial pivoting of T - lm I (as dgttrf); dcur / ucur are the
    // running diagonal and superdiagonal of the row being eliminated
    double dcur = d[0] - lm, ucur = n > 1 ? e[0] : 0.0;
    auto elim = [&](int64_t r, double er, double dn, double un) {
      if (fabs(dcur) >= fabs(er)) {
        const double f = (dcur != 0.0) ? er / dcur : 0.0;
        ip[r * S] = (int)r;
        dl[r * S] = f;
        dd[r * S] = fix(dcur);
        du[r * S] = ucur;
        du2[r * S] = 0.0;
        dcur = dn - f * ucur;
        ucur = un;
      } else {
        const double f = dcur / er;
        ip[r * S] = (int)r + 1;
        dl[r * S] = f;
        dd[r * S] = fix(er);
        du[r * S] = dn;
        du2[r * S] = un;
        dcur = ucur - f * dn;
        ucur = -f * un;
      }
    };
    int64_t r0 = 0;
    // chunks of IV rows: the chunk's inputs are loaded before its recurrence
    for (; r0 + IV + 1 < n; r0 += IV) {
      double er[IV], dn[IV], un[IV];
#pragma unroll
      for (int u = 0; u < IV; ++u) {
        er[u] = e[r0 + u];
        dn[u] = d[r0 + u + 1] - lm;
        un[u] = e[r0 + u + 1];
      }
#pragma unroll
      for (int u = 0; u < IV; ++u) elim(r0 + u, er[u], dn[u], un[u]);
    }
    for (int64_t r = r0; r + 1 < n; ++r) {
      const double er = e[r];
      const double dn = d[r + 1] - lm;
      const double un = (r + 2 < n) ? e[r + 1] : 0.0;
      if (fabs(dcur) >= fabs(er)) {
        const double f = (dcur != 0.0) ? er / dcur : 0.0;
        ip[r * S] = (int)r;
        dl[r * S] = f;
        dd[r * S] = fix(dcur);
        du[r * S] = ucur;
        du2[r * S] = 0.0;
        dcur = dn - f * ucur;
        ucur = un;
      } else {
        const double f = dcur / er;
        ip[r * S] = (int)r + 1;
        dl[r * S] = f;
        dd[r * S] = fix(er);
        du[r * S] = dn;
        du2[r * S] = un;
        dcur = ucur - f * dn;
        ucur = -f * un;
      }
    }
    dd[(n - 1) * S] = fix(dcur);
#pragma unroll 8
    for (int64_t r = 0; r < n; ++r) xa[r * S] = hash_unit((uint64_t)r + 1, (uint64_t)i + 7919ull * b);
    // three solves from a random start; the vector is normalised once at
    // the end (one solve grows it by at most ~1 / (eps ||T||), far from
    // overflow after three)
    for (int it = 0; it < 3; ++it) {
      {  // L with the row interchanges: xa -> xb, running value in xc
        const double* __restrict__ src = xa;
        double* __restrict__ dst = xb;
        double xc = src[0];
        int64_t q0 = 0;
        for (; q0 + IV < n; q0 += IV) {
          double xn[IV], f[IV];
          int pv[IV];
#pragma unroll
          for (int u = 0; u < IV; ++u) {
            xn[u] = src[(q0 + u + 1) * S];
            f[u] = dl[(q0 + u) * S];
            pv[u] = ip[(q0 + u) * S];
          }
#pragma unroll
          for (int u = 0; u < IV; ++u) {
            if (pv[u] == q0 + u) {
              dst[(q0 + u) * S] = xc;
              xc = xn[u] - f[u] * xc;
            } else {
              dst[(q0 + u) * S] = xn[u];
              xc = xc - f[u] * xn[u];
            }
          }
        }
        for (int64_t r = q0; r + 1 < n; ++r) {
          const double xn = src[(r + 1) * S];
          const double f = dl[r * S];
          if (ip[r * S] == r) {
            dst[r * S] = xc;
            xc = xn - f * xc;
          } else {
            dst[r * S] = xn;
            xc = xc - f * xn;
          }
        }
        dst[(n - 1) * S] = xc;
      }
      {  // U (two superdiagonals): xb -> xa, x1 = x[r + 1], x2 = x[r + 2]
        const double* __restrict__ src = xb;
        double* __restrict__ dst = xa;
        double x1 = src[(n - 1) * S] / dd[(n - 1) * S], x2 = 0.0;
        dst[(n - 1) * S] = x1;
        int64_t q1 = n - 2;
        for (; q1 - (IV - 1) >= 0; q1 -= IV) {
          double sv[IV], uu[IV], u2[IV], dv[IV];
#pragma unroll
          for (int u = 0; u < IV; ++u) {
            sv[u] = src[(q1 - u) * S];
            uu[u] = du[(q1 - u) * S];
            u2[u] = du2[(q1 - u) * S];
            dv[u] = dd[(q1 - u) * S];
          }
#pragma unroll
          for (int u = 0; u < IV; ++u) {
            const double v = (sv[u] - uu[u] * x1 - u2[u] * x2) / dv[u];
            dst[(q1 - u) * S] = v;
            x2 = x1;
            x1 = v;
          }
        }
        for (int64_t r = q1; r >= 0; --r) {
          const double v = (src[r * S] - du[r * S] * x1 - du2[r * S] * x2) / dd[r * S];
          dst[r * S] = v;
          x2 = x1;
          x1 = v;
        }
      }
      // orthogonalise against the previous members of the cluster (twice);
      // each pass moves the vector to the other buffer
      for (int pass = 0; pass < 2; ++pass)
        for (int q = i0; q < i; ++q) {
          const double* __restrict__ yq = y.re + (int64_t)q * y.ld;
          const double* __restrict__ src = xa;
          double* __restrict__ dst = xb;
          double dt = 0;
#pragma unroll 8
          for (int64_t r = 0; r < n; ++r) dt += yq[r] * src[r * S];
#pragma unroll 8
          for (int64_t r = 0; r < n; ++r) dst[r * S] = src[r * S] - dt * yq[r];
          double* t = xa;
          xa = xb;
          xb = t;
        }
    }
    // unit norm, sign convention: largest-magnitude component positive (the
    // norm is accumulated on a scaled copy so that a large vector cannot
    // overflow the sum of squares)
    const double* __restrict__ src = xa;
    int64_t am = 0;
    double best = -1.0;
#pragma unroll 8
    for (int64_t r = 0; r < n; ++r) {
      const double a = fabs(src[r * S]);
      if (a > best) {
        best = a;
        am = r;
      }
    }
    const double sc = best > 0 ? 1.0 / best : 0.0;
    double nrm = 0;
#pragma unroll 8
    for (int64_t r = 0; r < n; ++r) {
      const double v = src[r * S] * sc;
      nrm += v * v;
    }
    nrm = sqrt(nrm);
    const double f = (src[am * S] < 0 ? -1.0 : 1.0) * (nrm > 0 ? sc / nrm : 0.0);
    double* __restrict__ yi = y.re + (int64_t)i * y.ld;
#pragma unroll 8
    for (int64_t r = 0; r < n; ++r) yi[r] = f * src[r * S];
  }
}

void inverse_iteration(hipStream_t s, const TriWork& w, int64_t n, int batch, const double* lam,
                       const int* num, const int* clus, int64_t ld_lam, DMat<double> Y,
                       DevBuf& scratch) {
  if (ld_lam <= 0) return;
  const int64_t S = ld_lam * (int64_t)batch;  // interleaving stride (slots)
  scratch.alloc(sizeof(double) * 7 * n * S);
  dim3 g(grid1(ld_lam, 64), batch);
  k_invit<<<g, 64, 0, s>>>(w.d.as<double>(), w.e.as<double>(), n, lam, num, clus, ld_lam, Y,
                           scratch.as<double>(), S);
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Back-transformation.  Q = H_0 H_1 ... H_{n-3}; the reflectors of one panel
// of TRI_NB are combined as I - V T V^T (T upper triangular, built column by
// column from tau and the Gram matrix V^T V), and Y <- Q Y applies the panels
// last to first as Y -= V (T (V^T Y)), three GEMMs per panel.
// ---------------------------------------------------------------------------
// V[r, q] (rows i0 + 1 .. n - 1 of the panel's reflectors, explicit unit
// entry, zeros above it)
// Reflectors are applied in blocks of WY_NB (compact WY: I - V T V^T).

// V (m x WY_NB, m = n - i0 - 1) of the block of reflectors i0 .. i0 + nbp - 1,
// with the unit entries explicit and zero columns beyond nbp.
__global__ void k_wy_v(DMat<double> A, int64_t n, int64_t i0, int nbp, double* V) {
  const int b = blockIdx.y;
  DMat<double> a = A.item(b);
  const int64_t m = n - i0 - 1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * WY_NB) return;
  const int64_t rr = e % m, q = e / m;
  const int64_t r = i0 + 1 + rr, j = i0 + q;
  double v = 0.0;
  if (q < nbp) v = (r == j + 1) ? 1.0 : (r > j + 1 ? a.re[r + j * a.ld] : 0.0);
  V[(int64_t)b * m * WY_NB + rr + q * m] = v;
}

// T (WY_NB x WY_NB, upper) of the block from tau and G = V^T V.  The
// recurrence T[k][k] = tau_k, T[0:k, k] = -tau_k T[0:k, 0:k] G[0:k, k] runs
// on the four diagonal 32 x 32 blocks at once (a group of 64 threads each);
// then block column b takes T[0:32b, blk b] = -T[0:32b, 0:32b] G[0:32b, blk b]
// T_bb, which is the same recurrence applied a block at a time.  One
// workgroup of 256 per item; the upper triangle of T stays in shared memory
// (packed by columns) until it is written out whole.  Every operand read in
// a dependent chain (the block's tau, the diagonal blocks of G, the block
// column of G of each merge) is staged in shared memory first, with all its
// global loads in flight together.
constexpr int WY_SB = 32;
__global__ __launch_bounds__(256) void k_wy_t(const double* G, const double* tauv, int64_t n,
                                              int64_t i0, int nbp, double* T) {
  constexpr int NS = WY_NB / WY_SB;
  __shared__ double Ts[NS][WY_SB][WY_SB + 1];
  __shared__ double Tp[WY_NB * (WY_NB + 1) / 2];
  __shared__ double tl[WY_NB];
  // the diagonal blocks of G, later a block column of G, then X (each fits
  // in the larger of the two shapes)
  constexpr int SH = NS * WY_SB * (WY_SB + 1) > (WY_NB - WY_SB) * (WY_SB + 1)
                         ? NS * WY_SB * (WY_SB + 1)
                         : (WY_NB - WY_SB) * (WY_SB + 1);
  __shared__ double sh[SH];
  auto Gd = [&](int a, int r, int c) -> double& { return sh[(a * WY_SB + r) * (WY_SB + 1) + c]; };
  auto X = [&](int r, int c) -> double& { return sh[r * (WY_SB + 1) + c]; };
  auto Tu = [&](int r, int c) -> double& { return Tp[c * (c + 1) / 2 + r]; };  // r <= c
  const int b = blockIdx.x, t = threadIdx.x;
  const int grp = t / 64, lt = t % 64;
  const double* g = G + (int64_t)b * WY_NB * WY_NB;
  double* To = T + (int64_t)b * WY_NB * WY_NB;
  for (int e = t; e < NS * WY_SB * (WY_SB + 1); e += 256) (&Ts[0][0][0])[e] = 0.0;
  for (int e = t; e < WY_NB * (WY_NB + 1) / 2; e += 256) Tp[e] = 0.0;
  if (t < WY_NB) tl[t] = t < nbp ? tauv[(int64_t)b * n + i0 + t] : 0.0;
  {
    constexpr int NE = NS * WY_SB * WY_SB / 256;
    double gv[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = t + 256 * i;
      const int a = e / (WY_SB * WY_SB), r = e % WY_SB, c = (e / WY_SB) % WY_SB;
      gv[i] = g[(a * WY_SB + r) + (int64_t)(a * WY_SB + c) * WY_NB];
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = t + 256 * i;
      const int a = e / (WY_SB * WY_SB), r = e % WY_SB, c = (e / WY_SB) % WY_SB;
      Gd(a, r, c) = gv[i];
    }
  }
  __syncthreads();
  // diagonal blocks: group grp owns block grp (reflectors k0 + k)
  const int k0 = grp * WY_SB;
  for (int k = 0; k < WY_SB; ++k) {
    const double tk = tl[k0 + k];
    double v = 0.0;
    if (lt < k) {
#pragma unroll 8
      for (int q = lt; q < k; ++q) v += Ts[grp][lt][q] * Gd(grp, q, k);
      v *= -tk;
    }
    __syncthreads();
    if (lt < k) Ts[grp][lt][k] = v;
    if (lt == k) Ts[grp][k][k] = tk;
    __syncthreads();
  }
  for (int e = t; e < NS * WY_SB * WY_SB; e += 256) {
    const int a = e / (WY_SB * WY_SB), r = e % WY_SB, c = (e / WY_SB) % WY_SB;
    if (r <= c) Tu(a * WY_SB + r, a * WY_SB + c) = Ts[a][r][c];
  }
  __syncthreads();
  // off-diagonal block columns
  constexpr int NX = (WY_NB - WY_SB) * WY_SB / 256;  // entries of X per thread, at most
  for (int bc = 1; bc < NS; ++bc) {
    const int c0 = bc * WY_SB, rows = c0;
    // G[0:c0, blk] into shared memory (sh is free: the diagonal blocks of G
    // and the previous X are no longer read)
    {
      double gv[NX];
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        const int e = t + 256 * i;
        gv[i] = e < rows * WY_SB ? g[e % rows + (int64_t)(c0 + e / rows) * WY_NB] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        const int e = t + 256 * i;
        if (e < rows * WY_SB) X(e % rows, e / rows) = gv[i];
      }
    }
    __syncthreads();
    // X = G[0:c0, blk] T_bb, formed in registers, then written over G's block
    double xv[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int e = t + 256 * i;
      double acc = 0.0;
      if (e < rows * WY_SB) {
        const int r = e % rows, c = e / rows;
#pragma unroll 8
        for (int q = 0; q <= c; ++q) acc += X(r, q) * Ts[bc][q][c];
      }
      xv[i] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int e = t + 256 * i;
      if (e < rows * WY_SB) X(e % rows, e / rows) = xv[i];
    }
    __syncthreads();
    // T[0:c0, blk] = -T[0:c0, 0:c0] X (upper triangular: column q >= r)
    for (int e = t; e < rows * WY_SB; e += 256) {
      const int r = e % rows, c = e / rows;
      double acc = 0.0;
#pragma unroll 8
      for (int q = r; q < rows; ++q) acc += Tu(r, q) * X(q, c);
      Tu(r, c0 + c) = -acc;
    }
    __syncthreads();
  }
  for (int e = t; e < WY_NB * WY_NB; e += 256) {
    const int r = e % WY_NB, c = e / WY_NB;
    To[e] = r <= c ? Tu(r, c) : 0.0;
  }
}

void wy_triangle(hipStream_t s, const double* G, const double* tau, int64_t ld_tau, int64_t i0,
                 int nbp, double* T, int batch) {
  if (batch <= 0) return;
  if (nbp < 0 || nbp > WY_NB) throw Error(ST_EINVAL, "wy_triangle: block of more than WY_NB reflectors");
  k_wy_t<<<batch, 256, 0, s>>>(G, tau, ld_tau, i0, nbp, T);
  RFD_CHECK_LAUNCH();
}

void back_transform(hipStream_t s, DMat<double> A, TriWork& w, int64_t n, int batch,
                    DMat<double> Y, const int* num, int maxcols) {
  (void)num;
  if (maxcols <= 0 || n < 3) return;
  const int64_t nred = n - 2;
  DevBuf &Vb = w.wv, &Gb = w.wg, &Tb = w.wt, &W1 = w.w1, &W2 = w.w2;
  Vb.alloc(sizeof(double) * (n - 1) * WY_NB * batch);
  Gb.alloc(sizeof(double) * WY_NB * WY_NB * batch);
  Tb.alloc(sizeof(double) * WY_NB * WY_NB * batch);
  W1.alloc(sizeof(double) * WY_NB * maxcols * batch);
  W2.alloc(sizeof(double) * WY_NB * maxcols * batch);
  const int64_t nblk = (nred + WY_NB - 1) / WY_NB;
  for (int64_t pi = nblk - 1; pi >= 0; --pi) {
    const int64_t i0 = pi * WY_NB;
    const int nbp = (int)std::min<int64_t>(WY_NB, nred - i0);
    const int64_t m = n - i0 - 1;
    k_wy_v<<<dim3(grid1(m * WY_NB), batch), 256, 0, s>>>(A, n, i0, nbp, Vb.as<double>());
    RFD_CHECK_LAUNCH();
    DMat<double> Vm{Vb.as<double>(), nullptr, m, m * WY_NB};
    DMat<double> Gm{Gb.as<double>(), nullptr, WY_NB, WY_NB * WY_NB};
    DMat<double> Tm{Tb.as<double>(), nullptr, WY_NB, WY_NB * WY_NB};
    DMat<double> W1m{W1.as<double>(), nullptr, WY_NB, WY_NB * (int64_t)maxcols};
    DMat<double> W2m{W2.as<double>(), nullptr, WY_NB, WY_NB * (int64_t)maxcols};
    DMat<double> Ys = Y.sub(i0 + 1, 0);
    gemm<double>(s, true, false, WY_NB, WY_NB, m, 1.0, Vm, Vm, 0.0, Gm, batch);
    wy_triangle(s, Gb.as<double>(), w.tau.as<double>(), n, i0, nbp, Tb.as<double>(), batch);
    gemm<double>(s, true, false, WY_NB, maxcols, m, 1.0, Vm, Ys, 0.0, W1m, batch);
    gemm<double>(s, false, false, WY_NB, maxcols, WY_NB, 1.0, Tm, W1m, 0.0, W2m, batch);
    gemm<double>(s, false, false, m, maxcols, WY_NB, -1.0, Vm, W2m, 1.0, Ys, batch);
  }
}

}  // namespace rfd
