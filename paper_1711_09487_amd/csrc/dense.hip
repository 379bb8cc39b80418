// Dense batched kernels for gfx950 (the GEMM itself is in gemm.hip): LU
// factorization (blocked, right-looking; the diagonal block is
// factored and inverted in LDS), pivoted panel factorization, triangular
// solves through inverted diagonal blocks, elementwise helpers.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "dense.hpp"

namespace rfd {

// ---------------------------------------------------------------------------
// Per-launch accounting of the GEMM instantiations (key = 8 * fp64 + 4 * complex
// + 2 * ta + tb): HIP events on the launch stream and algorithmic flops.
// ---------------------------------------------------------------------------
KernelAccount& KernelAccount::get() {
  static KernelAccount a;
  return a;
}

KernelAccount::Scope::Scope(hipStream_t s, int key, double flops, double bytes) : s_(s) {
  KernelAccount& k = get();
  if (k.every <= 0 || key < 0 || key >= KA_KEYS) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> g(k.mu);
  // a pseudo-random one launch in `every` (a fixed hash of the launch count):
  // a plain stride would sample a periodic launch sequence at a few phases.
  // Launches of at least KA_ALWAYS_FLOPS are all timed: they are few, and a
  // pair of events costs nothing beside them.
  uint64_t h = (uint64_t)k.count[key]++ * 0x9E3779B97F4A7C15ull + (uint64_t)key;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 29;
  const bool always = flops >= KA_ALWAYS_FLOPS;
  if (!always) ++k.count_small[key];
  if (h % (uint64_t)k.every != 0 && !always) return;
  Rec r;
  r.key = key;
  r.always = always;
  r.flops = flops;
  r.bytes = bytes;
  if (hipEventCreate(&r.a) != hipSuccess) return;
  if (hipEventCreate(&r.b) != hipSuccess) {
    (void)hipEventDestroy(r.a);
    return;
  }
  a_ = r.a;
  b_ = r.b;
  k.recs.push_back(r);
}

void KernelAccount::Scope::mark_start() {
  if (a_) (void)hipEventRecord(a_, s_);
}

void KernelAccount::Scope::mark_stop() {
  if (b_) (void)hipEventRecord(b_, s_);
}

void KernelAccount::collect(double* launches, double* sampled, double* ms, double* flops,
                            double* bytes, int nkeys) {
  std::lock_guard<std::mutex> g(mu);
  // [0]: always-timed launches, [1]: hashed sample of the others
  std::vector<double> n[2], t[2], f[2], b[2];
  for (int q = 0; q < 2; ++q) {
    n[q].assign(KA_KEYS, 0.0);
    t[q].assign(KA_KEYS, 0.0);
    f[q].assign(KA_KEYS, 0.0);
    b[q].assign(KA_KEYS, 0.0);
  }
  for (auto& r : recs) {
    float el = 0;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&el, r.a, r.b) == hipSuccess &&
        r.key < KA_KEYS) {
      const int q = r.always ? 0 : 1;
      n[q][r.key] += 1;
      t[q][r.key] += el;
      f[q][r.key] += r.flops;
      b[q][r.key] += r.bytes;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (int k = 0; k < nkeys; ++k) {
    launches[k] = sampled[k] = ms[k] = flops[k] = bytes[k] = 0;
    if (k >= KA_KEYS) continue;
    const double sc = n[1][k] > 0 ? (double)count_small[k] / n[1][k] : 0.0;
    launches[k] = (double)count[k];
    sampled[k] = n[0][k] + n[1][k];
    ms[k] = t[0][k] + sc * t[1][k];
    flops[k] = f[0][k] + sc * f[1][k];
    bytes[k] = b[0][k] + sc * b[1][k];
  }
  recs.clear();
  for (auto& c : count) c = 0;
  for (auto& c : count_small) c = 0;
}

// ---------------------------------------------------------------------------
// Scalar complex helpers on (re, im) pairs.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void cmul(T ar, T ai, T br, T bi, T& cr, T& ci) {
  cr = ar * br - ai * bi;
  ci = ar * bi + ai * br;
}
template <typename T>
__device__ inline void cinv(T ar, T ai, T& cr, T& ci) {
  // 1 / (ar + i ai), scaled to avoid overflow of |a|^2
  const T s = fabs(ar) > fabs(ai) ? fabs(ar) : fabs(ai);
  const T xr = ar / s, xi = ai / s;
  const T d = (xr * xr + xi * xi) * s;
  cr = xr / d;
  ci = -xi / d;
}

// ---------------------------------------------------------------------------
// Diagonal block: factor an NB x NB block without pivoting in LDS, write it
// back, and write the inverses of its unit-lower and upper triangles.
// One workgroup per batch item.
// ---------------------------------------------------------------------------
template <typename T, bool CPLX>
__device__ inline void fma_sub(T& sr, T& si, T ar, T ai, T br, T bi) {
  if constexpr (CPLX) {
    sr -= ar * br - ai * bi;
    si -= ar * bi + ai * br;
  } else {
    sr -= ar * br;
  }
}

// The NB x NB block at a into F: every thread's 16 loads are issued before
// any is stored, one round trip to memory instead of sixteen.
template <typename T, bool CPLX>
__device__ inline void load_block(T (*F)[NB][NB + 1], const DMat<T>& a, int tid) {
  constexpr int NP = CPLX ? 2 : 1;
  constexpr int PER = NB * NB / 256;
  T vr[PER], vi[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, i = e % NB, j = e / NB;
    vr[q] = a.re[i + j * a.ld];
    vi[q] = CPLX ? a.im[i + j * a.ld] : T(0);
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, i = e % NB, j = e / NB;
    F[0][i][j] = vr[q];
    if constexpr (CPLX) F[NP - 1][i][j] = vi[q];
  }
}

// value of v in lane `lane` (uniform over the wave): a scalar read, not a
// trip through the shared-memory crossbar
template <typename T>
__device__ inline T lane_read(T v, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
  } else {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
}

template <typename T, bool CPLX>
__device__ inline void fma_add(T& sr, T& si, T ar, T ai, T br, T bi) {
  if constexpr (CPLX) {
    sr += ar * br - ai * bi;
    si += ar * bi + ai * br;
  } else {
    sr += ar * br;
  }
}

// Inverses of the unit-lower and the upper triangle of the factored block F
// (NB = 64), both at once, blocked.  X holds the two results in one array as F
// holds the factors: the strictly lower part is L^{-1} (unit diagonal
// implied), the upper part with the diagonal is U^{-1}.
//  * The four 16 x 16 diagonal blocks: wave g inverts block g, lanes 0-15 a
//    column of the lower inverse each, lanes 16-31 a column of the upper one
//    with rows and columns taken in reverse order, which turns the backward
//    substitution into the same forward recurrence (one instruction stream).
//  * Pairs of diagonal blocks are merged into 32 x 32, those into 64 x 64:
//      [A 0; B C]^{-1} = [A^{-1} 0; -C^{-1} B A^{-1}  C^{-1}]
//      [A E; 0 C]^{-1} = [A^{-1} -A^{-1} E C^{-1}; 0 C^{-1}]
//    two products per merge, whose sums run over the nonzero band of the
//    triangular factor only.  E C^{-1} is parked in the lower off-diagonal
//    block of the pair until the upper result has been formed from it.
// A dropped column (semidefinite mode) gets a zero row in Linv, so that the
// panel update leaves a zero row of U beside it.  Tb: 32 x 33 per plane.
template <typename T, bool CPLX>
__device__ __forceinline__ void tri_inverses(T (*F)[NB][NB + 1], T (*X)[NB][NB + 1], T (*Tb)[32][33],
                             DMat<T> Linv, DMat<T> Uinv, const int* dropped = nullptr) {
  constexpr int NP = CPLX ? 2 : 1;
  static_assert(NB == 64, "blocked inversion assumes 64 x 64 blocks");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto ld = [&](T (*Y)[NB][NB + 1], int i, int j, T& vr, T& vi) {
    vr = Y[0][i][j];
    vi = CPLX ? Y[NP - 1][i][j] : T(0);
  };
  auto st = [&](T (*Y)[NB][NB + 1], int i, int j, T vr, T vi) {
    Y[0][i][j] = vr;
    if constexpr (CPLX) Y[NP - 1][i][j] = vi;
  };
  if (lane < 32) {
    const int up = lane >> 4, c = lane & 15, b = 16 * wave;
    T xr[16], xi[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      xr[i] = (i == c) ? T(1) : T(0);
      xi[i] = 0;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      // one row of loads in flight at a time (the whole triangle would not
      // fit in registers)
      __builtin_amdgcn_sched_barrier(0);
      const int ri = up ? 15 - i : i;
      T sr = xr[i], si = xi[i];
#pragma unroll
      for (int t = 0; t < i; ++t) {
        T er, ei;
        ld(F, b + ri, b + (up ? 15 - t : t), er, ei);
        fma_sub<T, CPLX>(sr, si, er, ei, xr[t], xi[t]);
      }
      // unit diagonal for L, the pivot for U
      T dr = T(1), di = T(0);
      if (up) ld(F, b + ri, b + ri, dr, di);
      if constexpr (CPLX) {
        T ir, ii;
        cinv(dr, di, ir, ii);
        cmul(sr, si, ir, ii, xr[i], xi[i]);
      } else {
        xr[i] = sr / dr;
      }
    }
    // lower: rows below the diagonal of column c; upper: rows 15-i <= 15-c
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (up) {
        if (i >= c) st(X, b + 15 - i, b + 15 - c, xr[i], xi[i]);
      } else {
        if (i > c) st(X, b + i, b + c, xr[i], xi[i]);
      }
    }
  }
  __syncthreads();
  for (int w = 16; w <= 32; w *= 2) {
    const int per = w * w, half = (NB / (2 * w)) * per;
    // T_L = B A^{-1} into Tb (row pr w + i), T_U = E C^{-1} parked at X21
    for (int e = tid; e < 2 * half; e += 256) {
      const bool up = e >= half;
      const int q0 = up ? e - half : e;
      const int pr = q0 / per, q = q0 % per, i = q % w, j = q / w, b = 2 * w * pr;
      T sr = 0, si = 0, ar, ai, br, bi;
      if (!up) {
        ld(F, b + w + i, b + j, sr, si);
#pragma unroll 4
        for (int t = j + 1; t < w; ++t) {
          ld(F, b + w + i, b + t, ar, ai);
          ld(X, b + t, b + j, br, bi);
          fma_add<T, CPLX>(sr, si, ar, ai, br, bi);
        }
        Tb[0][pr * w + i][j] = sr;
        if constexpr (CPLX) Tb[NP - 1][pr * w + i][j] = si;
      } else {
#pragma unroll 4
        for (int t = 0; t <= j; ++t) {
          ld(F, b + i, b + w + t, ar, ai);
          ld(X, b + w + t, b + w + j, br, bi);
          fma_add<T, CPLX>(sr, si, ar, ai, br, bi);
        }
        st(X, b + w + i, b + j, sr, si);
      }
    }
    __syncthreads();
    // X12 = -A^{-1} T_U (upper triangle of A^{-1}: t >= i)
    for (int e = tid; e < half; e += 256) {
      const int pr = e / per, q = e % per, i = q % w, j = q / w, b = 2 * w * pr;
      T sr = 0, si = 0, ar, ai, br, bi;
#pragma unroll 4
      for (int t = i; t < w; ++t) {
        ld(X, b + i, b + t, ar, ai);
        ld(X, b + w + t, b + j, br, bi);
        fma_sub<T, CPLX>(sr, si, ar, ai, br, bi);
      }
      st(X, b + i, b + w + j, sr, si);
    }
    __syncthreads();
    // X21 = -C^{-1} T_L (unit lower C^{-1}: t < i, plus the diagonal)
    for (int e = tid; e < half; e += 256) {
      const int pr = e / per, q = e % per, i = q % w, j = q / w, b = 2 * w * pr;
      T sr = -Tb[0][pr * w + i][j], si = CPLX ? -Tb[NP - 1][pr * w + i][j] : T(0), ar, ai;
#pragma unroll 4
      for (int t = 0; t < i; ++t) {
        ld(X, b + w + i, b + w + t, ar, ai);
        fma_sub<T, CPLX>(sr, si, ar, ai, Tb[0][pr * w + t][j], CPLX ? Tb[NP - 1][pr * w + t][j] : T(0));
      }
      st(X, b + w + i, b + j, sr, si);
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e % NB, cc = e / NB;
    T xr, xi;
    ld(X, i, cc, xr, xi);
    const bool lo = i > cc, zr = dropped && dropped[i];
    Linv.re[i + cc * Linv.ld] = zr ? T(0) : lo ? xr : (i == cc ? T(1) : T(0));
    if constexpr (CPLX) Linv.im[i + cc * Linv.ld] = (zr || !lo) ? T(0) : xi;
    Uinv.re[i + cc * Uinv.ld] = lo ? T(0) : xr;
    if constexpr (CPLX) Uinv.im[i + cc * Uinv.ld] = lo ? T(0) : xi;
  }
}

// Factor one NB x NB diagonal block without pivoting in LDS, in four panels
// of 16 columns: wave 0 factors the panel (a lane per row, the pivot row
// passed by shuffles, no barrier per column), then 16 threads solve the
// block row of U right of the panel and all threads update the trailing
// block.
// (complex FP32: two workgroups per CU fit in shared memory; the bound keeps
// the registers within two waves per SIMD as well, for the 512-item batches)
template <typename T, bool CPLX>
__global__ __launch_bounds__(256, (CPLX && sizeof(T) == 4) ? 2 : 1) void k_lu_diag(
    DMat<T> A, int64_t k0, DMat<T> inv, int iblk,
                                                 unsigned* flags, T tiny, int* drop, T droptol) {
  constexpr int NP = CPLX ? 2 : 1;
  constexpr int PW = 16;
  __shared__ T F[NP][NB][NB + 1];
  __shared__ T X[NP][NB][NB + 1];
  __shared__ T Tb[NP][32][33];
  __shared__ int dl[NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < NB) dl[tid] = 0;
  DMat<T> a = A.item(blockIdx.x).sub(k0, k0);
  load_block<T, CPLX>(F, a, tid);
  __syncthreads();
  for (int c0 = 0; c0 < NB; c0 += PW) {
    if (wave == 0) {
      const int r = lane;
      T ar[PW], ai[PW];
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        ar[q] = F[0][r][c0 + q];
        ai[q] = CPLX ? F[NP - 1][r][c0 + q] : T(0);
      }
#pragma unroll
      for (int kk = 0; kk < PW; ++kk) {
        const int j = c0 + kk;
        const T pr = lane_read(ar[kk], j);
        const T pim = CPLX ? lane_read(ai[kk], j) : T(0);
        if (!CPLX && drop && !(pr > droptol)) {
          // semidefinite mode: the pivot of the Schur complement vanished,
          // so column j lies in the span of the earlier ones; it is removed
          // from the factor (unit column of L, unit row of U)
          if (r > j) ar[kk] = 0;
          if (r == j) {
            ar[kk] = 1;
#pragma unroll
            for (int q = 0; q < PW; ++q)
              if (q > kk) ar[q] = 0;
            dl[j] = 1;
            drop[k0 + j] = 1;
          }
          continue;
        }
        if (r == 0) {
          const T mag = CPLX ? sqrt(pr * pr + pim * pim) : fabs(pr);
          if (!(mag > tiny)) atomicOr(flags, (mag == mag) ? 1u : 2u);
        }
        T ir, ii = 0;
        if constexpr (CPLX) cinv(pr, pim, ir, ii);
        else ir = T(1) / pr;
        T lr = 0, li = 0;
        if (r > j) {
          if constexpr (CPLX) cmul(ar[kk], ai[kk], ir, ii, lr, li);
          else lr = ar[kk] * ir;
          ar[kk] = lr;
          ai[kk] = li;
        }
#pragma unroll
        for (int q = 0; q < PW; ++q)
          if (q > kk) {
            const T ur = lane_read(ar[q], j);
            const T ui = CPLX ? lane_read(ai[q], j) : T(0);
            if (r > j) fma_sub<T, CPLX>(ar[q], ai[q], lr, li, ur, ui);
          }
      }
      if (r >= c0) {
#pragma unroll
        for (int q = 0; q < PW; ++q) {
          F[0][r][c0 + q] = ar[q];
          if constexpr (CPLX) F[NP - 1][r][c0 + q] = ai[q];
        }
      }
    }
    __syncthreads();
    const int c1 = c0 + PW, m2 = NB - c1;
    if (m2 <= 0) break;
    // U12 = L11^{-1} A12: a thread per column right of the panel
    if (tid < m2) {
      const int cc = c1 + tid;
      T xr[PW], xi[PW];
#pragma unroll
      for (int i = 0; i < PW; ++i) {
        __builtin_amdgcn_sched_barrier(0);
        T sr = F[0][c0 + i][cc], si = CPLX ? F[NP - 1][c0 + i][cc] : T(0);
#pragma unroll
        for (int t = 0; t < PW; ++t)
          if (t < i)
            fma_sub<T, CPLX>(sr, si, F[0][c0 + i][c0 + t], CPLX ? F[NP - 1][c0 + i][c0 + t] : T(0),
                             xr[t], xi[t]);
        if (dl[c0 + i]) sr = si = 0;
        xr[i] = sr;
        xi[i] = si;
      }
#pragma unroll
      for (int i = 0; i < PW; ++i) {
        F[0][c0 + i][cc] = xr[i];
        if constexpr (CPLX) F[NP - 1][c0 + i][cc] = xi[i];
      }
    }
    __syncthreads();
    // A22 -= L21 U12
    for (int e = tid; e < m2 * m2; e += 256) {
      const int i = c1 + e % m2, cc = c1 + e / m2;
      T sr = F[0][i][cc], si = CPLX ? F[NP - 1][i][cc] : T(0);
#pragma unroll
      for (int t = 0; t < PW; ++t)
        fma_sub<T, CPLX>(sr, si, F[0][i][c0 + t], CPLX ? F[NP - 1][i][c0 + t] : T(0),
                         F[0][c0 + t][cc], CPLX ? F[NP - 1][c0 + t][cc] : T(0));
      F[0][i][cc] = sr;
      if constexpr (CPLX) F[NP - 1][i][cc] = si;
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e % NB, j = e / NB;
    a.re[i + j * a.ld] = F[0][i][j];
    if constexpr (CPLX) a.im[i + j * a.ld] = F[NP - 1][i][j];
  }
  DMat<T> iv = inv.item(blockIdx.x);
  tri_inverses<T, CPLX>(F, X, Tb, iv.sub(0, 2 * NB * iblk), iv.sub(0, 2 * NB * iblk + NB),
                        drop ? dl : nullptr);
}

// Inverses only (block already factored, e.g. by the pivoted panel).
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void k_tri_inv(DMat<T> A, int64_t k0, DMat<T> inv, int iblk) {
  constexpr int NP = CPLX ? 2 : 1;
  __shared__ T F[NP][NB][NB + 1];
  __shared__ T X[NP][NB][NB + 1];
  __shared__ T Tb[NP][32][33];
  const int tid = threadIdx.x;
  DMat<T> a = A.item(blockIdx.x).sub(k0, k0);
  load_block<T, CPLX>(F, a, tid);
  __syncthreads();
  DMat<T> iv = inv.item(blockIdx.x);
  tri_inverses<T, CPLX>(F, X, Tb, iv.sub(0, 2 * NB * iblk), iv.sub(0, 2 * NB * iblk + NB));
}

// ---------------------------------------------------------------------------
// Recursive block forms.  Splitting in halves (multiples of NB) puts most of
// the flops into products with K = n/2, n/4, ... instead of K = NB, so the
// matrix cores run the large-K GEMM tiles.  Leaves multiply by the inverted
// NB x NB diagonal blocks written by k_lu_diag (inv = [Linv_0 Uinv_0 Linv_1
// ...]); a leaf product overwrites its own operand, which is safe because it
// has a single tile row (M = NB) or column (N = NB).
// ---------------------------------------------------------------------------
// B <- L^{-1} B, L = unit-lower factor rows/cols n0 .. n0+nb-1; row i of B is row n0+i
// Optional wide leaves for the solves: inverses of the LW x LW diagonal
// blocks (merge_inverses) and a workspace for the leaf product, which cannot
// overwrite its operand once it spans several tile rows.
template <typename T>
struct WideLeaves {
  DMat<T> inv2;
  int LW = 0;
  DMat<T> work;
};

template <typename T>
static void trsm_ll(hipStream_t s, DMat<T> LU, DMat<T> inv, int64_t n0, int64_t nb, DMat<T> B,
                    int64_t cols, int batch, const WideLeaves<T>& wl = WideLeaves<T>{}) {
  if (wl.LW && nb == wl.LW) {
    gemm<T>(s, false, false, nb, cols, nb, T(1), wl.inv2.sub(0, 2 * n0), B, T(0), wl.work, batch);
    convert<T, T>(s, wl.work, B, nb, cols, batch);
    return;
  }
  if (nb == NB) {
    gemm<T>(s, false, false, NB, cols, NB, T(1), inv.sub(0, 2 * n0), B, T(0), B, batch);
    return;
  }
  const int64_t unit = wl.LW ? wl.LW : NB;
  const int64_t h = (nb / unit / 2) * unit;
  trsm_ll<T>(s, LU, inv, n0, h, B, cols, batch, wl);
  gemm<T>(s, false, false, nb - h, cols, h, T(-1), LU.sub(n0 + h, n0), B, T(1), B.sub(h, 0), batch);
  trsm_ll<T>(s, LU, inv, n0 + h, nb - h, B.sub(h, 0), cols, batch, wl);
}

// B <- U^{-1} B, U = upper factor rows/cols n0 .. n0+nb-1; row i of B is row n0+i
template <typename T>
static void trsm_ul(hipStream_t s, DMat<T> LU, DMat<T> inv, int64_t n0, int64_t nb, DMat<T> B,
                    int64_t cols, int batch, const WideLeaves<T>& wl = WideLeaves<T>{}) {
  if (wl.LW && nb == wl.LW) {
    gemm<T>(s, false, false, nb, cols, nb, T(1), wl.inv2.sub(0, 2 * n0 + nb), B, T(0), wl.work,
            batch);
    convert<T, T>(s, wl.work, B, nb, cols, batch);
    return;
  }
  if (nb == NB) {
    gemm<T>(s, false, false, NB, cols, NB, T(1), inv.sub(0, 2 * n0 + NB), B, T(0), B, batch);
    return;
  }
  const int64_t unit = wl.LW ? wl.LW : NB;
  const int64_t h = (nb / unit / 2) * unit;
  trsm_ul<T>(s, LU, inv, n0 + h, nb - h, B.sub(h, 0), cols, batch, wl);
  gemm<T>(s, false, false, h, cols, nb - h, T(-1), LU.sub(n0, n0 + h), B.sub(h, 0), T(1), B, batch);
  trsm_ul<T>(s, LU, inv, n0, h, B, cols, batch, wl);
}

// B <- B U^{-1}, U = upper factor rows/cols n0 .. n0+nb-1; column j of B is column n0+j
template <typename T>
static void trsm_ur(hipStream_t s, DMat<T> LU, DMat<T> inv, int64_t n0, int64_t nb, DMat<T> B,
                    int64_t rows, int batch) {
  if (nb == NB) {
    gemm<T>(s, false, false, rows, NB, NB, T(1), B, inv.sub(0, 2 * n0 + NB), T(0), B, batch);
    return;
  }
  const int64_t h = (nb / NB / 2) * NB;
  trsm_ur<T>(s, LU, inv, n0, h, B, rows, batch);
  gemm<T>(s, false, false, rows, nb - h, h, T(-1), B, LU.sub(n0, n0 + h), T(1), B.sub(0, h), batch);
  trsm_ur<T>(s, LU, inv, n0 + h, nb - h, B.sub(0, h), rows, batch);
}

// LU without pivoting of rows/cols n0 .. n0+nb-1 (all earlier updates applied)
template <typename T>
static void lu_rec(hipStream_t s, DMat<T> A, DMat<T> inv, int64_t n0, int64_t nb, int batch,
                   unsigned* flags, double tiny) {
  if (nb == NB) {
    if (A.cplx())
      k_lu_diag<T, true><<<batch, 256, 0, s>>>(A, n0, inv, (int)(n0 / NB), flags, (T)tiny, nullptr, T(0));
    else
      k_lu_diag<T, false><<<batch, 256, 0, s>>>(A, n0, inv, (int)(n0 / NB), flags, (T)tiny, nullptr, T(0));
    RFD_CHECK_LAUNCH();
    return;
  }
  const int64_t h = (nb / NB / 2) * NB, r = nb - h;
  lu_rec<T>(s, A, inv, n0, h, batch, flags, tiny);
  trsm_ll<T>(s, A, inv, n0, h, A.sub(n0, n0 + h), r, batch);   // U12 = L11^{-1} A12
  trsm_ur<T>(s, A, inv, n0, h, A.sub(n0 + h, n0), r, batch);   // L21 = A21 U11^{-1}
  gemm<T>(s, false, false, r, r, h, T(-1), A.sub(n0 + h, n0), A.sub(n0, n0 + h), T(1),
          A.sub(n0 + h, n0 + h), batch);
  lu_rec<T>(s, A, inv, n0 + h, r, batch, flags, tiny);
}

template <typename T>
void lu_nopiv(hipStream_t s, DMat<T> A, int64_t n, int batch, DMat<T> inv, unsigned* flags,
              double tiny, int* drop, double droptol) {
  if (n % NB) throw Error(ST_EINVAL, "lu_nopiv: n not a multiple of the block size");
  if (drop && (A.cplx() || batch != 1)) throw Error(ST_EINVAL, "lu_nopiv: drop mode is real, unbatched");
  if (!drop) {
    lu_rec<T>(s, A, inv, 0, n, batch, flags, tiny);
    return;
  }
  // semidefinite drop mode: right-looking, one NB block at a time
  const int64_t nblk = n / NB;
  for (int64_t i = 0; i < nblk; ++i) {
    const int64_t k0 = i * NB, rest = n - k0 - NB;
    if (A.cplx())
      k_lu_diag<T, true><<<batch, 256, 0, s>>>(A, k0, inv, (int)i, flags, (T)tiny, nullptr, T(0));
    else
      k_lu_diag<T, false><<<batch, 256, 0, s>>>(A, k0, inv, (int)i, flags, (T)tiny, drop,
                                                 (T)droptol);
    RFD_CHECK_LAUNCH();
    if (rest > 0) {
      DMat<T> Linv = inv.sub(0, 2 * NB * i), Uinv = inv.sub(0, 2 * NB * i + NB);
      gemm<T>(s, false, false, rest, NB, NB, T(1), A.sub(k0 + NB, k0), Uinv, T(0),
              A.sub(k0 + NB, k0), batch);
      gemm<T>(s, false, false, NB, rest, NB, T(1), Linv, A.sub(k0, k0 + NB), T(0),
              A.sub(k0, k0 + NB), batch);
      gemm<T>(s, false, false, rest, rest, NB, T(-1), A.sub(k0 + NB, k0), A.sub(k0, k0 + NB),
              T(1), A.sub(k0 + NB, k0 + NB), batch);
    }
  }
}

// ---------------------------------------------------------------------------
// Partial pivoting (real data): panel of width NB, rows k0..n-1, factored by
// one workgroup per item directly in global memory.  Each thread owns rows
// tid, tid + 256, ...; per column it loads the rest of its row's panel at
// once, applies the rank-1 update in registers and stores it, so a column
// costs one memory round trip per owned row instead of one per entry.  The
// pivot search of the next column rides along with the update.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_panel_piv(DMat<T> A, int64_t n, int64_t k0,
                                                   int32_t* ipiv, unsigned* flags, T tiny) {
  __shared__ T sval[256];
  __shared__ int sidx[256];
  __shared__ T prow[NB];
  const int tid = threadIdx.x;
  DMat<T> a = A.item(blockIdx.x);
  T* a0 = a.re + k0 * a.ld;  // column k0 of the panel
  const int64_t ld = a.ld;
  int32_t* piv = ipiv + (int64_t)blockIdx.x * n;
  // argmax |a(i, k0)|, i >= k0, per thread (rows in increasing order keep the
  // first index on ties)
  T best = -1;
  int bi = (int)k0;
  for (int64_t i = k0 + tid; i < n; i += 256) {
    const T v = fabs(a0[i]);
    if (v > best) { best = v; bi = (int)i; }
  }
  for (int j = 0; j < NB; ++j) {
    const int64_t col = k0 + j;
    sval[tid] = best;
    sidx[tid] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        const T v2 = sval[tid + w];
        const int i2 = sidx[tid + w];
        if (v2 > sval[tid] || (v2 == sval[tid] && i2 < sidx[tid])) {
          sval[tid] = v2;
          sidx[tid] = i2;
        }
      }
      __syncthreads();
    }
    const int p = sidx[0];
    const T pmag = sval[0];
    __syncthreads();
    if (tid == 0) {
      piv[col] = p;
      if (!(pmag > tiny)) atomicOr(flags, (pmag == pmag) ? 1u : 2u);
    }
    // swap rows col and p within the panel columns
    if (p != col && tid < NB) {
      const T t = a0[col + tid * ld];
      a0[col + tid * ld] = a0[p + tid * ld];
      a0[p + tid * ld] = t;
    }
    __syncthreads();
    if (tid < NB) prow[tid] = a0[col + tid * ld];
    __syncthreads();
    const T inv = T(1) / prow[j];
    best = -1;
    bi = (int)(col + 1);
    for (int64_t i = col + 1 + tid; i < n; i += 256) {
      T v[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c >= j) v[c] = a0[i + c * ld];
      // v[j] by a select over the unrolled indices (a runtime index would
      // move v to scratch memory)
      T vj = 0;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c == j) vj = v[c];
      const T l = vj * inv;
      a0[i + j * ld] = l;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c > j) {
          v[c] -= l * prow[c];
          a0[i + c * ld] = v[c];
        }
      if (j + 1 < NB) {
        T vn = 0;
#pragma unroll
        for (int c = 1; c < NB; ++c)
          if (c == j + 1) vn = v[c];
        const T m = fabs(vn);
        if (m > best) { best = m; bi = (int)i; }
      }
    }
    __syncthreads();
  }
}

// Row interchanges ipiv[k0 .. k0+cnt) applied in order to columns [c0, c1).
template <typename T>
__global__ void k_laswp(DMat<T> A, int64_t n, const int32_t* ipiv, int64_t k0, int64_t cnt,
                        int64_t c0, int64_t c1) {
  const int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  DMat<T> a = A.item(blockIdx.y);
  const int32_t* piv = ipiv + (int64_t)blockIdx.y * n;
  for (int64_t i = k0; i < k0 + cnt; ++i) {
    const int64_t p = piv[i];
    if (p != i) {
      const T t = a.re[i + c * a.ld];
      a.re[i + c * a.ld] = a.re[p + c * a.ld];
      a.re[p + c * a.ld] = t;
    }
  }
}

template <typename T>
static void laswp(hipStream_t s, DMat<T> A, int64_t n, const int32_t* ipiv, int64_t k0,
                  int64_t cnt, int64_t c0, int64_t c1, int batch) {
  if (c1 <= c0) return;
  dim3 g(grid1(c1 - c0), batch);
  k_laswp<T><<<g, 256, 0, s>>>(A, n, ipiv, k0, cnt, c0, c1);
  RFD_CHECK_LAUNCH();
}

template <typename T>
void lu_piv(hipStream_t s, DMat<T> A, int64_t n, int batch, DMat<T> inv, int32_t* ipiv,
            unsigned* flags, double tiny) {
  if (n % NB) throw Error(ST_EINVAL, "lu_piv: n not a multiple of the block size");
  if (A.cplx()) throw Error(ST_EINVAL, "lu_piv: real data only");
  const int64_t nblk = n / NB;
  for (int64_t i = 0; i < nblk; ++i) {
    const int64_t k0 = i * NB, rest = n - k0 - NB;
    k_panel_piv<T><<<batch, 256, 0, s>>>(A, n, k0, ipiv, flags, (T)tiny);
    RFD_CHECK_LAUNCH();
    laswp<T>(s, A, n, ipiv, k0, NB, 0, k0, batch);
    laswp<T>(s, A, n, ipiv, k0, NB, k0 + NB, n, batch);
    k_tri_inv<T, false><<<batch, 256, 0, s>>>(A, k0, inv, (int)i);
    RFD_CHECK_LAUNCH();
    if (rest > 0) {
      DMat<T> Linv = inv.sub(0, 2 * NB * i);
      gemm<T>(s, false, false, NB, rest, NB, T(1), Linv, A.sub(k0, k0 + NB), T(0),
              A.sub(k0, k0 + NB), batch);
      gemm<T>(s, false, false, rest, rest, NB, T(-1), A.sub(k0 + NB, k0), A.sub(k0, k0 + NB),
              T(1), A.sub(k0 + NB, k0 + NB), batch);
    }
  }
}

template <typename T>
void lu_solve(hipStream_t s, DMat<T> LU, DMat<T> inv, const int32_t* ipiv, int64_t n, DMat<T> R,
              int64_t r, int batch, int parts, DMat<T> inv2, int LW, DMat<T> work) {
  if (n % NB) throw Error(ST_EINVAL, "lu_solve: n not a multiple of the block size");
  if (n == 0 || r <= 0) return;
  WideLeaves<T> wl;
  if (LW > 0) {
    if (LW % NB || n % LW || !inv2.re || !work.re)
      throw Error(ST_EINVAL, "lu_solve: wide leaves need LW | n, NB | LW and their buffers");
    wl.inv2 = inv2;
    wl.LW = LW;
    wl.work = work;
  }
  if (ipiv && (parts & 1)) laswp<T>(s, R, n, ipiv, 0, n, 0, r, batch);
  if (parts & 1) trsm_ll<T>(s, LU, inv, 0, n, R, r, batch, wl);
  if (parts & 2) trsm_ul<T>(s, LU, inv, 0, n, R, r, batch, wl);
}

template <typename T>
void merge_inverses(hipStream_t s, DMat<T> LU, DMat<T> inv, int64_t n, int batch, DMat<T> inv2,
                    int LW, DMat<T> work) {
  if (LW % NB || n % LW || (LW / NB & (LW / NB - 1)))
    throw Error(ST_EINVAL, "merge_inverses: LW must be NB times a power of two dividing n");
  const int64_t nblk = n / LW;
  fill<T>(s, inv2, LW, 2 * n, batch, T(0));
  // one launch covers the diagonal blocks of one item (a strided batch), or
  // one block position of every item (the item stride), whichever is more
  const bool across_items = batch > nblk;
  const int outer = across_items ? (int)nblk : batch;
  const int cnt = across_items ? batch : (int)nblk;
  for (int it = 0; it < outer; ++it) {
    DMat<T> lu, iv, i2, wk = work;
    if (across_items) {
      lu = LU.sub((int64_t)it * LW, (int64_t)it * LW);
      iv = inv.sub(0, 2 * (int64_t)it * LW);
      i2 = inv2.sub(0, 2 * (int64_t)it * LW);
    } else {
      lu = LU.item(it);
      iv = inv.item(it);
      i2 = inv2.item(it);
      lu.bs = LW + LW * lu.ld;           // next diagonal block
      iv.bs = 2 * LW * iv.ld;            // its NB-block inverses
      i2.bs = 2 * LW * i2.ld;            // its wide inverses
    }
    for (int q = 0; q < LW / NB; ++q) {
      convert<T, T>(s, iv.sub(0, 2 * q * NB), i2.sub(q * NB, q * NB), NB, NB, cnt);
      convert<T, T>(s, iv.sub(0, 2 * q * NB + NB), i2.sub(q * NB, LW + q * NB), NB, NB, cnt);
    }
    // [A 0; B C]^{-1} = [A^{-1} 0; -C^{-1} B A^{-1} C^{-1}] and
    // [A B; 0 C]^{-1} = [A^{-1} -A^{-1} B C^{-1}; 0 C^{-1}], widths NB, 2 NB, ...
    for (int w = NB; 2 * w <= LW; w *= 2)
      for (int o = 0; o < LW; o += 2 * w) {
        DMat<T> tw = wk;
        tw.ld = w;
        tw.bs = (int64_t)w * w;
        gemm<T>(s, false, false, w, w, w, T(1), lu.sub(o + w, o), i2.sub(o, o), T(0), tw, cnt);
        gemm<T>(s, false, false, w, w, w, T(-1), i2.sub(o + w, o + w), tw, T(0), i2.sub(o + w, o),
                cnt);
        gemm<T>(s, false, false, w, w, w, T(1), lu.sub(o, o + w), i2.sub(o + w, LW + o + w), T(0),
                tw, cnt);
        gemm<T>(s, false, false, w, w, w, T(-1), i2.sub(o, LW + o), tw, T(0), i2.sub(o, LW + o + w),
                cnt);
      }
  }
}

// ---------------------------------------------------------------------------
// Elementwise helpers.  Grid: x over rows*cols, y over batch.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(DMat<T> X, int64_t rows, int64_t cols, T v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e % rows, j = e / rows;
  DMat<T> x = X.item(blockIdx.y);
  x.re[i + j * x.ld] = v;
  if (x.im) x.im[i + j * x.ld] = 0;
}

template <typename T>
void fill(hipStream_t s, DMat<T> X, int64_t rows, int64_t cols, int batch, T value) {
  if (rows <= 0 || cols <= 0) return;
  dim3 g(grid1(rows * cols), batch);
  k_fill<T><<<g, 256, 0, s>>>(X, rows, cols, value);
  RFD_CHECK_LAUNCH();
}

template <typename T>
__global__ void k_pad_identity(DMat<T> X, int64_t active, int64_t n) {
  const int64_t i = active + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  DMat<T> x = X.item(blockIdx.y);
  x.re[i + i * x.ld] = 1;
  if (x.im) x.im[i + i * x.ld] = 0;
}

template <typename T>
void pad_identity(hipStream_t s, DMat<T> X, int64_t active, int64_t n, int batch) {
  if (n <= active) return;
  dim3 g(grid1(n - active), batch);
  k_pad_identity<T><<<g, 256, 0, s>>>(X, active, n);
  RFD_CHECK_LAUNCH();
}

template <typename TD, typename TS>
__global__ void k_convert(DMat<TS> X, DMat<TD> Y, int64_t rows, int64_t cols, int add) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e % rows, j = e / rows;
  DMat<TS> x = X.item(blockIdx.y);
  DMat<TD> y = Y.item(blockIdx.y);
  const int64_t ox = i + j * x.ld, oy = i + j * y.ld;
  const TD vr = (TD)x.re[ox];
  const TD vi = x.im ? (TD)x.im[ox] : TD(0);
  if (add) {
    y.re[oy] += vr;
    if (y.im) y.im[oy] += vi;
  } else {
    y.re[oy] = vr;
    if (y.im) y.im[oy] = vi;
  }
}

template <typename TD, typename TS>
void convert(hipStream_t s, DMat<TS> X, DMat<TD> Y, int64_t rows, int64_t cols, int batch) {
  if (rows <= 0 || cols <= 0) return;
  dim3 g(grid1(rows * cols), batch);
  k_convert<TD, TS><<<g, 256, 0, s>>>(X, Y, rows, cols, 0);
  RFD_CHECK_LAUNCH();
}

template <typename TD, typename TS>
void add_to(hipStream_t s, DMat<TS> X, DMat<TD> Y, int64_t rows, int64_t cols, int batch) {
  if (rows <= 0 || cols <= 0) return;
  dim3 g(grid1(rows * cols), batch);
  k_convert<TD, TS><<<g, 256, 0, s>>>(X, Y, rows, cols, 1);
  RFD_CHECK_LAUNCH();
}

__device__ inline void atomic_max_nonneg(double* p, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

template <typename T>
__global__ void k_absmax(DMat<T> X, int64_t rows, int64_t cols, double* out) {
  __shared__ double red[256];
  double m = 0;
  DMat<T> x = X.item(blockIdx.y);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, j = e / rows;
    double v = fabs((double)x.re[i + j * x.ld]);
    if (x.im) v = fmax(v, fabs((double)x.im[i + j * x.ld]));
    if (!(v == v)) v = INFINITY;
    m = fmax(m, v);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomic_max_nonneg(out, red[0]);
}

template <typename T>
void absmax(hipStream_t s, DMat<T> X, int64_t rows, int64_t cols, int batch, double* out) {
  if (rows <= 0 || cols <= 0) return;
  const int64_t tot = rows * cols;
  dim3 g((unsigned)std::min<int64_t>(grid1(tot), 1024), batch);
  k_absmax<T><<<g, 256, 0, s>>>(X, rows, cols, out);
  RFD_CHECK_LAUNCH();
}

// explicit instantiations
#define RFD_INST(T)                                                                          \
  template void lu_nopiv<T>(hipStream_t, DMat<T>, int64_t, int, DMat<T>, unsigned*, double,     \
                            int*, double);                                                   \
  template void lu_piv<T>(hipStream_t, DMat<T>, int64_t, int, DMat<T>, int32_t*, unsigned*,  \
                          double);                                                           \
  template void lu_solve<T>(hipStream_t, DMat<T>, DMat<T>, const int32_t*, int64_t, DMat<T>, \
                            int64_t, int, int, DMat<T>, int, DMat<T>);                            \
  template void merge_inverses<T>(hipStream_t, DMat<T>, DMat<T>, int64_t, int, DMat<T>, int,   \
                                  DMat<T>);                                                   \
  template void fill<T>(hipStream_t, DMat<T>, int64_t, int64_t, int, T);                     \
  template void pad_identity<T>(hipStream_t, DMat<T>, int64_t, int64_t, int);                \
  template void absmax<T>(hipStream_t, DMat<T>, int64_t, int64_t, int, double*);
RFD_INST(float)
RFD_INST(double)
template void convert<float, double>(hipStream_t, DMat<double>, DMat<float>, int64_t, int64_t, int);
template void convert<double, float>(hipStream_t, DMat<float>, DMat<double>, int64_t, int64_t, int);
template void convert<double, double>(hipStream_t, DMat<double>, DMat<double>, int64_t, int64_t, int);
template void convert<float, float>(hipStream_t, DMat<float>, DMat<float>, int64_t, int64_t, int);
template void add_to<double, float>(hipStream_t, DMat<float>, DMat<double>, int64_t, int64_t, int);
template void add_to<double, double>(hipStream_t, DMat<double>, DMat<double>, int64_t, int64_t, int);

}  // namespace rfd
