// Batched MFMA GEMM for gfx950 (FP32 / FP64, real / planar complex).
//
// Workgroup tile BM x BN (64 or 128), 4 waves in a 2 x 2 arrangement, K slabs
// of 16 staged through double-buffered LDS: the next slab's global loads
// (16-byte vectors when the operand is aligned) are in flight while the
// current slab feeds the matrix cores.  FP32 uses v_mfma_f32_32x32x2f32 and
// FP64 v_mfma_f64_16x16x4f64.  The operands enter the MFMA swapped (the B
// tile as the row operand) so that the accumulator rows run down the columns
// of the column-major C and the epilogue stores are coalesced.  A complex
// product takes three real products (Gauss): P1 = Ar Br, P2 = Ai Bi and
// P3 = (Ar + Ai)(Br + Bi), then Re = P1 - P2 and Im = P3 - P1 - P2, a quarter
// fewer matrix-core cycles (in FP32 its rounding is the factorizations',
// which the FP64 refinement corrects; in FP64 the imaginary part's error
// bound grows by at most a factor of about two).  Complex FP64 products of
// the 64 x 64 k_gemm tile keep four real products into two accumulators.
//
// Operand lane layouts: 32x32x2 -- lane l holds X[l%32][l/32] of the row
// operand and Y[l/32][l%32] of the column operand; D register r of lane l is
// element (8 (r/4) + 4 (l/32) + r%4, l%32).  16x16x4 -- lane l holds
// X[l%16][l/16], Y[l/16][l%16]; D register r is element ((l/16) + 4 r, l%16).
//
// Few output tiles over a long K (the tall-skinny products of basis
// orthogonalisation and projection) split K over extra workgroups; partial
// tiles go to a per-stream workspace and a second kernel sums them in a fixed
// order, so results do not depend on scheduling.
//
// Real FP32 products with many output tiles over a long K take 128 x 128
// tiles, large real FP64 products the 64 x 128 tile of k_dgemm (scalar
// loads from clamped indices, no bounds branches in the K loop, alpha and
// beta folded into the operands and accumulators); everything else the 64 x
// 64 tile.
#include <hip/hip_ext.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <unordered_map>

#include "dense.hpp"

namespace rfd {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct V16;
template <> struct V16<float> { using t = float4; };
template <> struct V16<double> { using t = double2; };

constexpr int GBK = 16;

// Logical block index of this workgroup.  The dispatcher deals the
// workgroups of a grid to the 8 XCDs in turn (linear id L, x fastest, runs on
// XCD L % 8), and each XCD has its own L2.  Numbering the blocks so that XCD c
// works the c-th contiguous eighth of the (x, y, z) order keeps the tiles that
// share an operand panel (same item, same K chunk, neighbouring rows and
// columns) on one L2 instead of fetching every panel into all eight.
constexpr unsigned NXCD = 8;
__device__ inline uint3 xcd_block() {
  const unsigned gx = gridDim.x, gy = gridDim.y;
  const unsigned total = gx * gy * gridDim.z;
  const unsigned L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const unsigned q = total / NXCD, r = total % NXCD, c = L % NXCD, j = L / NXCD;
  // XCD c holds q + 1 blocks when c < r, else q
  const unsigned l = (c < r ? c * (q + 1) : r * (q + 1) + (c - r) * q) + j;
  return make_uint3(l % gx, (l / gx) % gy, l / (gx * gy));
}

// Registers holding one K slab of an operand tile.  In memory the tile is a
// column-major FE x SE block (FE along the contiguous dimension).
template <typename T, int FE, int SE>
struct Slab {
  static constexpr int VW = 16 / (int)sizeof(T);
  static constexpr int NV = FE * SE / VW / 256;
  static_assert(NV >= 1 && (FE * SE) % (VW * 256) == 0, "tile does not split over 256 threads");
  typename V16<T>::t v[NV];

  // base: tile element (0, 0) or null (zero operand); nf x ns valid extent;
  // fast: the whole tile is valid and 16-byte aligned.
  __device__ void load(const T* base, int64_t ld, int nf, int ns, bool fast, int tid) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = tid + 256 * q;
      const int f = (e % (FE / VW)) * VW, sl = e / (FE / VW);
      T* o = reinterpret_cast<T*>(&v[q]);
      if (base == nullptr) {
#pragma unroll
        for (int w = 0; w < VW; ++w) o[w] = T(0);
      } else if (fast) {
        v[q] = *reinterpret_cast<const typename V16<T>::t*>(base + f + sl * ld);
      } else {
#pragma unroll
        for (int w = 0; w < VW; ++w)
          o[w] = (f + w < nf && sl < ns) ? base[f + w + sl * ld] : T(0);
      }
    }
  }

  // LDS tile L[k][x] (row length P).  kfast: the contiguous dimension is k
  // (scattered into LDS columns); otherwise it is x (vector stores).
  template <bool KFAST, int P>
  __device__ void store(T (*L)[P], int tid) const {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = tid + 256 * q;
      const int f = (e % (FE / VW)) * VW, sl = e / (FE / VW);
      const T* o = reinterpret_cast<const T*>(&v[q]);
      if (KFAST) {
#pragma unroll
        for (int w = 0; w < VW; ++w) L[f + w][sl] = o[w];
      } else {
        *reinterpret_cast<typename V16<T>::t*>(&L[sl][f]) = v[q];
      }
    }
  }
};

template <typename T, bool CPLX, bool TA, bool TB, int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm(int64_t M, int64_t N, int64_t K, T alpha, T beta,
                                              DMat<T> A, DMat<T> B, DMat<T> C, int splits,
                                              int64_t kchunk, T* part, int vec_a, int vec_b,
                                              int tri) {
  constexpr int NP = CPLX ? 2 : 1;
  constexpr int VW = 16 / (int)sizeof(T);
  constexpr int PA = BM + VW, PB = BN + VW;
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int BLK = F32 ? 32 : 16;                 // MFMA block edge
  constexpr int XM = BM / 2 / BLK, XN = BN / 2 / BLK;  // blocks per wave
  __shared__ __attribute__((aligned(16))) T As[2][NP][GBK][PA];
  __shared__ __attribute__((aligned(16))) T Bs[2][NP][GBK][PB];

  const uint3 blk = xcd_block();
  const int64_t m0 = (int64_t)blk.x * BM, n0 = (int64_t)blk.y * BN;
  if (tri && n0 >= m0 + BM) return;  // strictly upper tile, not wanted
  const int batch = (int)gridDim.z / splits;
  const int b = (int)blk.z / splits, sk = (int)blk.z - b * splits;
  A = A.item(b);
  B = B.item(b);
  C = C.item(b);
  const int64_t kb = (int64_t)sk * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
  const int mv = (int)((M - m0) < BM ? (M - m0) : BM);
  const int nv = (int)((N - n0) < BN ? (N - n0) : BN);

  using SA = Slab<T, TA ? GBK : BM, TA ? BM : GBK>;
  using SB = Slab<T, TB ? BN : GBK, TB ? GBK : BN>;
  SA ra[NP];
  SB rb[NP];
  const bool aim = CPLX && A.im != nullptr, bim = CPLX && B.im != nullptr;

  auto gload = [&](int64_t k0) {
    const int kv = (int)((ke - k0) < GBK ? (ke - k0) : GBK);
    const int64_t oa = TA ? (k0 + m0 * A.ld) : (m0 + k0 * A.ld);
    const bool fa = vec_a && kv == GBK && mv == BM;
    ra[0].load(A.re + oa, A.ld, TA ? kv : mv, TA ? mv : kv, fa, tid);
    if constexpr (CPLX) ra[NP - 1].load(aim ? A.im + oa : nullptr, A.ld, TA ? kv : mv, TA ? mv : kv, fa, tid);
    const int64_t ob = TB ? (n0 + k0 * B.ld) : (k0 + n0 * B.ld);
    const bool fb = vec_b && kv == GBK && nv == BN;
    rb[0].load(B.re + ob, B.ld, TB ? nv : kv, TB ? kv : nv, fb, tid);
    if constexpr (CPLX) rb[NP - 1].load(bim ? B.im + ob : nullptr, B.ld, TB ? nv : kv, TB ? kv : nv, fb, tid);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      ra[p].template store<TA, PA>(As[buf][p], tid);
      rb[p].template store<!TB, PB>(Bs[buf][p], tid);
    }
  };

  // FP32 complex: fr, fi, fs accumulate P1, P2, P3 of the Gauss product
  floatx16 fr[XM][XN], fi[XM][XN], fs[XM][XN];
  doublex4 dr[XM][XN], di[XM][XN];
#pragma unroll
  for (int x = 0; x < XM; ++x)
#pragma unroll
    for (int y = 0; y < XN; ++y) {
      if constexpr (F32) {
        for (int r = 0; r < 16; ++r) fr[x][y][r] = 0.f, fi[x][y][r] = 0.f, fs[x][y][r] = 0.f;
      } else {
        dr[x][y] = doublex4{0, 0, 0, 0};
        di[x][y] = doublex4{0, 0, 0, 0};
      }
    }

  auto compute = [&](int buf) {
    if constexpr (F32) {
#pragma unroll
      for (int kk = 0; kk < GBK; kk += 2) {
        const int kr = kk + (lane >> 5), r = lane & 31;
        float ar[XM], ai[XM], br[XN], bi[XN], sa[XM], sb[XN];
#pragma unroll
        for (int x = 0; x < XM; ++x) {
          ar[x] = As[buf][0][kr][wm + 32 * x + r];
          if constexpr (CPLX) {
            ai[x] = As[buf][NP - 1][kr][wm + 32 * x + r];
            sa[x] = ar[x] + ai[x];
          }
        }
#pragma unroll
        for (int y = 0; y < XN; ++y) {
          br[y] = Bs[buf][0][kr][wn + 32 * y + r];
          if constexpr (CPLX) {
            bi[y] = Bs[buf][NP - 1][kr][wn + 32 * y + r];
            sb[y] = br[y] + bi[y];
          }
        }
#pragma unroll
        for (int x = 0; x < XM; ++x)
#pragma unroll
          for (int y = 0; y < XN; ++y) {
            fr[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(br[y], ar[x], fr[x][y], 0, 0, 0);
            if constexpr (CPLX) {
              fi[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(bi[y], ai[x], fi[x][y], 0, 0, 0);
              fs[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(sb[y], sa[x], fs[x][y], 0, 0, 0);
            }
          }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < GBK; kk += 4) {
        const int kr = kk + (lane >> 4), r = lane & 15;
        double ar[XM], ai[XM], br[XN], bi[XN];
#pragma unroll
        for (int x = 0; x < XM; ++x) {
          ar[x] = As[buf][0][kr][wm + 16 * x + r];
          if constexpr (CPLX) ai[x] = As[buf][NP - 1][kr][wm + 16 * x + r];
        }
#pragma unroll
        for (int y = 0; y < XN; ++y) {
          br[y] = Bs[buf][0][kr][wn + 16 * y + r];
          if constexpr (CPLX) bi[y] = Bs[buf][NP - 1][kr][wn + 16 * y + r];
        }
#pragma unroll
        for (int x = 0; x < XM; ++x)
#pragma unroll
          for (int y = 0; y < XN; ++y) {
            dr[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(br[y], ar[x], dr[x][y], 0, 0, 0);
            if constexpr (CPLX) {
              dr[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-bi[y], ai[x], dr[x][y], 0, 0, 0);
              di[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(br[y], ai[x], di[x][y], 0, 0, 0);
              di[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bi[y], ar[x], di[x][y], 0, 0, 0);
            }
          }
      }
    }
  };

  if (kb < ke) {
    gload(kb);
    lstore(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += GBK) {
    const bool more = k0 + GBK < ke;
    if (more) gload(k0 + GBK);
    compute(buf);
    // the other buffer was last read before the previous barrier
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  T* pr = nullptr;
  T* pi = nullptr;
  if (splits > 1) {
    pr = part + ((int64_t)(sk * batch + b) * NP) * M * N;
    pi = pr + (NP - 1) * M * N;
  }
  // this lane's outputs: RE per MFMA block
  constexpr int RE = F32 ? 16 : 4;
  auto ij = [&](int x, int y, int r, int64_t& i, int64_t& j) {
    if constexpr (F32) {
      i = m0 + wm + 32 * x + (lane & 31);
      j = n0 + wn + 32 * y + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    } else {
      i = m0 + wm + 16 * x + (lane & 15);
      j = n0 + wn + 16 * y + (lane >> 4) + 4 * r;
    }
  };
  // beta C in rounds of CH elements per lane (all of them in FP64; 8 in
  // FP32, whose larger accumulator sets leave fewer registers): a round's
  // loads are all issued before the first is used, from offsets clamped into
  // C.  (Loads in per-element branches would each wait in turn, and the
  // wait also covers every store issued before it.)
  const bool use_c = splits == 1 && beta != T(0);
  auto put = [&](int64_t i, int64_t j, T vr, T vi, T cr, T ci) {
    if (i >= M || j >= N) return;
    if (splits > 1) {
      pr[i + j * M] = alpha * vr;
      if constexpr (CPLX) pi[i + j * M] = alpha * vi;
      return;
    }
    const int64_t off = i + j * C.ld;
    T outr = alpha * vr, outi = alpha * vi;
    if (use_c) {
      outr += beta * cr;
      if constexpr (CPLX) outi += beta * ci;
    }
    C.re[off] = outr;
    if constexpr (CPLX) C.im[off] = outi;
  };
  constexpr int E = XM * XN * RE;
  constexpr int CH = F32 ? 8 : E;
  static_assert(E % CH == 0, "rounds of C loads do not divide the outputs");
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += CH) {
    T cr[CH], ci[CH];
    if (use_c) {
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = e0 + u, r = e % RE, y = (e / RE) % XN, x = e / (RE * XN);
        int64_t i, j;
        ij(x, y, r, i, j);
        const int64_t off = (i < M && j < N) ? i + j * C.ld : 0;
        cr[u] = C.re[off];
        ci[u] = CPLX ? C.im[off] : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = e0 + u, r = e % RE, y = (e / RE) % XN, x = e / (RE * XN);
      int64_t i, j;
      ij(x, y, r, i, j);
      if constexpr (F32) {
        if constexpr (CPLX)
          put(i, j, fr[x][y][r] - fi[x][y][r], (fs[x][y][r] - fr[x][y][r]) - fi[x][y][r], cr[u],
              ci[u]);
        else
          put(i, j, fr[x][y][r], 0.0f, cr[u], ci[u]);
      } else {
        put(i, j, dr[x][y][r], CPLX ? di[x][y][r] : 0.0, cr[u], ci[u]);
      }
    }
  }
}

// Large FP64 products: real on 64 x 128 tiles (each of the 4 waves, 2 x 2,
// computes 32 x 64 of v_mfma_f64_16x16x4f64 blocks), complex on 64 x 64
// tiles in Gauss's form (three real products per block: P1 = Ar Br, P2 =
// Ai Bi, P3 = (Ar + Ai)(Br + Bi), the operand sums formed from the LDS
// reads; Re = P1 - P2 and Im = P3 - P1 - P2 in the epilogue); two waves per
// SIMD.  Loads are scalar 8-byte loads
// (no alignment condition: the long operands of the solve have odd leading
// dimensions) at a block-uniform base per K slab plus a per-thread 32-bit
// offset fixed for the whole loop, from row and column indices clamped into
// the matrices, so the loop has no bounds branches: rows of op(A) beyond M
// and columns of op(B) beyond N only feed outputs that are never stored,
// and K indices beyond the range (last slab only) read as 0.  Consecutive
// lanes read consecutive addresses of the contiguous dimension.  alpha
// (real) scales op(A) as it is staged and the accumulators start from
// beta C (in Gauss's split for complex products), so the epilogue only
// stores (and, complex, combines) them.
template <bool CPLX, bool TA, bool TB, int BM, int BN>
__global__ __launch_bounds__(256, 2) void k_dgemm(int64_t M, int64_t N, int64_t K, double alpha,
                                                  double beta, DMat<double> A, DMat<double> B,
                                                  DMat<double> C, int tri) {
  constexpr int NP = CPLX ? 2 : 1;
  constexpr int PA = BM + 2, PB = BN + 2;
  constexpr int XM = BM / 32, XN = BN / 32;                // 16 x 16 blocks per wave
  constexpr int LA = BM * GBK / 256, LB = BN * GBK / 256;  // loads per plane, thread and slab
  __shared__ __attribute__((aligned(16))) double As[2][NP][GBK][PA];
  __shared__ __attribute__((aligned(16))) double Bs[2][NP][GBK][PB];

  const uint3 blk = xcd_block();
  const int64_t m0 = (int64_t)blk.x * BM, n0 = (int64_t)blk.y * BN;
  if (tri == 1 && n0 >= m0 + BM) return;
  const int b = (int)blk.z;
  A = A.item(b);
  B = B.item(b);
  C = C.item(b);
  // tri == 2: op(B) upper triangular, so the tile's columns need k < n0 + BN only
  const int64_t ke = (tri == 2 && n0 + BN < K) ? n0 + BN : K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);

  constexpr int ASTEP = TA ? 256 / GBK : 256 / BM;  // stride of the other index per load
  constexpr int BSTEP = TB ? 256 / BN : 256 / GBK;
  const int a_c = TA ? tid % GBK : tid % BM;  // contiguous index (k if TA, else m)
  const int a_o = TA ? tid / GBK : tid / BM;  // first other index
  const int b_c = TB ? tid % BN : tid % GBK;  // contiguous index (n if TB, else k)
  const int b_o = TB ? tid / BN : tid / GBK;
  const int lda = (int)A.ld, ldb = (int)B.ld;
  uint32_t offa[LA], offb[LB];
#pragma unroll
  for (int q = 0; q < LA; ++q) {
    const int64_t mi = TA ? m0 + a_o + ASTEP * q : m0 + a_c;
    const int mr = (int)((mi < M ? mi : M - 1) - m0);
    const int kr = TA ? a_c : a_o + ASTEP * q;
    offa[q] = TA ? (uint32_t)(kr + mr * lda) : (uint32_t)(mr + kr * lda);
  }
#pragma unroll
  for (int q = 0; q < LB; ++q) {
    const int64_t ni = TB ? n0 + b_c : n0 + b_o + BSTEP * q;
    const int nr = (int)((ni < N ? ni : N - 1) - n0);
    const int kr = TB ? b_o + BSTEP * q : b_c;
    offb[q] = TB ? (uint32_t)(nr + kr * ldb) : (uint32_t)(kr + nr * ldb);
  }
  const int64_t a_tile = TA ? m0 * A.ld : m0, b_tile = TB ? n0 : n0 * B.ld;
  // real products: two register sets, a slab's loads issued two slabs
  // before it is used (complex ones use set 0 only)
  double ra0[NP][LA], rb0[NP][LB], ra1[NP][LA], rb1[NP][LB];
  auto gload = [&](int64_t k0, double (&ra)[NP][LA], double (&rb)[NP][LB]) {
    const int64_t ka = TA ? k0 : k0 * A.ld, kb_ = TB ? k0 * B.ld : k0;
    const double* pa[2] = {A.re + a_tile + ka, CPLX ? A.im + a_tile + ka : nullptr};
    const double* pb[2] = {B.re + b_tile + kb_, CPLX ? B.im + b_tile + kb_ : nullptr};
    if (k0 + GBK <= ke) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int q = 0; q < LA; ++q) ra[p][q] = pa[p][offa[q]];
#pragma unroll
        for (int q = 0; q < LB; ++q) rb[p][q] = pb[p][offb[q]];
      }
    } else {
      // the last slab: K indices beyond ke load from index ke - 1 and read as 0
      const int kl = (int)(ke - 1 - k0);
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int kr = TA ? a_c : a_o + ASTEP * q;
        const int kc = kr < kl ? kr : kl;
        const uint32_t o = TA ? offa[q] - (uint32_t)kr + (uint32_t)kc
                              : offa[q] - (uint32_t)(kr * lda) + (uint32_t)(kc * lda);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const double v = pa[p][o];
          ra[p][q] = kr <= kl ? v : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int kr = TB ? b_o + BSTEP * q : b_c;
        const int kc = kr < kl ? kr : kl;
        const uint32_t o = TB ? offb[q] - (uint32_t)(kr * ldb) + (uint32_t)(kc * ldb)
                              : offb[q] - (uint32_t)kr + (uint32_t)kc;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const double v = pb[p][o];
          rb[p][q] = kr <= kl ? v : 0.0;
        }
      }
    }
  };
  auto lstore = [&](int buf, const double (&ra)[NP][LA], const double (&rb)[NP][LB]) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        if (TA) As[buf][p][a_c][a_o + ASTEP * q] = alpha * ra[p][q];
        else As[buf][p][a_o + ASTEP * q][a_c] = alpha * ra[p][q];
      }
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        if (TB) Bs[buf][p][b_o + BSTEP * q][b_c] = rb[p][q];
        else Bs[buf][p][b_c][b_o + BSTEP * q] = rb[p][q];
      }
    }
  };

  const int64_t il = m0 + wm + (lane & 15), jl = n0 + wn + (lane >> 4);
  const bool use_c = beta != 0.0;
  // real: acc[0] = C.  complex: acc[0] = P1, acc[1] = P2, acc[2] = P3,
  // started at beta Re C, 0 and beta (Re C + Im C)
  constexpr int NA = CPLX ? 3 : 1;
  doublex4 acc[NA][XM][XN];
  // (the loads of C are all issued before the first is used, from offsets
  // clamped into C: loads in per-element branches would each wait in turn)
  if (use_c) {
#pragma unroll
    for (int x = 0; x < XM; ++x)
#pragma unroll
      for (int y = 0; y < XN; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = il + 16 * x, j = jl + 16 * y + 4 * r;
          const int64_t off = (i < M && j < N) ? i + j * C.ld : 0;
          acc[0][x][y][r] = C.re[off];
          if constexpr (CPLX) acc[1][x][y][r] = C.im[off];
        }
  }
#pragma unroll
  for (int x = 0; x < XM; ++x)
#pragma unroll
    for (int y = 0; y < XN; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = il + 16 * x, j = jl + 16 * y + 4 * r;
        const bool in = use_c && i < M && j < N;
        const double cr = in ? beta * acc[0][x][y][r] : 0.0;
        acc[0][x][y][r] = cr;
        if constexpr (CPLX) {
          const double ci = in ? beta * acc[1][x][y][r] : 0.0;
          acc[1][x][y][r] = 0.0;
          acc[2][x][y][r] = cr + ci;
        }
      }

  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 4) {
      const int kr = kk + (lane >> 4), r = lane & 15;
      double ar[NP][XM], br[NP][XN];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int x = 0; x < XM; ++x) ar[p][x] = As[buf][p][kr][wm + 16 * x + r];
#pragma unroll
        for (int y = 0; y < XN; ++y) br[p][y] = Bs[buf][p][kr][wn + 16 * y + r];
      }
#pragma unroll
      for (int x = 0; x < XM; ++x)
#pragma unroll
        for (int y = 0; y < XN; ++y) {
          acc[0][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(br[0][y], ar[0][x], acc[0][x][y], 0, 0, 0);
          if constexpr (CPLX) {
            acc[1][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(br[1][y], ar[1][x], acc[1][x][y], 0, 0, 0);
            acc[2][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(br[0][y] + br[1][y], ar[0][x] + ar[1][x],
                                                                acc[2][x][y], 0, 0, 0);
          }
        }
    }
  };
  if constexpr (!CPLX) {
    // slab s lives in LDS buffer s % 2; register set 0 carries the even
    // slabs, set 1 the odd ones.  Each LDS buffer is rewritten only after the
    // barrier that follows its last read.
    gload(0, ra0, rb0);
    lstore(0, ra0, rb0);
    if (GBK < ke) gload(GBK, ra1, rb1);
    __syncthreads();
    for (int64_t k0 = 0; k0 < ke; k0 += 2 * GBK) {
      if (k0 + 2 * GBK < ke) gload(k0 + 2 * GBK, ra0, rb0);
      compute(0);
      if (k0 + GBK < ke) lstore(1, ra1, rb1);
      __syncthreads();
      if (k0 + GBK >= ke) break;
      if (k0 + 3 * GBK < ke) gload(k0 + 3 * GBK, ra1, rb1);
      compute(1);
      if (k0 + 2 * GBK < ke) lstore(0, ra0, rb0);
      __syncthreads();
    }
  } else {
    // complex: the three accumulator sets leave room for one register set,
    // so each slab's loads are issued one slab ahead
    gload(0, ra0, rb0);
    lstore(0, ra0, rb0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = 0; k0 < ke; k0 += GBK) {
      const bool more = k0 + GBK < ke;
      if (more) gload(k0 + GBK, ra0, rb0);
      compute(buf);
      // the other buffer was last read before the previous barrier
      if (more) lstore(buf ^ 1, ra0, rb0);
      __syncthreads();
      buf ^= 1;
    }
  }

#pragma unroll
  for (int x = 0; x < XM; ++x)
#pragma unroll
    for (int y = 0; y < XN; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = il + 16 * x, j = jl + 16 * y + 4 * r;
        if (i < M && j < N) {
          if constexpr (CPLX) {
            const double p1 = acc[0][x][y][r], p2 = acc[1][x][y][r], p3 = acc[2][x][y][r];
            C.re[i + j * C.ld] = p1 - p2;
            C.im[i + j * C.ld] = p3 - p1 - p2;
          } else {
            C.re[i + j * C.ld] = acc[0][x][y][r];
          }
        }
      }
}

// C_b = sum over splits of the partial tiles (alpha applied) + beta C_b.
template <typename T, bool CPLX>
__global__ void k_splitk_sum(int64_t M, int64_t N, int splits, int batch, const T* part, T beta,
                             DMat<T> C, int tri) {
  constexpr int NP = CPLX ? 2 : 1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int b = blockIdx.y;
  C = C.item(b);
  const int64_t i = e % M, j = e / M;
  if (tri && j > i) return;
  const int64_t plane = M * N;
  T sr = 0, si = 0;
  for (int s = 0; s < splits; ++s) {
    const T* p = part + ((int64_t)(s * batch + b) * NP) * plane;
    sr += p[e];
    if constexpr (CPLX) si += p[plane + e];
  }
  const int64_t off = i + j * C.ld;
  if (beta != T(0)) {
    sr += beta * C.re[off];
    if constexpr (CPLX) si += beta * C.im[off];
  }
  C.re[off] = sr;
  if constexpr (CPLX) C.im[off] = si;
}

// Per-stream split-K workspace (grown on demand; a stream's earlier work is
// finished before its buffer is replaced).
static std::mutex ws_mu;
static std::map<std::pair<int, hipStream_t>, DevBuf> ws_map;
static void* splitk_workspace(hipStream_t s, size_t bytes) {
  std::mutex& mu = ws_mu;
  auto& ws = ws_map;
  int dev = 0;
  RFD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  DevBuf& w = ws[{dev, s}];
  if (w.bytes < bytes) {
    if (w.p) RFD_HIP(hipStreamSynchronize(s));
    w.alloc(bytes);
  }
  return w.p;
}

void release_stream_resources(hipStream_t s) {
  int dev = 0;
  RFD_HIP(hipGetDevice(&dev));
  RFD_HIP(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> g(ws_mu);
  ws_map.erase({dev, s});
}

template <typename T, bool CPLX, int BM, int BN>
static void launch(hipStream_t s, bool ta, bool tb, dim3 g, int64_t M, int64_t N, int64_t K,
                   T alpha, T beta, DMat<T> A, DMat<T> B, DMat<T> C, int splits, int64_t kchunk,
                   T* part, int va, int vb, int tri, hipEvent_t ea, hipEvent_t eb) {
#define RFD_GEMM_GO(TA_, TB_)                                                                  \
  hipExtLaunchKernelGGL(k_gemm<T, CPLX, TA_, TB_, BM, BN>, g, dim3(256), 0, s, ea, eb, 0, M, N, \
                        K, alpha, beta, A, B, C, splits, kchunk, part, va, vb, tri)
  if (!ta && !tb) RFD_GEMM_GO(false, false);
  else if (ta && !tb) RFD_GEMM_GO(true, false);
  else if (!ta && tb) RFD_GEMM_GO(false, true);
  else RFD_GEMM_GO(true, true);
#undef RFD_GEMM_GO
}

template <bool CPLX, int BM, int BN>
static void launch_d(hipStream_t s, bool ta, bool tb, dim3 g, int64_t M, int64_t N, int64_t K,
                     double alpha, double beta, DMat<double> A, DMat<double> B, DMat<double> C,
                     int tri, hipEvent_t ea, hipEvent_t eb) {
#define RFD_DGEMM_GO(TA_, TB_)                                                                  \
  hipExtLaunchKernelGGL(k_dgemm<CPLX, TA_, TB_, BM, BN>, g, dim3(256), 0, s, ea, eb, 0, M, N, K, \
                        alpha, beta, A, B, C, tri)
  if (!ta && !tb) RFD_DGEMM_GO(false, false);
  else if (ta && !tb) RFD_DGEMM_GO(true, false);
  else if (!ta && tb) RFD_DGEMM_GO(false, true);
  else RFD_DGEMM_GO(true, true);
#undef RFD_DGEMM_GO
}

// Workgroups of one k_gemm variant that the device holds at once (per-CU
// occupancy from registers and LDS, times the CU count), per device.
template <typename T, bool CPLX, int BM, int BN>
static int64_t resident_blocks() {
  static std::atomic<int64_t> cached[16];
  int dev = 0;
  RFD_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < 16) {
    const int64_t c = cached[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int per_cu = 0, cus = 0;
  RFD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(k_gemm<T, CPLX, false, false, BM, BN>), 256, 0));
  RFD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t r = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);
  if (dev >= 0 && dev < 16) cached[dev].store(r, std::memory_order_relaxed);
  return r;
}

template <typename T>
static int64_t resident_for(bool cplx, int bt) {
  if constexpr (sizeof(T) == 4) {
    if (bt == 128) return resident_blocks<T, false, 128, 128>();
    return cplx ? resident_blocks<T, true, 64, 64>() : resident_blocks<T, false, 64, 64>();
  } else {
    return cplx ? resident_blocks<T, true, 64, 64>() : resident_blocks<T, false, 64, 64>();
  }
}

template <typename T>
static bool aligned16(const DMat<T>& X, int vw) {
  auto al = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
  return X.ld % vw == 0 && X.bs % vw == 0 && al(X.re) && (X.im == nullptr || al(X.im));
}

// ---------------------------------------------------------------------------
// Tile choices measured by an autotuner (set_gemm_tuning): per class of
// (precision, complex, transposes, floor log2 of M, N, K and the batch) the variant that
// ran fastest -- 1: k_gemm 64 x 64, 2: k_gemm 128 x 128 (real FP32), 3:
// k_dgemm (FP64).  Classes without an entry keep the built-in rules, and so
// do lower-triangle and triangular-operand products.  A variant that cannot
// run a product (an aliased output, sizes beyond its limits) falls back to
// the built-in rules; the test hook that forces a variant reports it instead.
// ---------------------------------------------------------------------------
namespace {
std::mutex tune_mu;
std::shared_ptr<const std::unordered_map<uint64_t, int>> tune_table;
thread_local int forced_variant = 0;

int ilog2(int64_t x) {
  int l = 0;
  while (x > 1 && l < 62) {
    x >>= 1;
    ++l;
  }
  return l;
}

uint64_t tune_key(int dt, int cplx, int ta, int tb, int lm, int ln, int lk, int lb) {
  return (uint64_t)dt | (uint64_t)cplx << 1 | (uint64_t)ta << 2 | (uint64_t)tb << 3 |
         (uint64_t)lm << 4 | (uint64_t)ln << 12 | (uint64_t)lk << 20 | (uint64_t)lb << 28;
}

int tuned_variant(bool fp64, bool cplx, bool ta, bool tb, int64_t M, int64_t N, int64_t K,
                  int batch) {
  if (forced_variant) return forced_variant;
  std::shared_ptr<const std::unordered_map<uint64_t, int>> t;
  {
    std::lock_guard<std::mutex> g(tune_mu);
    t = tune_table;
  }
  if (!t || t->empty()) return 0;
  const auto it =
      t->find(tune_key(fp64, cplx, ta, tb, ilog2(M), ilog2(N), ilog2(K), ilog2(batch)));
  return it == t->end() ? 0 : it->second;
}
}  // namespace

void set_gemm_tuning(const int32_t* e, int count) {
  if (count < 0 || (count > 0 && !e)) throw Error(ST_EINVAL, "gemm tuning: bad table");
  auto t = std::make_shared<std::unordered_map<uint64_t, int>>();
  for (int i = 0; i < count; ++i) {
    const int32_t* r = e + 9 * (int64_t)i;
    const int dt = r[0], cplx = r[1], ta = r[2], tb = r[3], v = r[8];
    bool ok = (dt == 0 || dt == 1) && (cplx == 0 || cplx == 1) && (ta == 0 || ta == 1) &&
              (tb == 0 || tb == 1) && v >= 1 && v <= 3;
    for (int q = 4; q < 8; ++q) ok = ok && r[q] >= 0 && r[q] <= 62;
    if (ok && v == 2) ok = dt == 0 && cplx == 0;
    if (ok && v == 3) ok = dt == 1;
    if (!ok) throw Error(ST_EINVAL, "gemm tuning: entry " + std::to_string(i) + " is malformed");
    (*t)[tune_key(dt, cplx, ta, tb, r[4], r[5], r[6], r[7])] = v;
  }
  std::lock_guard<std::mutex> g(tune_mu);
  tune_table = std::move(t);
}

int gemm_tuning_size() {
  std::lock_guard<std::mutex> g(tune_mu);
  return tune_table ? (int)tune_table->size() : 0;
}

void gemm_force_variant(int v) { forced_variant = v; }

// fixed_part: caller-provided memory of fixed_bytes for the split-K partial
// tiles (the split count is lowered until they fit; no allocation and no
// kernel accounting), or null for the per-stream workspace.
// triub: op(B) is upper triangular (zero below its diagonal); the large-tile
// FP64 kernel then skips the zero K range of each tile column (other paths
// multiply the zeros).
template <typename T>
static void gemm_impl(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha,
                      DMat<T> A, DMat<T> B, T beta, DMat<T> C, int batch, int tri,
                      T* fixed_part = nullptr, size_t fixed_bytes = 0, bool triub = false) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  const bool cplx = C.cplx();
  const int NP = cplx ? 2 : 1;
  constexpr int VW = 16 / (int)sizeof(T);
  // tile: 128 x 128 for real FP32 products large enough to fill the chip with
  // it, over a long K (with a few K slabs the large tile cannot hide its
  // prologue and epilogue).  Complex products keep 64 x 64: measured on
  // gfx950 at 105-120 TF/s against 64-88 for the 128-wide complex tile, whose
  // accumulators leave one wave per SIMD.
  // Large real FP64 products go to k_dgemm below; the rest keep the 64 x 64
  // tile here.
  const int var = (tri || triub) ? 0 : tuned_variant(sizeof(T) == 8, cplx, ta, tb, M, N, K, batch);
  if (forced_variant == 2 && (sizeof(T) != 4 || cplx))
    throw Error(ST_EINVAL, "gemm variant 2 (128 x 128) takes real FP32 products only");
  if (forced_variant == 3 && sizeof(T) != 8)
    throw Error(ST_EINVAL, "gemm variant 3 (k_dgemm) takes FP64 products only");
  const bool big_ok = sizeof(T) == 4 && !cplx && M >= 128 && N >= 128 && K >= 256;
  const int64_t t128 = ((M + 127) / 128) * ((N + 127) / 128) * batch;
  const int bt = var == 2 ? 128 : var == 1 ? 64 : (big_ok && t128 >= 240) ? 128 : 64;
  const int64_t gm = (M + bt - 1) / bt, gn = (N + bt - 1) / bt;
  // tiles that do work (a lower-triangle product skips the strictly upper ones)
  const int64_t tiles = (tri ? gm * (gm + 1) / 2 : gm * gn) * batch;
  // split K when the tiles fill less than half the device, into as many
  // chunks as give one full round of resident workgroups: a second, partial
  // round would take as long as the first
  const int64_t slots = resident_for<T>(cplx, bt);
  int splits = 1;
  if (tiles < slots && K >= 256) {
    // fewer tiles than one round of resident workgroups: split K into the
    // chunk count that minimises rounds x (chunk length + a per-workgroup
    // overhead worth 256 of K)
    const int64_t smax = std::min<int64_t>(K / 64, 64);
    double best = (double)K + 256.0;
    for (int64_t sp = 2; sp <= smax; ++sp) {
      const double rounds = (double)((tiles * sp + slots - 1) / slots);
      const double c = rounds * ((double)K / (double)sp + 256.0);
      if (c < best) {
        best = c;
        splits = (int)sp;
      }
    }
    while (splits > 1 && (double)splits * batch * M * N * NP * sizeof(T) > 512.0 * (1 << 20))
      --splits;
    while (splits > 1 && (int64_t)splits * batch > 65535) --splits;
    if (splits < 1) splits = 1;
  }
  // large FP64 products go to k_dgemm (unless the output overwrites an
  // operand: its tiles would read what other tiles have written, or a complex
  // operand has no imaginary plane)
  if constexpr (sizeof(T) == 8) {
    const bool alias = C.re == A.re || C.re == B.re ||
                       (cplx && (C.im == A.im || C.im == B.im || !A.im || !B.im));
    if (!alias && batch <= 65535) {
      // real: 64 x 128 tiles when they fill the device twice and a 128-wide
      // tile column is not mostly padding (measured on the solve's shapes:
      // 63 / 54 TFLOP/s against 50 / 40 for 64 x 64; 128 x 128 tiles ran no
      // faster and need more registers than two waves per SIMD allow);
      // complex: 64 x 64 tiles
      const int bn = cplx ? 64 : 128;
      const int64_t nt = (N + bn - 1) / bn, g64 = (M + 63) / 64;
      const int64_t t64 = (tri ? g64 * (g64 + 1) / (bn / 32) : g64 * nt) * batch;
      const bool wide_ok = cplx || nt * bn <= N + N / 4 || N >= 512;
      // per-thread element offsets within a tile's K slab must fit 32 bits
      const int64_t span_a = ta ? (int64_t)GBK + 64 * A.ld : (int64_t)64 + GBK * A.ld;
      const int64_t span_b = tb ? (int64_t)bn + GBK * B.ld : (int64_t)GBK + bn * B.ld;
      // (short K, as in the LU trailing updates, stays on the 64 x 64 tile:
      // a few K slabs do not repay the larger tile's epilogue)
      const bool fits = K >= GBK && nt <= 65535 && g64 <= 0x7fffffff &&
                        span_a < (int64_t(1) << 31) && span_b < (int64_t(1) << 31);
      if (forced_variant == 3 && !fits)
        throw Error(ST_EINVAL, "gemm variant 3 (k_dgemm) cannot run this product");
      const bool rule = wide_ok && t64 >= 512 && K >= 256;
      if (fits && (var == 3 || (var == 0 && rule))) {
        const int key = KA_DGEMM + (cplx ? 4 : 0) + (ta ? 2 : 0) + (tb ? 1 : 0);
        const double outs = tri ? 0.5 * (double)N * (double)(N + 1) : (double)M * (double)N;
        // (with a triangular op(B), column j takes min(j + 1, K) terms)
        const double kavg = triub ? (double)(std::min(N, K) * (std::min(N, K) + 1) / 2 +
                                             std::max<int64_t>(N - K, 0) * K) / (double)N
                                  : (double)K;
        const double flops = (cplx ? 8.0 : 2.0) * outs * kavg * batch;
        const double bytes = (cplx ? 2.0 : 1.0) * 8.0 *
                             ((double)M * K + (double)K * N + (beta != T(0) ? 2.0 : 1.0) * outs) *
                             batch;
        KernelAccount::Scope acct(s, fixed_part ? -1 : key, flops, bytes);
        dim3 g((unsigned)g64, (unsigned)nt, (unsigned)batch);
        const int dtri = triub ? 2 : (tri ? 1 : 0);
        if (cplx)
          launch_d<true, 64, 64>(s, ta, tb, g, M, N, K, alpha, beta, A, B, C, dtri, acct.start(),
                                 acct.stop());
        else
          launch_d<false, 64, 128>(s, ta, tb, g, M, N, K, alpha, beta, A, B, C, dtri,
                                   acct.start(), acct.stop());
        RFD_CHECK_LAUNCH();
        return;
      }
    }
  }
  if (forced_variant == 3) throw Error(ST_EINVAL, "gemm variant 3 (k_dgemm) cannot run this product");
  if ((int64_t)batch * splits > 65535) throw Error(ST_EINVAL, "gemm: batch too large");
  if (gm * gn * batch * splits >= ((int64_t)1 << 32)) throw Error(ST_EINVAL, "gemm: grid too large");
  if (gm > 0x7fffffff || gn > 65535) throw Error(ST_EINVAL, "gemm: matrix too large");
  int64_t kchunk = K;
  if (splits > 1) {
    kchunk = round_up((K + splits - 1) / splits, GBK);
    splits = (int)((K + kchunk - 1) / kchunk);
  }
  if (fixed_part) {
    while (splits > 1 && sizeof(T) * (size_t)splits * batch * M * N * NP > fixed_bytes) {
      --splits;
      kchunk = round_up((K + splits - 1) / splits, GBK);
      splits = (int)((K + kchunk - 1) / kchunk);
    }
    if (splits <= 1) {
      splits = 1;
      kchunk = K;
    }
  }
  T* part = nullptr;
  if (splits > 1)
    part = fixed_part ? fixed_part
                      : static_cast<T*>(splitk_workspace(s, sizeof(T) * (size_t)splits * batch * M *
                                                                N * NP));
  const int va = aligned16(A, VW), vb = aligned16(B, VW);
  dim3 g((unsigned)gm, (unsigned)gn, (unsigned)(batch * splits));
  const int key = (sizeof(T) == 8 ? 8 : 0) + (cplx ? 4 : 0) + (ta ? 2 : 0) + (tb ? 1 : 0);
  // a lower-triangle product counts the N (N + 1) / 2 entries it must produce
  const double outs = tri ? 0.5 * (double)N * (double)(N + 1) : (double)M * (double)N;
  const double flops = (cplx ? 8.0 : 2.0) * outs * (double)K * batch;
  // algorithmic bytes: A and B read once, C written (and read when beta != 0)
  const double planes = cplx ? 2.0 : 1.0;
  const double bytes = planes * sizeof(T) *
                       ((double)M * K + (double)K * N + (beta != T(0) ? 2.0 : 1.0) * outs) * batch;
  KernelAccount::Scope acct(s, fixed_part ? -1 : key, flops, bytes);
  if constexpr (sizeof(T) == 4) {
    if (bt == 128)
      launch<T, false, 128, 128>(s, ta, tb, g, M, N, K, alpha, beta, A, B, C, splits, kchunk, part, va, vb, tri, acct.start(), splits > 1 ? nullptr : acct.stop());
  }
  if (bt == 64) {
    if (cplx) launch<T, true, 64, 64>(s, ta, tb, g, M, N, K, alpha, beta, A, B, C, splits, kchunk, part, va, vb, tri, acct.start(), splits > 1 ? nullptr : acct.stop());
    else launch<T, false, 64, 64>(s, ta, tb, g, M, N, K, alpha, beta, A, B, C, splits, kchunk, part, va, vb, tri, acct.start(), splits > 1 ? nullptr : acct.stop());
  }
  RFD_CHECK_LAUNCH();
  if (splits > 1) {
    dim3 gr(grid1(M * N), (unsigned)batch);
    if (cplx)
      hipExtLaunchKernelGGL(k_splitk_sum<T, true>, gr, dim3(256), 0, s, nullptr, acct.stop(), 0, M,
                            N, splits, batch, (const T*)part, beta, C, tri);
    else
      hipExtLaunchKernelGGL(k_splitk_sum<T, false>, gr, dim3(256), 0, s, nullptr, acct.stop(), 0,
                            M, N, splits, batch, (const T*)part, beta, C, tri);
    RFD_CHECK_LAUNCH();
  }
}

template <typename T>
void gemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha, DMat<T> A,
          DMat<T> B, T beta, DMat<T> C, int batch) {
  gemm_impl<T>(s, ta, tb, M, N, K, alpha, A, B, beta, C, batch, 0);
}

template <typename T>
void gemm_lower(hipStream_t s, bool ta, bool tb, int64_t N, int64_t K, T alpha, DMat<T> A,
                DMat<T> B, T beta, DMat<T> C, int batch) {
  gemm_impl<T>(s, ta, tb, N, N, K, alpha, A, B, beta, C, batch, 1);
}

void gemm_triu_b(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, DMat<double> A,
                 DMat<double> B, double beta, DMat<double> C, int batch) {
  if (C.cplx()) throw Error(ST_EINVAL, "gemm_triu_b: real operands only");
  gemm_impl<double>(s, false, false, M, N, K, alpha, A, B, beta, C, batch, 0, nullptr, 0, true);
}

// ---------------------------------------------------------------------------
// Products for callers that cannot allocate: the split-K partial tiles go to
// a file-scope device array instead of the per-stream workspace.  Each device
// holds its own copy; its address is looked up once per device (with that
// device current) and kept.  Every call on a device shares the array, so
// calls that overlap on one device race; nothing in it needs to start at zero
// (every partial tile is written before it is summed).
static __device__ __align__(256) unsigned char scratch[GEMM_STATIC_SCRATCH_BYTES];

static void* static_scratch() {
  static std::mutex mu;
  static void* ptr[64] = {};
  int dev = 0;
  RFD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(ST_EDEVICE, "gemm_static: device index out of range");
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(ST_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    ptr[dev] = p;
  }
  return ptr[dev];
}

template <typename T>
void gemm_static(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha,
                 DMat<T> A, DMat<T> B, T beta, DMat<T> C, int batch) {
  const int64_t NP = C.cplx() ? 2 : 1;
  if (M > 0 && N > 0 && batch > 0 &&
      (double)M * N * batch * NP * sizeof(T) > 0.5 * (double)GEMM_STATIC_SCRATCH_BYTES)
    throw Error(ST_EINVAL, "gemm_static: the output (M N batch planes elements) may take at most " +
                               std::to_string(GEMM_STATIC_SCRATCH_BYTES / 2) + " bytes");
  gemm_impl<T>(s, ta, tb, M, N, K, alpha, A, B, beta, C, batch, 0,
               static_cast<T*>(static_scratch()), GEMM_STATIC_SCRATCH_BYTES);
}

#define RFD_GEMM_INST(T)                                                                        \
  template void gemm<T>(hipStream_t, bool, bool, int64_t, int64_t, int64_t, T, DMat<T>, DMat<T>, \
                        T, DMat<T>, int);                                                        \
  template void gemm_lower<T>(hipStream_t, bool, bool, int64_t, int64_t, T, DMat<T>, DMat<T>, T, \
                              DMat<T>, int);                                                  \
  template void gemm_static<T>(hipStream_t, bool, bool, int64_t, int64_t, int64_t, T, DMat<T>,  \
                               DMat<T>, T, DMat<T>, int);
RFD_GEMM_INST(float)
RFD_GEMM_INST(double)

}  // namespace rfd
