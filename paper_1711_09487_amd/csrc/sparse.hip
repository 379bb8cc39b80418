// Sparse-structured kernels of the interface filter (see sparse.hpp).
#include "sparse.hpp"

namespace rfd {

__device__ inline void atomic_max_nonneg_d(double* p, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_expand_shifted(DMat<T> K, int64_t D, int p, int pole0, const int32_t* dj,
                                 DevPairCsr B, Shifts z, int sig_real, double sigma) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y, j = b % p, l = pole0 + b / p;
  if (r >= D) return;
  DMat<T> k = K.item(b);
  const int d = dj[j];
  if (r >= d) {
    k.re[r + r * k.ld] = T(1);
    return;
  }
  const double zr = sig_real ? sigma : z.z[2 * l], zi = sig_real ? 0.0 : z.z[2 * l + 1];
  const int64_t* ptr = B.ptr + B.roff[j];
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const int64_t c = B.idx[e];
    const int64_t off = r + c * k.ld;
    k.re[off] = (T)(B.a[e] - zr * B.m[e]);
    if (k.im) k.im[off] = (T)(-zi * B.m[e]);
  }
}

template <typename T>
void expand_shifted(hipStream_t s, DMat<T> K, int64_t D, int p, int npoles, int pole0,
                    const int32_t* dj, DevPairCsr B, Shifts z, bool sig_real, double sigma) {
  dim3 g(grid1(D), p * npoles);
  k_expand_shifted<T><<<g, 256, 0, s>>>(K, D, p, pole0, dj, B, z, sig_real ? 1 : 0, sigma);
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_expand_rhs(DMat<T> R, int p, int pole0, const int32_t* dj, DevPairCsr E,
                             Shifts z) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y, j = b % p, l = pole0 + b / p;
  if (r >= dj[j]) return;
  DMat<T> x = R.item(b);
  const double zr = z.z[2 * l], zi = z.z[2 * l + 1];
  const int64_t* ptr = E.ptr + E.roff[j];
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const int64_t c = E.idx[e];
    const int64_t off = r + c * x.ld;
    x.re[off] = (T)(E.a[e] - zr * E.m[e]);
    if (x.im) x.im[off] = (T)(-zi * E.m[e]);
  }
}

template <typename T>
void expand_rhs(hipStream_t s, DMat<T> R, int p, int npoles, int pole0, const int32_t* dj,
                DevPairCsr E, Shifts z) {
  // rows up to the largest d_j; the kernel bounds each item by its own d_j
  int64_t D = R.ld;
  dim3 g(grid1(D), p * npoles);
  k_expand_rhs<T><<<g, 256, 0, s>>>(R, p, pole0, dj, E, z);
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// FP64 residual of the Schur-contribution solves, R = E_z - K_z X per item
// (local CSR of B_j and E_j with their mass values, shift of the item's pole),
// and max |R| into rmax.  A thread owns one row r and RS_C consecutive
// columns: it reads the row's
// CSR entries and forms the shifted values once, then gathers the columns'
// entries of X together.
constexpr int RS_C = 8;
__global__ void k_residual_shifted(DMat<double> X, DMat<double> R, int64_t D, int64_t SJ, int p,
                                   int pole0, const int32_t* dj, const int32_t* sj, DevPairCsr B,
                                   DevPairCsr E, Shifts z, double* rmax) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y, j = b % p, l = pole0 + b / p;
  const int64_t ncg = (SJ + RS_C - 1) / RS_C;
  double mx = 0;
  if (t0 < D * ncg) {
    const int64_t r = t0 % D, c0 = (t0 / D) * RS_C;
    DMat<double> x = X.item(b), rr = R.item(b);
    const int64_t dr = dj[j], sc = sj[j];
    double vr[RS_C], vi[RS_C];
#pragma unroll
    for (int q = 0; q < RS_C; ++q) vr[q] = vi[q] = 0.0;
    if (r < dr) {
      const double zr = z.z[2 * l], zi = z.z[2 * l + 1];
      const int64_t* pe = E.ptr + E.roff[j];
      for (int64_t e = pe[r]; e < pe[r + 1]; ++e) {
        const int64_t c = E.idx[e] - c0;
        const double er = E.a[e] - zr * E.m[e], ei = -zi * E.m[e];
#pragma unroll
        for (int q = 0; q < RS_C; ++q)
          if (q == c) {
            vr[q] += er;
            vi[q] += ei;
          }
      }
      const int64_t* pb = B.ptr + B.roff[j];
      for (int64_t e = pb[r]; e < pb[r + 1]; ++e) {
        const double kr = B.a[e] - zr * B.m[e], ki = -zi * B.m[e];
        const int64_t base = B.idx[e] + c0 * x.ld;
        double xr[RS_C], xi[RS_C];
#pragma unroll
        for (int q = 0; q < RS_C; ++q) {
          const bool ok = c0 + q < sc;
          xr[q] = ok ? x.re[base + q * x.ld] : 0.0;
          xi[q] = ok ? x.im[base + q * x.ld] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < RS_C; ++q) {
          vr[q] -= kr * xr[q] - ki * xi[q];
          vi[q] -= kr * xi[q] + ki * xr[q];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RS_C; ++q) {
      const int64_t c = c0 + q;
      if (c >= SJ) break;
      const bool ok = r < dr && c < sc;
      const double wr = ok ? vr[q] : 0.0, wi = ok ? vi[q] : 0.0;
      rr.re[r + c * rr.ld] = wr;
      rr.im[r + c * rr.ld] = wi;
      if (ok) {
        const double m = fmax(fabs(wr), fabs(wi));
        mx = (m == m) ? fmax(mx, m) : INFINITY;
      }
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0) atomic_max_nonneg_d(rmax, red[0]);
}

void residual_shifted(hipStream_t s, DMat<double> X, DMat<double> R, int64_t D, int64_t SJ, int p,
                      int npoles, int pole0, const int32_t* dj, const int32_t* sj, DevPairCsr B,
                      DevPairCsr E, Shifts z, double* rmax) {
  dim3 g(grid1(D * ((SJ + RS_C - 1) / RS_C)), p * npoles);
  k_residual_shifted<<<g, 256, 0, s>>>(X, R, D, SJ, p, pole0, dj, sj, B, E, z, rmax);
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
__global__ void k_schur_init(DMat<double> S, int64_t s_act, int64_t SP, int pole0, DevPairCsr Cc,
                             Shifts z) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y, l = pole0 + b;
  if (r >= SP) return;
  DMat<double> x = S.item(b);
  if (r >= s_act) {
    x.re[r + r * x.ld] = 1.0;
    return;
  }
  const double zr = z.z[2 * l], zi = z.z[2 * l + 1];
  for (int64_t e = Cc.ptr[r]; e < Cc.ptr[r + 1]; ++e) {
    const int64_t off = r + (int64_t)Cc.idx[e] * x.ld;
    x.re[off] = Cc.a[e] - zr * Cc.m[e];
    x.im[off] = -zi * Cc.m[e];
  }
}

void schur_init(hipStream_t s, DMat<double> S, int64_t s_act, int64_t SP, int npoles, int pole0,
                DevPairCsr Cc, Shifts z) {
  dim3 g(grid1(SP), npoles);
  k_schur_init<<<g, 256, 0, s>>>(S, s_act, SP, pole0, Cc, z);
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Thread per (a, b) of item (member i, local pole l).  Subdomains in one
// launch have disjoint adjacency sets, so every S entry has one writer.
__global__ void k_schur_scatter(DMat<double> S, DMat<double> X, int64_t SJ, int p, int pole0,
                                const int32_t* members, int nmembers, const int32_t* sj,
                                const int32_t* adj, DevPairCsr Et, Shifts z) {
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int it = blockIdx.y % nmembers, ll = blockIdx.y / nmembers;
  const int j = members[it], l = pole0 + ll;
  const int n_j = sj[j];
  if (e0 >= (int64_t)n_j * n_j) return;
  const int a = (int)(e0 % n_j), bcol = (int)(e0 / n_j);
  DMat<double> x = X.item((int64_t)ll * p + j);
  const double zr = z.z[2 * l], zi = z.z[2 * l + 1];
  const int64_t* pt = Et.ptr + Et.roff[j];
  double gr = 0, gi = 0;
  for (int64_t e = pt[a]; e < pt[a + 1]; ++e) {
    const double er = Et.a[e] - zr * Et.m[e], ei = -zi * Et.m[e];
    const int64_t q = Et.idx[e] + (int64_t)bcol * x.ld;
    const double xr = x.re[q], xi = x.im[q];
    gr += er * xr - ei * xi;
    gi += er * xi + ei * xr;
  }
  DMat<double> sm = S.item(ll);
  const int64_t ia = adj[(int64_t)j * SJ + a], ib = adj[(int64_t)j * SJ + bcol];
  const int64_t off = ia + ib * sm.ld;
  sm.re[off] -= gr;
  sm.im[off] -= gi;
}

void schur_scatter(hipStream_t s, DMat<double> S, DMat<double> X, int64_t SJ, int p, int npoles,
                   int pole0, const int32_t* members, int nmembers, const int32_t* sj,
                   const int32_t* adj, DevPairCsr Et, Shifts z) {
  if (nmembers <= 0) return;
  dim3 g(grid1(SJ * SJ), nmembers * npoles);
  k_schur_scatter<<<g, 256, 0, s>>>(S, X, SJ, p, pole0, members, nmembers, sj, adj, Et, z);
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
__global__ void k_broadcast_rhs(const double* Y, int64_t ldy, int64_t s_act, int64_t m,
                                DMat<double> Yc, int64_t SP, int64_t MP) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= SP * MP) return;
  const int64_t r = e % SP, c = e / SP;
  DMat<double> x = Yc.item(blockIdx.y);
  x.re[r + c * x.ld] = (r < s_act && c < m) ? Y[r + c * ldy] : 0.0;
  x.im[r + c * x.ld] = 0.0;
}

void broadcast_rhs(hipStream_t s, const double* Y, int64_t ldy, int64_t s_act, int64_t m,
                   DMat<double> Yc, int64_t SP, int64_t MP, int npoles) {
  dim3 g(grid1(SP * MP), npoles);
  k_broadcast_rhs<<<g, 256, 0, s>>>(Y, ldy, s_act, m, Yc, SP, MP);
  RFD_CHECK_LAUNCH();
}

__global__ void k_filter_accumulate(DMat<double> X, const double* omega, int npoles, double* W,
                                    int64_t ldw, int64_t s_act, int64_t m, int add) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s_act * m) return;
  const int64_t r = e % s_act, c = e / s_act;
  double acc = add ? W[r + c * ldw] : 0.0;
  for (int l = 0; l < npoles; ++l) {
    DMat<double> x = X.item(l);
    const int64_t q = r + c * x.ld;
    acc += 2.0 * (omega[2 * l] * x.re[q] - omega[2 * l + 1] * x.im[q]);
  }
  W[r + c * ldw] = acc;
}

void filter_accumulate(hipStream_t s, DMat<double> X, const double* omega, int npoles, double* W,
                       int64_t ldw, int64_t s_act, int64_t m, bool add) {
  k_filter_accumulate<<<grid1(s_act * m), 256, 0, s>>>(X, omega, npoles, W, ldw, s_act, m,
                                                       add ? 1 : 0);
  RFD_CHECK_LAUNCH();
}

template void expand_shifted<float>(hipStream_t, DMat<float>, int64_t, int, int, int,
                                    const int32_t*, DevPairCsr, Shifts, bool, double);
template void expand_shifted<double>(hipStream_t, DMat<double>, int64_t, int, int, int,
                                     const int32_t*, DevPairCsr, Shifts, bool, double);
template void expand_rhs<float>(hipStream_t, DMat<float>, int, int, int, const int32_t*,
                                DevPairCsr, Shifts);
template void expand_rhs<double>(hipStream_t, DMat<double>, int, int, int, const int32_t*,
                                 DevPairCsr, Shifts);

}  // namespace rfd
