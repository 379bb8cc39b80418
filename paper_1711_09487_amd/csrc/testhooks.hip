// Kernel-level entry points for the test-suite: each wraps one batched
// building block so that it can be checked element by element against a
// host computation.  Declared in include/rfd_testing.h.
#include <cstring>

#include <algorithm>
#include <cmath>

#include "dense.hpp"
#include "eig.hpp"
#include "pencil.hpp"
#include "rfd_capi_util.hpp"

using namespace rfd;

template <typename T>
static DMat<T> dm(void* re, void* im, int64_t ld, int64_t bs) {
  DMat<T> m;
  m.re = (T*)re;
  m.im = (T*)im;
  m.ld = ld;
  m.bs = bs;
  return m;
}

// Operands of a product that will run must exist: null real planes, or a
// complex C with a null imaginary operand plane that is not meant as real,
// are rejected before anything is launched.
static void check_gemm_args(int64_t M, int64_t N, int64_t K, int batch, const void* a_re,
                            const void* b_re, const void* c_re, const void* a_im,
                            const void* b_im, const void* c_im) {
  if (M < 0 || N < 0 || K < 0 || batch < 0) throw Error(ST_EINVAL, "gemm: negative size");
  if (M == 0 || N == 0 || batch == 0) return;
  if (!c_re || (K > 0 && (!a_re || !b_re)))
    throw Error(ST_EINVAL, "gemm: null operand pointer");
  (void)a_im;
  (void)b_im;
  (void)c_im;
}

extern "C" int rfd_test_gemm(int dtype, int ta, int tb, int64_t M, int64_t N, int64_t K,
                             double alpha, double beta, void* a_re, void* a_im, int64_t lda,
                             int64_t sa, void* b_re, void* b_im, int64_t ldb, int64_t sb,
                             void* c_re, void* c_im, int64_t ldc, int64_t sc, int batch,
                             void* stream) {
  return capi_guard([&] {
    hipStream_t s = (hipStream_t)stream;
    check_gemm_args(M, N, K, batch, a_re, b_re, c_re, a_im, b_im, c_im);
    if (dtype == 0)
      gemm<float>(s, ta, tb, M, N, K, (float)alpha, dm<float>(a_re, a_im, lda, sa),
                  dm<float>(b_re, b_im, ldb, sb), (float)beta, dm<float>(c_re, c_im, ldc, sc),
                  batch);
    else
      gemm<double>(s, ta, tb, M, N, K, alpha, dm<double>(a_re, a_im, lda, sa),
                   dm<double>(b_re, b_im, ldb, sb), beta, dm<double>(c_re, c_im, ldc, sc),
                   batch);
  });
}

// rfd_test_gemm with the kernel variant forced (1: k_gemm 64 x 64, 2: k_gemm
// 128 x 128, 3: k_dgemm): the candidates an autotuner times.
extern "C" int rfd_test_gemm_variant(int variant, int dtype, int ta, int tb, int64_t M, int64_t N,
                                     int64_t K, double alpha, double beta, void* a_re,
                                     void* a_im, int64_t lda, int64_t sa, void* b_re, void* b_im,
                                     int64_t ldb, int64_t sb, void* c_re, void* c_im, int64_t ldc,
                                     int64_t sc, int batch, void* stream) {
  return capi_guard([&] {
    if (variant < 1 || variant > 3) throw Error(ST_EINVAL, "variant must be 1, 2 or 3");
    hipStream_t s = (hipStream_t)stream;
    check_gemm_args(M, N, K, batch, a_re, b_re, c_re, a_im, b_im, c_im);
    struct Reset {
      ~Reset() { gemm_force_variant(0); }
    } reset;
    gemm_force_variant(variant);
    if (dtype == 0)
      gemm<float>(s, ta, tb, M, N, K, (float)alpha, dm<float>(a_re, a_im, lda, sa),
                  dm<float>(b_re, b_im, ldb, sb), (float)beta, dm<float>(c_re, c_im, ldc, sc),
                  batch);
    else
      gemm<double>(s, ta, tb, M, N, K, alpha, dm<double>(a_re, a_im, lda, sa),
                   dm<double>(b_re, b_im, ldb, sb), beta, dm<double>(c_re, c_im, ldc, sc),
                   batch);
  });
}

// rfd_test_gemm for callers that cannot allocate: split-K partial tiles in
// the library's fixed per-device scratch array (gemm_static).
extern "C" int rfd_test_gemm_static(int dtype, int ta, int tb, int64_t M, int64_t N, int64_t K,
                                    double alpha, double beta, void* a_re, void* a_im,
                                    int64_t lda, int64_t sa, void* b_re, void* b_im, int64_t ldb,
                                    int64_t sb, void* c_re, void* c_im, int64_t ldc, int64_t sc,
                                    int batch, void* stream) {
  return capi_guard([&] {
    hipStream_t s = (hipStream_t)stream;
    check_gemm_args(M, N, K, batch, a_re, b_re, c_re, a_im, b_im, c_im);
    if (dtype == 0)
      gemm_static<float>(s, ta, tb, M, N, K, (float)alpha, dm<float>(a_re, a_im, lda, sa),
                         dm<float>(b_re, b_im, ldb, sb), (float)beta,
                         dm<float>(c_re, c_im, ldc, sc), batch);
    else
      gemm_static<double>(s, ta, tb, M, N, K, alpha, dm<double>(a_re, a_im, lda, sa),
                          dm<double>(b_re, b_im, ldb, sb), beta, dm<double>(c_re, c_im, ldc, sc),
                          batch);
  });
}

// C_b = alpha A_b B_b + beta C_b, real FP64, with every B_b upper triangular
// (gemm_triu_b).
extern "C" int rfd_test_gemm_triu_b(int64_t M, int64_t N, int64_t K, double alpha, double beta,
                                    void* a, int64_t lda, int64_t sa, void* b, int64_t ldb,
                                    int64_t sb, void* c, int64_t ldc, int64_t sc, int batch,
                                    void* stream) {
  return capi_guard([&] {
    check_gemm_args(M, N, K, batch, a, b, c, nullptr, nullptr, nullptr);
    gemm_triu_b((hipStream_t)stream, M, N, K, alpha, dm<double>(a, nullptr, lda, sa),
                dm<double>(b, nullptr, ldb, sb), beta, dm<double>(c, nullptr, ldc, sc), batch);
  });
}

// Factors A (n x n items, in place) and solves A X = R in place (n x r items).
// pivot = 1 selects partial pivoting (real only).  *flags_out receives the
// breakdown flags.
extern "C" int rfd_test_lu(int dtype, int pivot, int64_t n, int batch, void* a_re, void* a_im,
                           int64_t lda, int64_t sa, void* r_re, void* r_im, int64_t ldr,
                           int64_t sr, int64_t r, unsigned* flags_out, void* stream) {
  return capi_guard([&] {
    hipStream_t s = (hipStream_t)stream;
    const size_t es = dtype == 0 ? 4 : 8;
    const int64_t ibs = NB * 2 * n;
    const int planes = a_im ? 2 : 1;
    void* inv = nullptr;
    unsigned* flags = nullptr;
    int32_t* ipiv = nullptr;
    RFD_HIP(hipMalloc(&inv, es * ibs * batch * planes));
    RFD_HIP(hipMalloc(&flags, sizeof(unsigned)));
    RFD_HIP(hipMalloc(&ipiv, sizeof(int32_t) * n * batch));
    RFD_HIP(hipMemsetAsync(flags, 0, sizeof(unsigned), s));
    char* ib = (char*)inv;
    void* iim = planes == 2 ? (void*)(ib + es * ibs * batch) : nullptr;
    if (dtype == 0) {
      auto A = dm<float>(a_re, a_im, lda, sa);
      auto I = dm<float>(inv, iim, NB, ibs);
      if (pivot) lu_piv<float>(s, A, n, batch, I, ipiv, flags, 1e-30);
      else lu_nopiv<float>(s, A, n, batch, I, flags, 1e-30);
      if (r > 0) lu_solve<float>(s, A, I, pivot ? ipiv : nullptr, n, dm<float>(r_re, r_im, ldr, sr), r, batch);
    } else {
      auto A = dm<double>(a_re, a_im, lda, sa);
      auto I = dm<double>(inv, iim, NB, ibs);
      if (pivot) lu_piv<double>(s, A, n, batch, I, ipiv, flags, 1e-300);
      else lu_nopiv<double>(s, A, n, batch, I, flags, 1e-300);
      if (r > 0) lu_solve<double>(s, A, I, pivot ? ipiv : nullptr, n, dm<double>(r_re, r_im, ldr, sr), r, batch);
    }
    RFD_HIP(hipMemcpyAsync(flags_out, flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    RFD_HIP(hipStreamSynchronize(s));
    RFD_HIP(hipFree(inv));
    RFD_HIP(hipFree(flags));
    RFD_HIP(hipFree(ipiv));
  });
}

// Copies the current M-orthonormal basis of range(Z) (reordered numbering,
// n x k, ld n) to dst (device, room for n * cap doubles); returns k in *k_out.


// Eigenpairs lo .. lo + num - 1 (ascending, 0-based) of each symmetric
// n x n item of A (device, ld n, item stride n * n, destroyed): blocked
// tridiagonalization, bisection, inverse iteration with eigenvalues closer
// than 1e-10 ||A|| treated as one cluster, back-transformation.  lam: device,
// num per item; Y: device, n x num per item.
extern "C" int rfd_test_syevx(int64_t n, int batch, double* A, int lo, int num, double* lam,
                              double* Y, void* stream) {
  return capi_guard([&] {
    hipStream_t s = (hipStream_t)stream;
    if (n < 1 || batch < 1 || lo < 0 || num < 1 || lo + num > n)
      throw Error(ST_EINVAL, "bad eigenvalue range");
    DMat<double> Am{A, nullptr, n, n * n};
    TriWork tw;
    sy_tridiag(s, Am, n, batch, tw);
    std::vector<int> lov(batch, lo), nv(batch, num);
    DevBuf lo_d, num_d, cl_d, scr;
    lo_d.alloc(sizeof(int) * batch);
    num_d.alloc(sizeof(int) * batch);
    RFD_HIP(hipMemcpyAsync(lo_d.p, lov.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s));
    RFD_HIP(hipMemcpyAsync(num_d.p, nv.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s));
    bisect(s, tw, n, batch, lo_d.as<int>(), num_d.as<int>(), num, lam, num);
    std::vector<double> lh((size_t)batch * num), dh((size_t)n * batch), eh((size_t)n * batch);
    RFD_HIP(hipMemcpyAsync(lh.data(), lam, sizeof(double) * lh.size(), hipMemcpyDeviceToHost, s));
    RFD_HIP(hipMemcpyAsync(dh.data(), tw.d.p, sizeof(double) * dh.size(), hipMemcpyDeviceToHost, s));
    RFD_HIP(hipMemcpyAsync(eh.data(), tw.e.p, sizeof(double) * eh.size(), hipMemcpyDeviceToHost, s));
    RFD_HIP(hipStreamSynchronize(s));
    std::vector<int> cl((size_t)batch * num);
    for (int b = 0; b < batch; ++b) {
      double tn = 0;
      for (int64_t r = 0; r < n; ++r)
        tn = std::max(tn, std::fabs(dh[b * n + r]) + std::fabs(eh[b * n + r]) +
                              (r ? std::fabs(eh[b * n + r - 1]) : 0.0));
      for (int i = 0; i < num; ++i) {
        const double* l = lh.data() + (size_t)b * num;
        cl[(size_t)b * num + i] = (i > 0 && l[i] - l[i - 1] <= 1e-10 * tn) ? cl[(size_t)b * num + i - 1] : i;
      }
    }
    cl_d.alloc(sizeof(int) * cl.size());
    RFD_HIP(hipMemcpyAsync(cl_d.p, cl.data(), sizeof(int) * cl.size(), hipMemcpyHostToDevice, s));
    DMat<double> Ym{Y, nullptr, n, n * num};
    inverse_iteration(s, tw, n, batch, lam, num_d.as<int>(), cl_d.as<int>(), num, Ym, scr);
    back_transform(s, Am, tw, n, batch, Ym, num_d.as<int>(), num);
    RFD_HIP(hipStreamSynchronize(s));
  });
}

extern "C" int rfd_test_schur_renumber(int64_t n, const int64_t* A_ptr, const int32_t* A_idx,
                                       const double* A_val, const int64_t* M_ptr,
                                       const int32_t* M_idx, const double* M_val, int32_t p,
                                       const int32_t* part, int64_t* D_out, int64_t* TS_out,
                                       int64_t* SJ_out, int32_t* pos) {
  return capi_guard([&] {
    if (!D_out || !TS_out || !SJ_out || !pos) throw Error(ST_EINVAL, "null output");
    const Csr A = make_csr(n, A_ptr, A_idx, A_val, "A");
    const Csr M = make_csr(n, M_ptr, M_idx, M_val, "M");
    check_symmetric(A, "A");
    check_symmetric(M, "M");
    const Partition P = make_partition(A, M, p, part);
    const int64_t D = (P.d_max + NB - 1) / NB * NB;
    const SchurRenumber R = make_schur_renumber(P, D, NB);
    *D_out = D;
    *TS_out = R.TS;
    *SJ_out = R.SJ;
    for (int64_t i = 0; i < n; ++i) pos[i] = -1;
    for (int j = 0; j < P.p; ++j)
      for (size_t r = 0; r < P.interior[j].size(); ++r) pos[P.interior[j][r]] = R.pos[j][r];
  });
}
