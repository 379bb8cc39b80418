/* Kernel-level test entry points of the RF-DDES gfx950 library.
 *
 * These expose single building blocks of the filter path so that a test
 * can check each one element by element against a host computation.  They
 * are not part of the solver interface (rfd.h) and allocate and free device
 * workspace on every call.  All pointers named a_*, b_*, c_*, r_*, A, lam, Y,
 * dst are device pointers; matrices are column-major strided batches (leading
 * dimension ld*, item stride s*), complex data planar (re, im; im may be NULL
 * for real data).  Every function returns 0 (RFD_OK) or an rfd_status code,
 * with the message in rfd_last_error(); stream may be NULL (default stream). */
#ifndef RFD_TESTING_H
#define RFD_TESTING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C_b = alpha op(A_b) op(B_b) + beta C_b for b < batch (op = transpose when
 * ta / tb).  dtype 0 = FP32, 1 = FP64.  Complex when c_im != NULL.  This is
 * the matrix-core GEMM every dense step of the filter and of the basis
 * construction runs on (Schur products, eq. (3.3)-(3.5)). */
int rfd_test_gemm(int dtype, int ta, int tb, int64_t M, int64_t N, int64_t K, double alpha,
                  double beta, void* a_re, void* a_im, int64_t lda, int64_t sa, void* b_re,
                  void* b_im, int64_t ldb, int64_t sb, void* c_re, void* c_im, int64_t ldc,
                  int64_t sc, int batch, void* stream);

/* rfd_test_gemm with the kernel variant forced (1: the 64 x 64 tile, 2: the
 * 128 x 128 tile, real FP32 only, 3: the large-tile FP64 kernel, FP64 only):
 * the candidates the autotuner behind rfd_set_gemm_tuning times for each
 * product class.  RFD_EINVAL when the variant cannot run the product. */
int rfd_test_gemm_variant(int variant, int dtype, int ta, int tb, int64_t M, int64_t N, int64_t K,
                          double alpha, double beta, void* a_re, void* a_im, int64_t lda,
                          int64_t sa, void* b_re, void* b_im, int64_t ldb, int64_t sb,
                          void* c_re, void* c_im, int64_t ldc, int64_t sc, int batch,
                          void* stream);

/* rfd_test_gemm for real FP64 operands, neither transposed, with every B_b
 * upper triangular (B_b[k, j] = 0 for k > j; the entries below the diagonal
 * are not read by the large-tile path, so they must be zero): the product
 * Q = B U^{-1} D^{1/2} of the Cholesky QR that builds the M-orthonormal basis
 * of range(Z) (Alg. 5.1 step 7), whose large instances skip the zero part of
 * K. */
int rfd_test_gemm_triu_b(int64_t M, int64_t N, int64_t K, double alpha, double beta, void* a,
                         int64_t lda, int64_t sa, void* b, int64_t ldb, int64_t sb, void* c,
                         int64_t ldc, int64_t sc, int batch, void* stream);

/* Largest |U_j^T U_j - I| over the subdomain eigenvector blocks of the last
 * spectral decomposition (U_j = M_Bj^{1/2} V_j, after its orthonormalising
 * steps), or 0 when the pencil has none: the departure from M_Bj-orthonormal
 * eigenvectors on which the expansion of rfd_set_interior_solver rests. */
int rfd_test_spectral_orthogonality(void* pencil, double* dev);

/* rfd_test_gemm for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same product, allocating nothing.  The split-K partial tiles of
 * products with few output tiles go to a fixed 64 MiB device array that the
 * library holds on each device until the process ends (the per-call split
 * count is lowered until they fit).  Products whose output (M * N * batch
 * elements, times 2 when complex, of 4 or 8 bytes) takes more than 32 MiB are
 * rejected with RFD_EINVAL.  Every call on a device shares that array: calls
 * that overlap on one device (other streams or threads) race, so serialise
 * them.  Nothing in the array needs clearing between calls. */
int rfd_test_gemm_static(int dtype, int ta, int tb, int64_t M, int64_t N, int64_t K,
                         double alpha, double beta, void* a_re, void* a_im, int64_t lda,
                         int64_t sa, void* b_re, void* b_im, int64_t ldb, int64_t sb,
                         void* c_re, void* c_im, int64_t ldc, int64_t sc, int batch,
                         void* stream);

/* Factors each n x n item of A in place (pivot = 0: LU without pivoting, as
 * for the shifted blocks B_j - zeta M_Bj and S(zeta) of Section 3; pivot = 1:
 * partial pivoting, real only, as for B_j - sigma M_Bj of Section 4) and
 * solves A X = R in place for the n x r items of R (r may be 0).  n must be a
 * multiple of 64.  *flags_out receives the breakdown bits (1: tiny pivot,
 * 2: non-finite value). */
int rfd_test_lu(int dtype, int pivot, int64_t n, int batch, void* a_re, void* a_im, int64_t lda,
                int64_t sa, void* r_re, void* r_im, int64_t ldr, int64_t sr, int64_t r,
                unsigned* flags_out, void* stream);

/* Eigenpairs with ascending indices lo .. lo + num - 1 (0-based) of each
 * symmetric n x n item of A (FP64, ld n, item stride n * n; destroyed), the
 * dense eigensolver of the Rayleigh-Ritz step (Section 5) and of the
 * subdomain eigenvectors of Section 4.3: lam receives num values per item,
 * Y the n x num eigenvectors per item (ld n, item stride n * num). */
int rfd_test_syevx(int64_t n, int batch, double* A, int lo, int num, double* lam, double* Y,
                   void* stream);

/* Copies the M-orthonormal basis of the projection subspace (eq. (5.5)) built
 * by the last rfd_solve_interior call, in the library's internal interior-
 * first numbering (n x k, ld n), to dst (room for n * cap doubles);
 * *k_out = k. */
int rfd_test_basis(void* pencil, double* dst, int64_t cap, int64_t* k_out, void* stream);

/* The renumbering behind the Schur solves on trailing blocks (Sec. 3.1:
 * S(zeta) = C_zeta - sum_j Ehat_j^T (B_j - zeta M_Bj)^{-1} Ehat_j reads the
 * solution only on the rows Ehat_j touches), computed on the host for the
 * pencil and partition given as to rfd_create_pencil and rfd_set_partition
 * (same validation and errors).  Blocks are padded to D = the largest
 * interior rounded up to 64 rows; in subdomain j's block the padding comes
 * first, then the rows Ehat_j does not touch, then those it touches.
 * Outputs: *D_out; *TS_out, the trailing rows (a multiple of 64, at most D)
 * that hold every touched row; *SJ_out, the largest number of interface
 * nodes coupled to one subdomain; pos[i] (room for n) = the row of interior
 * node i in its subdomain's renumbered block, -1 for interface nodes.  No
 * device work. */
int rfd_test_schur_renumber(int64_t n, const int64_t* A_ptr, const int32_t* A_idx,
                            const double* A_val, const int64_t* M_ptr, const int32_t* M_idx,
                            const double* M_val, int32_t p, const int32_t* part, int64_t* D_out,
                            int64_t* TS_out, int64_t* SJ_out, int32_t* pos);

#ifdef __cplusplus
}
#endif

#endif /* RFD_TESTING_H */
