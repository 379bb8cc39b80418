// Dense batched building blocks on the gfx950 matrix cores: GEMM, LU
// (no pivoting and partial pivoting), triangular solves through inverted
// diagonal blocks, and elementwise helpers.  All operate on strided batches
// (DMat) of uniform size; complex data is planar.
#pragma once

#include <mutex>

#include "rfd_common.hpp"

namespace rfd {

constexpr int NB = 64;  // LU / triangular-solve block size (= GEMM tile edge)

// Optional per-launch timing of the GEMM kernel instantiations.
struct KernelAccount {
  struct Rec {
    int key;
    double flops;
    hipEvent_t a, b;
  };
  bool enabled = false;
  std::mutex mu;
  std::vector<Rec> recs;
  static KernelAccount& get();
  void collect(double* launches, double* ms, double* flops, int nkeys);
  struct Scope {
    Scope(hipStream_t s, int key, double flops);
    ~Scope();
    hipStream_t s_;
    int rec_ = -1;
  };
};

// C_b = alpha * op(A_b) * op(B_b) + beta * C_b for b < batch.  op = transpose
// when ta/tb.  Complex when C is complex; a real A or B (im == nullptr) is
// taken with zero imaginary part.  beta == 0 never reads C.
template <typename T>
void gemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha,
          DMat<T> A, DMat<T> B, T beta, DMat<T> C, int batch);

// As gemm for square N x N results, computing only the output tiles that
// meet the lower triangle (i >= j); entries above the diagonal are left
// undefined (the caller mirrors the lower triangle of a symmetric result).
template <typename T>
void gemm_lower(hipStream_t s, bool ta, bool tb, int64_t N, int64_t K, T alpha, DMat<T> A,
                DMat<T> B, T beta, DMat<T> C, int batch);

// In-place LU without pivoting of n x n items (n multiple of NB).  inv
// receives, per item, the inverses of the unit-lower and upper diagonal
// blocks: an NB x (2 n) matrix [Linv_0 Uinv_0 Linv_1 Uinv_1 ...].  A pivot
// with |u_kk| <= tiny or a non-finite value sets bits in *flags.
// Semidefinite mode (drop != nullptr; real, batch 1): a pivot <= droptol marks
// its column dependent (drop[k] = 1) and removes it from the factor: L column
// and U row become unit vectors and the column adds nothing to later steps.
template <typename T>
void lu_nopiv(hipStream_t s, DMat<T> A, int64_t n, int batch, DMat<T> inv, unsigned* flags,
              double tiny, int* drop = nullptr, double droptol = 0.0);

// In-place LU with partial pivoting of real n x n items.  ipiv: per item n
// int32 (0-based row swapped with row i at step i), item stride n.
template <typename T>
void lu_piv(hipStream_t s, DMat<T> A, int64_t n, int batch, DMat<T> inv, int32_t* ipiv,
            unsigned* flags, double tiny);

// Solves (LU) X = R in place for n x r items R (n multiple of NB), using the
// factors and block inverses of lu_nopiv / lu_piv (ipiv may be null).
// parts: 1 = forward (L) only, 2 = backward (U) only, 3 = both.
template <typename T>
void lu_solve(hipStream_t s, DMat<T> LU, DMat<T> inv, const int32_t* ipiv, int64_t n,
              DMat<T> R, int64_t r, int batch, int parts = 3);

// Y (n x r, complex planar) <- fill with zero, or with the identity pattern
// on the padding rows/cols beyond `active` when ident_pad.
template <typename T>
void fill(hipStream_t s, DMat<T> X, int64_t rows, int64_t cols, int batch, T value);

template <typename T>
void pad_identity(hipStream_t s, DMat<T> X, int64_t active, int64_t n, int batch);

// Y = convert(X) elementwise (rows x cols per item), both planes.
template <typename TD, typename TS>
void convert(hipStream_t s, DMat<TS> X, DMat<TD> Y, int64_t rows, int64_t cols, int batch);

// Y += convert(X) elementwise.
template <typename TD, typename TS>
void add_to(hipStream_t s, DMat<TS> X, DMat<TD> Y, int64_t rows, int64_t cols, int batch);

// max |X| over every item into *out (non-negative double, bitwise atomicMax).
template <typename T>
void absmax(hipStream_t s, DMat<T> X, int64_t rows, int64_t cols, int batch, double* out);

}  // namespace rfd
