// Dense batched building blocks on the gfx950 matrix cores: GEMM, LU
// (no pivoting and partial pivoting), triangular solves through inverted
// diagonal blocks, and elementwise helpers.  All operate on strided batches
// (DMat) of uniform size; complex data is planar.
#pragma once

#include <mutex>

#include "rfd_common.hpp"

namespace rfd {

constexpr int NB = 64;  // LU / triangular-solve block size (= GEMM tile edge)

// Optional per-launch timing of selected kernels, sampled: every `every`-th
// launch of a key gets a pair of HIP events on its launch stream, stamped by
// the launch itself (hipExtLaunchKernelGGL) where the kernel is launched
// here, around the call otherwise, together with the launch's algorithmic
// flops and bytes.  Keys 0..15: the GEMM instantiations (8 fp64 + 4 complex
// + 2 transA + transB) of the hand-written kernel; KA_TRI_SYMV: the
// symmetric mat-vec of the tridiagonalization; KA_DGEMM + (4 complex + 2
// transA + transB): the large-tile FP64 kernel.
constexpr int KA_KEYS = 32;
constexpr int KA_TRI_SYMV = 16;
constexpr int KA_DGEMM = 17;
constexpr double KA_ALWAYS_FLOPS = 1e11;  // launches this large are always sampled
struct KernelAccount {
  struct Rec {
    int key;
    bool always;  // timed for its size (not picked by the hash)
    double flops, bytes;
    hipEvent_t a, b;
  };
  int every = 0;  // 0: off
  std::mutex mu;
  std::vector<Rec> recs;
  int64_t count[KA_KEYS] = {};        // launches
  int64_t count_small[KA_KEYS] = {};  // launches below KA_ALWAYS_FLOPS
  static KernelAccount& get();
  // Per key: launches, launches timed, and the estimated milliseconds, flops
  // and bytes of all launches (the always-timed ones summed, the hashed
  // sample of the others scaled by their launch count over the sample).
  void collect(double* launches, double* sampled, double* ms, double* flops, double* bytes,
               int nkeys);
  // Decides whether this launch is sampled and holds its events.
  struct Scope {
    Scope(hipStream_t s, int key, double flops, double bytes = 0.0);
    hipEvent_t start() const { return a_; }
    hipEvent_t stop() const { return b_; }
    void mark_start();  // for launches that cannot stamp the events themselves
    void mark_stop();
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
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
// As gemm (real FP64, neither operand transposed) for an upper triangular B
// (B[k, j] = 0 for k > j): the large products skip the zero part of K.
void gemm_triu_b(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, DMat<double> A,
                 DMat<double> B, double beta, DMat<double> C, int batch);

// Autotuned tile choices (rfd_set_gemm_tuning): count entries of 9 int32 each,
// {fp64, complex, transA, transB, floor log2 M, N, K, batch, variant}; count
// = 0 clears.  Process-wide.  gemm_tuning_size: entries held.
void set_gemm_tuning(const int32_t* entries, int count);
int gemm_tuning_size();
// Forces a variant (0 = none) for the calling thread's next products.
void gemm_force_variant(int v);

// Drops the split-K workspace kept for stream s (call
// before destroying a stream that ran products).
void release_stream_resources(hipStream_t s);

template <typename T>
void gemm_lower(hipStream_t s, bool ta, bool tb, int64_t N, int64_t K, T alpha, DMat<T> A,
                DMat<T> B, T beta, DMat<T> C, int batch);

// As gemm, allocating nothing: split-K partial tiles go to a fixed device
// array of GEMM_STATIC_SCRATCH_BYTES per device (shared by every call on the
// device; overlapping calls race).  Products whose output (M N batch planes
// elements) takes more than half of it are rejected (ST_EINVAL).
constexpr size_t GEMM_STATIC_SCRATCH_BYTES = size_t(64) << 20;
template <typename T>
void gemm_static(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha,
                 DMat<T> A, DMat<T> B, T beta, DMat<T> C, int batch);

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
              DMat<T> R, int64_t r, int batch, int parts = 3, DMat<T> inv2 = DMat<T>{},
              int LW = 0, DMat<T> work = DMat<T>{});

// Wide leaves for lu_solve: inverses of the LW x LW diagonal blocks of the
// factors of lu_nopiv (LW = NB times a power of two, dividing n), merged from
// the NB-block inverses in inv: inv2 is LW x 2n per item, [Linv_0 Uinv_0
// Linv_1 ...] as inv.  work: (LW / 2)^2 max(n / LW, batch) elements per
// plane.  lu_solve with inv2, LW and a work of LW x r per item then stops its
// recursion at LW (fewer, larger products).  Works for the factors of lu_piv
// as well: the rows a later panel interchanges lie below every leaf it
// touches.
template <typename T>
void merge_inverses(hipStream_t s, DMat<T> LU, DMat<T> inv, int64_t n, int batch, DMat<T> inv2,
                    int LW, DMat<T> work);

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
