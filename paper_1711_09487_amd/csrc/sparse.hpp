// Sparse-structured kernels of the interface filter: expansion of the shifted
// interior blocks and their right-hand sides from the local CSR images, the
// FP64 residual of the shifted interior solves, Schur-complement assembly
// (owner-computes scatter by subdomain colour), and the filter accumulation.
#pragma once

#include "rfd_common.hpp"

namespace rfd {

// Concatenated local CSR blocks of all subdomains ("pair" values a = A, m = M).
// Row r of subdomain j spans entries [ptr[roff[j] + r], ptr[roff[j] + r + 1]).
struct DevPairCsr {
  const int64_t* roff = nullptr;  // p + 1 (row-pointer offset of each subdomain)
  const int64_t* ptr = nullptr;
  const int32_t* idx = nullptr;
  const double* a = nullptr;
  const double* m = nullptr;
};

struct Shifts {
  const double* z = nullptr;  // n_c x 2 (re, im) per pole, device
};

// K_(l,j) = B_j - zeta_l M_Bj (or - sigma M_Bj when sig_real) into a D x D
// item b = l p + j (l = pole offset + local); identity on the padding rows.
// K must be zero on entry.
template <typename T>
void expand_shifted(hipStream_t s, DMat<T> K, int64_t D, int p, int npoles, int pole0,
                    const int32_t* dj, DevPairCsr B, Shifts z, bool sig_real, double sigma);

// R_(l,j) = Ehat_j - zeta_l Mhat_E^(j)  (D x SJ, zero on entry).
template <typename T>
void expand_rhs(hipStream_t s, DMat<T> R, int p, int npoles, int pole0, const int32_t* dj,
                DevPairCsr E, Shifts z);

// R = (Ehat - zeta Mhat_E) - (B - zeta M_B) X over the active d_j x s_j part
// of every item (zeros elsewhere); max |R| into *rmax (bitwise atomic max).
void residual_shifted(hipStream_t s, DMat<double> X, DMat<double> R, int64_t D, int64_t SJ, int p,
                      int npoles, int pole0, const int32_t* dj, const int32_t* sj, DevPairCsr B,
                      DevPairCsr E, Shifts z, double* rmax);

// S_l = C - zeta_l M_C (SP x SP, zero on entry), identity on padding rows.
void schur_init(hipStream_t s, DMat<double> S, int64_t s_act, int64_t SP, int npoles, int pole0,
                DevPairCsr Cc, Shifts z);

// S_l[adj_j(a), adj_j(b)] -= sum_r (Ehat - zeta Mhat_E)[r, a] X_(l,j)[r, b] for the
// subdomains listed in `members` (pairwise disjoint adjacency sets).
void schur_scatter(hipStream_t s, DMat<double> S, DMat<double> X, int64_t SJ, int p, int npoles,
                   int pole0, const int32_t* members, int nmembers, const int32_t* sj,
                   const int32_t* adj, DevPairCsr Et, Shifts z);

// Yc_l = Y (real, s x m, ld ldy) as complex (zero imaginary part), padded
// with zeros to SP x MP, for every pole l.
void broadcast_rhs(hipStream_t s, const double* Y, int64_t ldy, int64_t s_act, int64_t m,
                   DMat<double> Yc, int64_t SP, int64_t MP, int npoles);

// W (+)= sum_l 2 Re(omega_l X_l) over s_act x m (W real, ld ldw), poles summed in order.
void filter_accumulate(hipStream_t s, DMat<double> X, const double* omega, int npoles,
                       double* W, int64_t ldw, int64_t s_act, int64_t m, bool add);

}  // namespace rfd
