// Host-side model of a pencil: validated CSR copies, the interior-first
// reordering maps (Sec. 2.3, eq. (2.5)), local sparse blocks of every
// subdomain, the rational filter poles (Sec. 2.1) and the precision mode.
#pragma once

#include <complex>
#include <memory>
#include <vector>

#include "rfd_common.hpp"

namespace rfd {

struct Csr {
  int64_t n = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  std::vector<double> val;
};

// Entries of one sparse block with both the A and the M value at every
// position of the union pattern (rows are local, cols local).
struct PairCsr {
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> ptr;   // rows + 1
  std::vector<int32_t> idx;   // local column
  std::vector<double> a, m;   // A and M values
};

struct Partition {
  int p = 0;
  std::vector<int32_t> part;                    // n
  std::vector<std::vector<int32_t>> interior;   // global ids, ascending
  std::vector<int32_t> iface;                   // global ids, ascending
  std::vector<std::vector<int32_t>> adj;        // interface positions adjacent to j
  std::vector<PairCsr> Bloc;                    // d_j x d_j   (B_j, M_B^(j))
  std::vector<PairCsr> Eloc;                    // d_j x s_j   (Ehat_j, Mhat_E^(j))
  std::vector<PairCsr> EtLoc;                   // s_j x d_j   transposes of Eloc
  PairCsr Cloc;                                 // s x s       (C, M_C)
  std::vector<std::vector<int>> colors;         // subdomains whose adj sets are disjoint
  bool m_e_zero = true;
  bool m_diag = true;                           // M diagonal
  int64_t d_max = 0, sj_max = 0;
};

struct Poles {
  double alpha = 0, beta = 0;
  int n_c = 0;
  std::vector<std::complex<double>> zeta, omega;   // upper half plane
  bool set = false;
};

std::vector<std::complex<double>> gauss_legendre(int n, std::vector<double>* w);
void make_poles(Poles& P, double alpha, double beta, int n_c, int rule, const double* zeta,
                const double* omega);

// Validates and copies a CSR; sums duplicates, sorts columns.
Csr make_csr(int64_t n, const int64_t* ptr, const int32_t* idx, const double* val,
             const char* name);
void check_symmetric(const Csr& A, const char* name);
Partition make_partition(const Csr& A, const Csr& M, int p, const int32_t* part);

// The subdomain blocks renumbered for Schur solves on trailing blocks: in
// each D-row item the padding rows come first (a unit diagonal entry each),
// then the rows of B_j that Ehat_j does not touch, then the rows it touches
// (both in ascending order).  pos[j][r] = new row of local row r; TS = the
// trailing rows (a multiple of nb, at most D) that hold every touched row of
// every subdomain; SJ = the largest number of columns of an Ehat_j.
struct SchurRenumber {
  std::vector<PairCsr> B, E, Et;  // D x D, D x s_j, s_j x D
  std::vector<std::vector<int32_t>> pos;
  int64_t TS = 0, SJ = 0;
};
SchurRenumber make_schur_renumber(const Partition& P, int64_t D, int64_t nb);
double abs_row_sum_max(const Csr& A);

}  // namespace rfd
