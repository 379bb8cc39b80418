// Two-level (nested-dissection) form of the interface Schur complement S(zeta).
//
// The interface is split by the caller into L groups and a top set T such
// that S(zeta) couples two different groups through nothing: no entry of C or
// M_C joins them, and no subdomain touches both (Sec. 3.1: S = C_zeta - sum_j
// Ehat_j^T B_j(zeta)^{-1} Ehat_j, so S_ab != 0 only when a and b are coupled
// in C or adjacent to one subdomain).  Ordering the groups first and T last,
//
//   S = [ S_GG  S_GT ]   S_GG = diag(S_11, .., S_LL),  S_TG = S_GT^T
//       [ S_TG  S_TT ]   (A - zeta M is complex symmetric, so S is too),
//
// and S is factored as the block LU of that arrow: each S_gg, then
// X_g = S_gg^{-1} S_gT and the top Schur complement
// S_TT' = S_TT - sum_g S_gT^T X_g, then S_TT'.  This is the paper's
// domain-decomposition reordering (Sec. 2.3, eq. (2.5)) applied once more, to
// S itself, in the spirit of the recursive RF-DDES the paper proposes
// (Sec. 7).  The result is S(zeta)^{-1} exactly (up to rounding): the groups
// are eliminated first, as a dense LU without pivoting would after the same
// symmetric permutation.
//
// Storage per pole (planar complex, column-major):
//   S_gg   L items of NGP x NGP    (group-local order, identity on padding)
//   S_gT   L items of NGP x TGP    (columns: T_g, the top nodes coupled to g)
//   S_TT   one TP x TP item        (top-local order, identity on padding)
// Items of all poles are consecutive: item (l, g) = l * L + g.
#pragma once

#include <vector>

#include "pencil.hpp"
#include "rfd_common.hpp"
#include "sparse.hpp"

namespace rfd {

struct TreeHost {
  int L = 0;
  int64_t s = 0, t = 0, NGP = 0, TGP = 0, TP = 0;
  std::vector<int32_t> ng, tgn;              // group sizes, |T_g|
  std::vector<int32_t> kind, grp, loc;       // per interface position: 0 group / 1 top,
                                             // group, group-local or top-local index
  std::vector<int32_t> gpos;                 // L x NGP: position of group-local row (-1 pad)
  std::vector<int32_t> tpos;                 // TP: position of top-local row (-1 pad)
  std::vector<int32_t> tgidx;                // L x TGP: top-local index of T_g row (-1 pad)
  std::vector<int32_t> tptr, tent;           // top row b -> entries g * TGP + lb (b = T_g[lb])
  // C entries by destination block (kind 0: S_gg, 1: S_gT, 2: S_TT; a top
  // row with a group column is the transpose of a stored S_gT entry and is
  // not listed): entries coff[k] .. coff[k] + ccnt[k] - 1 of ce (index of the
  // C entry), cg (group), cr, cc (row and column in the block)
  std::vector<int32_t> ce, cg, cr, cc;
  int64_t ccnt[3] = {0, 0, 0}, coff[3] = {0, 0, 0};
  std::vector<int32_t> jkind, jloc, jtl;     // p x SJ per adjacent node of subdomain j:
                                             // 0 group / 1 top, group-local or T_g position,
                                             // top-local index (top nodes)
  std::vector<int32_t> jgrp;                 // p: group of subdomain j (-1: touches T only)
  std::vector<std::vector<int32_t>> gcolors; // groups with pairwise disjoint T_g
};

// Validates the grouping (group[a] in {-1, 0..L-1} per interface position,
// every group non-empty, no C/M_C entry between two groups, no subdomain
// adjacent to two groups) and builds the maps.  Throws Error(ST_EINVAL).
TreeHost build_tree(const Partition& P, int64_t SJ, int L, const int32_t* group);

struct TreeDev {
  int L = 0;
  int64_t s = 0, t = 0, NGP = 0, TGP = 0, TP = 0;
  std::vector<int32_t> ng, tgn;
  std::vector<std::vector<int32_t>> gcolors;
  DevBuf kind, grp, loc, gpos, tpos, tgidx, tptr, tent, ce, cg, cr, cc, jkind, jloc, jtl, jgrp,
      ngd;
  std::vector<DevBuf> gcol_d;
  int64_t ccnt[3] = {0, 0, 0}, coff[3] = {0, 0, 0};
  void upload(const TreeHost& h);
};

// S blocks of the window's poles: C_zeta (as the dense path's schur_init),
// identity on the padding.  The blocks must be zero on entry.
void tree_init(hipStream_t s, DMat<double> Sgg, DMat<double> SgT, DMat<double> STT, int npoles,
               int pole0, DevPairCsr Cc, const TreeDev& tr, Shifts z);

// S -= Ehat_zeta^T X for the listed subdomains (pairwise disjoint adjacency
// sets); X items ll * p + j, S items of local pole ll, zeta index pole0 + ll.
void tree_scatter(hipStream_t s, DMat<double> Sgg, DMat<double> SgT, DMat<double> STT,
                  DMat<double> X, int64_t SJ, int p, int npoles, int pole0, const int32_t* members,
                  int nmembers, const int32_t* sj, DevPairCsr Et, const TreeDev& tr, Shifts z);

// S_TT -= sum_g scatter(Gt_g) onto the rows and columns T_g (groups of one
// colour per launch, colours in order).
template <typename T>
void tree_tt_update(hipStream_t s, DMat<T> STT, DMat<T> Gt, int npoles, const TreeDev& tr);

// Y (real s x m) into the blocked right-hand sides YG (items l * L + g,
// NGP x MP) and YT (items l, TP x MP), zero imaginary part and padding.
void tree_broadcast(hipStream_t s, const double* Y, int64_t ldy, int64_t m, DMat<double> YG,
                    DMat<double> YT, int64_t MP, int npoles, const TreeDev& tr);

// W (+)= sum_l 2 Re(omega_l X_l), X_l read from the blocked XG / XT.
void tree_accumulate(hipStream_t s, DMat<double> XG, DMat<double> XT, const double* omega,
                     int npoles, double* W, int64_t ldw, int64_t m, bool add, const TreeDev& tr);

// XTg (items l * L + g, TGP x cols) = rows T_g of XT (items l).
template <typename T>
void tree_gather_top(hipStream_t s, DMat<T> XT, DMat<T> XTg, int64_t cols, int npoles,
                     const TreeDev& tr);

// RT (items l) -= sum over g of U_(l, g) scattered onto the rows T_g, each top
// row summing its groups in a fixed order.
template <typename T>
void tree_top_subtract(hipStream_t s, DMat<T> RT, DMat<T> U, int64_t cols, int npoles,
                       const TreeDev& tr);

}  // namespace rfd
