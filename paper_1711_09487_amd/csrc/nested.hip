// Two-level interface Schur complement: maps (host) and the sparse-structured
// kernels that assemble S(zeta) into its group / top blocks and move
// right-hand sides between the interface order and the blocked order.  The
// dense work (LU of the blocks, the top Schur complement, solves) runs on the
// batched GEMM / LU kernels; see engine.hip.
#include <algorithm>

#include "nested.hpp"

namespace rfd {

template <typename V>
static void up(DevBuf& b, const std::vector<V>& v) {
  b.alloc(sizeof(V) * std::max<size_t>(v.size(), 1));
  if (!v.empty()) RFD_HIP(hipMemcpy(b.p, v.data(), sizeof(V) * v.size(), hipMemcpyHostToDevice));
}

void TreeDev::upload(const TreeHost& h) {
  L = h.L;
  s = h.s;
  t = h.t;
  NGP = h.NGP;
  TGP = h.TGP;
  TP = h.TP;
  ng = h.ng;
  tgn = h.tgn;
  gcolors = h.gcolors;
  for (int k = 0; k < 3; ++k) {
    ccnt[k] = h.ccnt[k];
    coff[k] = h.coff[k];
  }
  up(kind, h.kind);
  up(grp, h.grp);
  up(loc, h.loc);
  up(gpos, h.gpos);
  up(tpos, h.tpos);
  up(tgidx, h.tgidx);
  up(tptr, h.tptr);
  up(tent, h.tent);
  up(ce, h.ce);
  up(cg, h.cg);
  up(cr, h.cr);
  up(cc, h.cc);
  up(jkind, h.jkind);
  up(jloc, h.jloc);
  up(jtl, h.jtl);
  up(jgrp, h.jgrp);
  up(ngd, h.ng);
  gcol_d.clear();
  gcol_d.resize(gcolors.size());
  for (size_t c = 0; c < gcolors.size(); ++c) up(gcol_d[c], gcolors[c]);
}

// ---------------------------------------------------------------------------
// C_zeta into one kind of block: a thread per listed C entry and pole.  The
// entries of each kind are launched separately so that every thread writes
// through one block handle (item ll * per + g, element (row, col)).
__global__ void k_tree_cput(DMat<double> Dst, int per, int pole0, int64_t cnt, const int32_t* ent,
                            const int32_t* eg, const int32_t* er, const int32_t* ec,
                            const double* ca, const double* cm, Shifts z) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cnt) return;
  const int ll = blockIdx.y, l = pole0 + ll;
  const int64_t e = ent[q];
  const double zr = z.z[2 * l], zi = z.z[2 * l + 1];
  const DMat<double> d = Dst.item((int64_t)ll * per + eg[q]);
  const int64_t off = er[q] + (int64_t)ec[q] * d.ld;
  d.re[off] = ca[e] - zr * cm[e];
  d.im[off] = -zi * cm[e];
}

// identity on the padding rows of each group block (sizes per group)
__global__ void k_tree_pad_groups(DMat<double> Sgg, int L, const int32_t* ng, int64_t NGP) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y, g = b % L;
  if (i >= NGP || i < ng[g]) return;
  DMat<double> x = Sgg.item(b);
  x.re[i + i * x.ld] = 1.0;
  x.im[i + i * x.ld] = 0.0;
}

__global__ void k_tree_pad_top(DMat<double> STT, int64_t t, int64_t TP) {
  const int64_t i = t + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= TP) return;
  DMat<double> x = STT.item(blockIdx.y);
  x.re[i + i * x.ld] = 1.0;
  x.im[i + i * x.ld] = 0.0;
}

void tree_init(hipStream_t s, DMat<double> Sgg, DMat<double> SgT, DMat<double> STT, int npoles,
               int pole0, DevPairCsr Cc, const TreeDev& tr, Shifts z) {
  const DMat<double> dst[3] = {Sgg, SgT, STT};
  for (int k = 0; k < 3; ++k) {
    const int64_t cnt = tr.ccnt[k];
    if (cnt == 0) continue;
    const int64_t o = tr.coff[k];
    k_tree_cput<<<dim3(grid1(cnt), npoles), 256, 0, s>>>(
        dst[k], k == 2 ? 1 : tr.L, pole0, cnt, tr.ce.as<int32_t>() + o, tr.cg.as<int32_t>() + o,
        tr.cr.as<int32_t>() + o, tr.cc.as<int32_t>() + o, Cc.a, Cc.m, z);
    RFD_CHECK_LAUNCH();
  }
  k_tree_pad_groups<<<dim3(grid1(tr.NGP), npoles * tr.L), 256, 0, s>>>(Sgg, tr.L,
                                                                       tr.ngd.as<int32_t>(), tr.NGP);
  RFD_CHECK_LAUNCH();
  if (tr.TP > tr.t) {
    k_tree_pad_top<<<dim3(grid1(tr.TP - tr.t), npoles), 256, 0, s>>>(STT, tr.t, tr.TP);
    RFD_CHECK_LAUNCH();
  }
}

// ---------------------------------------------------------------------------
// Thread per (a, b) of subdomain j's adjacency and local pole: G_ab =
// sum_r (Ehat - zeta Mhat_E)[r, a] X[r, b] goes to the block that holds the
// pair (a top row with a group column is the transpose of a stored entry and
// is skipped).  Subdomains in one launch have disjoint adjacency sets, so
// every destination has one writer.
__global__ void k_tree_scatter(DMat<double> Sgg, DMat<double> SgT, DMat<double> STT,
                               DMat<double> X, int64_t SJ, int p, int L, int pole0,
                               const int32_t* members, int nmembers, const int32_t* sj,
                               DevPairCsr Et, const int32_t* jkind, const int32_t* jloc,
                               const int32_t* jtl, const int32_t* jgrp, Shifts z) {
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int it = blockIdx.y % nmembers, ll = blockIdx.y / nmembers;
  const int j = members[it], l = pole0 + ll;
  const int n_j = sj[j];
  if (e0 >= (int64_t)n_j * n_j) return;
  const int a = (int)(e0 % n_j), bcol = (int)(e0 / n_j);
  const int64_t oa = (int64_t)j * SJ + a, ob = (int64_t)j * SJ + bcol;
  const int ka = jkind[oa], kb = jkind[ob];
  if (ka == 1 && kb == 0) return;
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
  if (ka == 1) {  // both top
    const DMat<double> d = STT.item(ll);
    const int64_t off = jtl[oa] + (int64_t)jtl[ob] * d.ld;
    d.re[off] -= gr;
    d.im[off] -= gi;
  } else if (kb == 0) {
    const DMat<double> d = Sgg.item((int64_t)ll * L + jgrp[j]);
    const int64_t off = jloc[oa] + (int64_t)jloc[ob] * d.ld;
    d.re[off] -= gr;
    d.im[off] -= gi;
  } else {
    const DMat<double> d = SgT.item((int64_t)ll * L + jgrp[j]);
    const int64_t off = jloc[oa] + (int64_t)jloc[ob] * d.ld;
    d.re[off] -= gr;
    d.im[off] -= gi;
  }
}

void tree_scatter(hipStream_t s, DMat<double> Sgg, DMat<double> SgT, DMat<double> STT,
                  DMat<double> X, int64_t SJ, int p, int npoles, int pole0, const int32_t* members,
                  int nmembers, const int32_t* sj, DevPairCsr Et, const TreeDev& tr, Shifts z) {
  if (nmembers <= 0) return;
  dim3 g(grid1(SJ * SJ), nmembers * npoles);
  k_tree_scatter<<<g, 256, 0, s>>>(Sgg, SgT, STT, X, SJ, p, tr.L, pole0, members, nmembers, sj,
                                   Et, tr.jkind.as<int32_t>(), tr.jloc.as<int32_t>(),
                                   tr.jtl.as<int32_t>(), tr.jgrp.as<int32_t>(), z);
  RFD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Thread per (i, j) of T_g x T_g, group listed in `members`, local pole.
template <typename T>
__global__ void k_tree_tt(DMat<T> STT, DMat<T> Gt, int L, const int32_t* members, int nmembers,
                          const int32_t* tgidx, int64_t TGP, int64_t w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= w * w) return;
  const int it = blockIdx.y % nmembers, ll = blockIdx.y / nmembers;
  const int g = members[it];
  const int64_t i = e % w, j = e / w;
  const int32_t bi = tgidx[(int64_t)g * TGP + i], bj = tgidx[(int64_t)g * TGP + j];
  if (bi < 0 || bj < 0) return;
  const DMat<T> x = Gt.item((int64_t)ll * L + g), d = STT.item(ll);
  const int64_t o = bi + (int64_t)bj * d.ld, q = i + j * x.ld;
  d.re[o] -= x.re[q];
  d.im[o] -= x.im[q];
}

template <typename T>
void tree_tt_update(hipStream_t s, DMat<T> STT, DMat<T> Gt, int npoles, const TreeDev& tr) {
  for (size_t c = 0; c < tr.gcolors.size(); ++c) {
    int64_t w = 0;
    for (int g : tr.gcolors[c]) w = std::max<int64_t>(w, tr.tgn[g]);
    const int nm = (int)tr.gcolors[c].size();
    if (w == 0 || nm == 0) continue;
    dim3 g(grid1(w * w), nm * npoles);
    k_tree_tt<T><<<g, 256, 0, s>>>(STT, Gt, tr.L, tr.gcol_d[c].as<int32_t>(), nm,
                                   tr.tgidx.as<int32_t>(), tr.TGP, w);
    RFD_CHECK_LAUNCH();
  }
}

// ---------------------------------------------------------------------------
// Rows of a real s x m block into a blocked complex layout: item b uses the
// row map segment (b % nseg) of length rows.
__global__ void k_tree_rows(const double* Y, int64_t ldy, int64_t m, DMat<double> D,
                            int64_t rows, int64_t cols, const int32_t* map, int nseg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e % rows, c = e / rows;
  const int b = blockIdx.y;
  const int32_t a = map[(int64_t)(b % nseg) * rows + i];
  DMat<double> d = D.item(b);
  d.re[i + c * d.ld] = (a >= 0 && c < m) ? Y[a + c * ldy] : 0.0;
  d.im[i + c * d.ld] = 0.0;
}

void tree_broadcast(hipStream_t s, const double* Y, int64_t ldy, int64_t m, DMat<double> YG,
                    DMat<double> YT, int64_t MP, int npoles, const TreeDev& tr) {
  k_tree_rows<<<dim3(grid1(tr.NGP * MP), npoles * tr.L), 256, 0, s>>>(
      Y, ldy, m, YG, tr.NGP, MP, tr.gpos.as<int32_t>(), tr.L);
  RFD_CHECK_LAUNCH();
  k_tree_rows<<<dim3(grid1(tr.TP * MP), npoles), 256, 0, s>>>(Y, ldy, m, YT, tr.TP, MP,
                                                            tr.tpos.as<int32_t>(), 1);
  RFD_CHECK_LAUNCH();
}

__global__ void k_tree_accumulate(DMat<double> XG, DMat<double> XT, const double* omega,
                                  int npoles, double* W, int64_t ldw, int64_t s_act, int64_t m,
                                  int add, int L, const int32_t* kind, const int32_t* grp,
                                  const int32_t* loc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s_act * m) return;
  const int64_t a = e % s_act, c = e / s_act;
  const bool top = kind[a] != 0;
  const int g = grp[a];
  const int64_t r = loc[a];
  double acc = add ? W[a + c * ldw] : 0.0;
  // (each lane reads through one block handle: a top row or a group row)
  if (top) {
    for (int l = 0; l < npoles; ++l) {
      const DMat<double> x = XT.item(l);
      const int64_t q = r + c * x.ld;
      acc += 2.0 * (omega[2 * l] * x.re[q] - omega[2 * l + 1] * x.im[q]);
    }
  } else {
    for (int l = 0; l < npoles; ++l) {
      const DMat<double> x = XG.item((int64_t)l * L + g);
      const int64_t q = r + c * x.ld;
      acc += 2.0 * (omega[2 * l] * x.re[q] - omega[2 * l + 1] * x.im[q]);
    }
  }
  W[a + c * ldw] = acc;
}

void tree_accumulate(hipStream_t s, DMat<double> XG, DMat<double> XT, const double* omega,
                     int npoles, double* W, int64_t ldw, int64_t m, bool add, const TreeDev& tr) {
  k_tree_accumulate<<<grid1(tr.s * m), 256, 0, s>>>(XG, XT, omega, npoles, W, ldw, tr.s, m,
                                                    add ? 1 : 0, tr.L, tr.kind.as<int32_t>(),
                                                    tr.grp.as<int32_t>(), tr.loc.as<int32_t>());
  RFD_CHECK_LAUNCH();
}

template <typename T>
__global__ void k_tree_gather_top(DMat<T> XT, DMat<T> XTg, int64_t cols, int L,
                                  const int32_t* tgidx, int64_t TGP) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= TGP * cols) return;
  const int64_t i = e % TGP, c = e / TGP;
  const int b = blockIdx.y, g = b % L, l = b / L;
  const int32_t r = tgidx[(int64_t)g * TGP + i];
  const DMat<T> x = XT.item(l), d = XTg.item(b);
  d.re[i + c * d.ld] = r >= 0 ? x.re[r + c * x.ld] : T(0);
  d.im[i + c * d.ld] = r >= 0 ? x.im[r + c * x.ld] : T(0);
}

template <typename T>
void tree_gather_top(hipStream_t s, DMat<T> XT, DMat<T> XTg, int64_t cols, int npoles,
                     const TreeDev& tr) {
  k_tree_gather_top<T><<<dim3(grid1(tr.TGP * cols), npoles * tr.L), 256, 0, s>>>(
      XT, XTg, cols, tr.L, tr.tgidx.as<int32_t>(), tr.TGP);
  RFD_CHECK_LAUNCH();
}

template <typename T>
__global__ void k_tree_top_subtract(DMat<T> RT, DMat<T> U, int64_t rows, int64_t cols, int L,
                                    const int32_t* tptr, const int32_t* tent, int64_t TGP) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t b = e % rows, c = e / rows;
  const int l = blockIdx.y;
  const int32_t e0 = tptr[b], e1 = tptr[b + 1];
  if (e0 == e1) return;
  T sr = 0, si = 0;
  for (int32_t q = e0; q < e1; ++q) {
    const int32_t v = tent[q];
    const int g = v / (int32_t)TGP;
    const int64_t lb = v - (int64_t)g * TGP;
    const DMat<T> u = U.item((int64_t)l * L + g);
    sr += u.re[lb + c * u.ld];
    si += u.im[lb + c * u.ld];
  }
  const DMat<T> r = RT.item(l);
  r.re[b + c * r.ld] -= sr;
  r.im[b + c * r.ld] -= si;
}

template <typename T>
void tree_top_subtract(hipStream_t s, DMat<T> RT, DMat<T> U, int64_t cols, int npoles,
                       const TreeDev& tr) {
  k_tree_top_subtract<T><<<dim3(grid1(tr.TP * cols), npoles), 256, 0, s>>>(
      RT, U, tr.TP, cols, tr.L, tr.tptr.as<int32_t>(), tr.tent.as<int32_t>(), tr.TGP);
  RFD_CHECK_LAUNCH();
}

#define RFD_TREE_INST(T)                                                                     \
  template void tree_tt_update<T>(hipStream_t, DMat<T>, DMat<T>, int, const TreeDev&);      \
  template void tree_gather_top<T>(hipStream_t, DMat<T>, DMat<T>, int64_t, int,             \
                                   const TreeDev&);                                          \
  template void tree_top_subtract<T>(hipStream_t, DMat<T>, DMat<T>, int64_t, int,           \
                                     const TreeDev&);
RFD_TREE_INST(float)
RFD_TREE_INST(double)

}  // namespace rfd
