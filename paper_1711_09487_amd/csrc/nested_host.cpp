// Two-level interface Schur complement: validation of the caller's grouping
// and the index maps of the blocked layout (host only; see nested.hpp).
#include <algorithm>
#include <set>

#include "nested.hpp"

namespace rfd {

TreeHost build_tree(const Partition& P, int64_t SJ, int L, const int32_t* group) {
  TreeHost h;
  const int64_t s = (int64_t)P.iface.size();
  if (L < 1) throw Error(ST_EINVAL, "interface groups: need at least one group");
  if (!group) throw Error(ST_EINVAL, "interface groups: null array");
  h.L = L;
  h.s = s;
  h.ng.assign(L, 0);
  h.kind.assign(s, 1);
  h.grp.assign(s, -1);
  h.loc.assign(s, -1);
  int64_t t = 0;
  for (int64_t a = 0; a < s; ++a) {
    const int32_t g = group[a];
    if (g < -1 || g >= L) throw Error(ST_EINVAL, "interface groups: value out of range");
    if (g >= 0) {
      h.kind[a] = 0;
      h.grp[a] = g;
      h.loc[a] = h.ng[g]++;
    } else {
      h.loc[a] = (int32_t)t++;
    }
  }
  for (int g = 0; g < L; ++g)
    if (h.ng[g] == 0) throw Error(ST_EINVAL, "interface groups: empty group");
  if (t == 0) throw Error(ST_EINVAL, "interface groups: empty top set");
  h.t = t;
  // C / M_C couple two different groups: not a two-level structure
  const PairCsr& C = P.Cloc;
  std::vector<std::set<int32_t>> tg(L);
  for (int64_t a = 0; a < s; ++a)
    for (int64_t e = C.ptr[a]; e < C.ptr[a + 1]; ++e) {
      const int32_t b = C.idx[e];
      const int32_t ga = group[a], gb = group[b];
      if (ga >= 0 && gb >= 0 && ga != gb && (C.a[e] != 0.0 || C.m[e] != 0.0))
        throw Error(ST_EINVAL, "interface groups: two groups are coupled in C");
      if (ga >= 0 && gb < 0) tg[ga].insert(h.loc[b]);
    }
  // subdomains: all adjacent group nodes in one group
  const int p = P.p;
  h.jgrp.assign(p, -1);
  for (int j = 0; j < p; ++j) {
    int gj = -1;
    for (int32_t a : P.adj[j])
      if (group[a] >= 0) {
        if (gj >= 0 && gj != group[a])
          throw Error(ST_EINVAL, "interface groups: a subdomain is adjacent to two groups");
        gj = group[a];
      }
    h.jgrp[j] = gj;
    if (gj >= 0)
      for (int32_t a : P.adj[j])
        if (group[a] < 0) tg[gj].insert(h.loc[a]);
  }
  int64_t ngmax = 0, tgmax = 1;
  h.tgn.assign(L, 0);
  for (int g = 0; g < L; ++g) {
    ngmax = std::max<int64_t>(ngmax, h.ng[g]);
    tgmax = std::max<int64_t>(tgmax, (int64_t)tg[g].size());
    h.tgn[g] = (int32_t)tg[g].size();
  }
  h.NGP = round_up(ngmax, 64);
  h.TGP = round_up(tgmax, 64);
  h.TP = round_up(t, 64);
  h.gpos.assign((size_t)L * h.NGP, -1);
  h.tpos.assign(h.TP, -1);
  for (int64_t a = 0; a < s; ++a) {
    if (h.kind[a] == 0)
      h.gpos[(size_t)h.grp[a] * h.NGP + h.loc[a]] = (int32_t)a;
    else
      h.tpos[h.loc[a]] = (int32_t)a;
  }
  // T_g (ascending top-local index) and, per top row, the (g, position) pairs
  h.tgidx.assign((size_t)L * h.TGP, -1);
  std::vector<std::vector<int32_t>> rows_of(t);
  std::vector<std::vector<int32_t>> posmap(L);  // top-local -> position in T_g (-1)
  for (int g = 0; g < L; ++g) {
    posmap[g].assign(t, -1);
    int32_t i = 0;
    for (int32_t b : tg[g]) {
      h.tgidx[(size_t)g * h.TGP + i] = b;
      posmap[g][b] = i;
      rows_of[b].push_back(g * (int32_t)h.TGP + i);
      ++i;
    }
  }
  h.tptr.assign(h.TP + 1, 0);
  for (int64_t b = 0; b < h.TP; ++b) {
    if (b < t)
      for (int32_t e : rows_of[b]) h.tent.push_back(e);
    h.tptr[b + 1] = (int32_t)h.tent.size();
  }
  if (h.tent.empty()) h.tent.push_back(0);
  // destinations of the C entries, grouped by block kind
  {
    std::vector<int32_t> e3[3], g3[3], r3[3], c3[3];
    for (int64_t a = 0; a < s; ++a)
      for (int64_t e = C.ptr[a]; e < C.ptr[a + 1]; ++e) {
        const int32_t b = C.idx[e];
        int k = -1, g = 0, r = 0, c = 0;
        if (h.kind[a] == 0 && h.kind[b] == 0) {
          if (h.grp[a] != h.grp[b]) continue;  // a zero entry between two groups
          k = 0, g = h.grp[a], r = h.loc[a], c = h.loc[b];
        } else if (h.kind[a] == 0) {
          k = 1, g = h.grp[a], r = h.loc[a], c = posmap[h.grp[a]][h.loc[b]];
        } else if (h.kind[b] == 1) {
          k = 2, r = h.loc[a], c = h.loc[b];
        } else {
          continue;  // top row, group column: the transpose of a stored S_gT entry
        }
        e3[k].push_back((int32_t)e);
        g3[k].push_back(g);
        r3[k].push_back(r);
        c3[k].push_back(c);
      }
    for (int k = 0; k < 3; ++k) {
      h.coff[k] = (int64_t)h.ce.size();
      h.ccnt[k] = (int64_t)e3[k].size();
      h.ce.insert(h.ce.end(), e3[k].begin(), e3[k].end());
      h.cg.insert(h.cg.end(), g3[k].begin(), g3[k].end());
      h.cr.insert(h.cr.end(), r3[k].begin(), r3[k].end());
      h.cc.insert(h.cc.end(), c3[k].begin(), c3[k].end());
    }
  }
  // per subdomain adjacency
  h.jkind.assign((size_t)p * SJ, 1);
  h.jloc.assign((size_t)p * SJ, -1);
  h.jtl.assign((size_t)p * SJ, -1);
  for (int j = 0; j < p; ++j)
    for (size_t q = 0; q < P.adj[j].size(); ++q) {
      const int32_t a = P.adj[j][q];
      const size_t o = (size_t)j * SJ + q;
      if (h.kind[a] == 0) {
        h.jkind[o] = 0;
        h.jloc[o] = h.loc[a];
      } else {
        h.jkind[o] = 1;
        h.jtl[o] = h.loc[a];
        h.jloc[o] = h.jgrp[j] >= 0 ? posmap[h.jgrp[j]][h.loc[a]] : -1;
      }
    }
  // colours of groups with disjoint T_g
  std::vector<int> color(L, -1);
  int ncol = 0;
  for (int g = 0; g < L; ++g) {
    std::vector<char> used(ncol + 1, 0);
    for (int g2 = 0; g2 < g; ++g2) {
      bool meet = false;
      for (int32_t b : tg[g])
        if (tg[g2].count(b)) {
          meet = true;
          break;
        }
      if (meet) used[color[g2]] = 1;
    }
    int c = 0;
    while (used[c]) ++c;
    color[g] = c;
    ncol = std::max(ncol, c + 1);
  }
  h.gcolors.assign(ncol, {});
  for (int g = 0; g < L; ++g) h.gcolors[color[g]].push_back(g);
  return h;
}

}  // namespace rfd
