// Host-side pencil model: CSR validation, the interior-first reordering maps
// (Sec. 2.3, eq. (2.5)), local blocks, subdomain colouring, filter poles.
#include "pencil.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <string>

namespace rfd {

Csr make_csr(int64_t n, const int64_t* ptr, const int32_t* idx, const double* val,
             const char* name) {
  if (n < 1) throw Error(ST_EINVAL, std::string(name) + ": n < 1");
  if (!ptr || !idx || !val) throw Error(ST_EINVAL, std::string(name) + ": null array");
  if (ptr[0] != 0) throw Error(ST_EINVAL, std::string(name) + ": ptr[0] != 0");
  for (int64_t i = 0; i < n; ++i)
    if (ptr[i + 1] < ptr[i]) throw Error(ST_EINVAL, std::string(name) + ": ptr not monotone");
  Csr A;
  A.n = n;
  A.ptr.assign(n + 1, 0);
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < n; ++i) {
    row.clear();
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
      if (idx[e] < 0 || idx[e] >= n)
        throw Error(ST_EINVAL, std::string(name) + ": column index out of range");
      if (!std::isfinite(val[e])) throw Error(ST_EINVAL, std::string(name) + ": non-finite value");
      row.emplace_back(idx[e], val[e]);
    }
    std::sort(row.begin(), row.end(),
              [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                return a.first < b.first;
              });
    for (size_t k = 0; k < row.size();) {
      size_t l = k;
      double v = 0;
      while (l < row.size() && row[l].first == row[k].first) v += row[l++].second;
      A.idx.push_back(row[k].first);
      A.val.push_back(v);
      k = l;
    }
    A.ptr[i + 1] = (int64_t)A.idx.size();
  }
  return A;
}

static double csr_get(const Csr& A, int64_t i, int32_t j) {
  auto b = A.idx.begin() + A.ptr[i], e = A.idx.begin() + A.ptr[i + 1];
  auto it = std::lower_bound(b, e, j);
  if (it != e && *it == j) return A.val[it - A.idx.begin()];
  return 0.0;
}

void check_symmetric(const Csr& A, const char* name) {
  double mx = 0;
  for (double v : A.val) mx = std::max(mx, std::fabs(v));
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
      if (std::fabs(A.val[e] - csr_get(A, A.idx[e], (int32_t)i)) > 1e-12 * mx)
        throw Error(ST_EINVAL, std::string(name) + " is not symmetric");
}

SchurRenumber make_schur_renumber(const Partition& P, int64_t D, int64_t nb) {
  SchurRenumber R;
  const int p = P.p;
  R.B.resize(p);
  R.E.resize(p);
  R.Et.resize(p);
  R.pos.resize(p);
  int64_t smax = 0;
  for (int j = 0; j < p; ++j) {
    const PairCsr &B = P.Bloc[j], &E = P.Eloc[j], &Et = P.EtLoc[j];
    const int64_t d = B.rows, pad = D - d;
    if (pad < 0) throw Error(ST_EINVAL, "schur renumbering: block larger than D");
    std::vector<int32_t> perm;
    std::vector<int32_t>& pinv = R.pos[j];
    pinv.assign(d, 0);
    int64_t touched = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int64_t r = 0; r < d; ++r)
        if ((E.ptr[r + 1] > E.ptr[r]) == (pass == 1)) perm.push_back((int32_t)r);
    for (int64_t q = 0; q < d; ++q) pinv[perm[q]] = (int32_t)(pad + q);
    for (int64_t r = 0; r < d; ++r) touched += E.ptr[r + 1] > E.ptr[r] ? 1 : 0;
    smax = std::max(smax, touched);
    R.SJ = std::max<int64_t>(R.SJ, E.cols);
    PairCsr& b = R.B[j];
    PairCsr& ee = R.E[j];
    b.rows = b.cols = D;
    ee.rows = D;
    ee.cols = E.cols;
    b.ptr.assign(1, 0);
    ee.ptr.assign(1, 0);
    for (int64_t q = 0; q < pad; ++q) {
      b.idx.push_back((int32_t)q);
      b.a.push_back(1.0);
      b.m.push_back(0.0);
      b.ptr.push_back((int64_t)b.idx.size());
      ee.ptr.push_back((int64_t)ee.idx.size());
    }
    for (int64_t q = 0; q < d; ++q) {
      const int32_t r = perm[q];
      for (int64_t k = B.ptr[r]; k < B.ptr[r + 1]; ++k) {
        b.idx.push_back(pinv[B.idx[k]]);
        b.a.push_back(B.a[k]);
        b.m.push_back(B.m[k]);
      }
      b.ptr.push_back((int64_t)b.idx.size());
      for (int64_t k = E.ptr[r]; k < E.ptr[r + 1]; ++k) {
        ee.idx.push_back(E.idx[k]);
        ee.a.push_back(E.a[k]);
        ee.m.push_back(E.m[k]);
      }
      ee.ptr.push_back((int64_t)ee.idx.size());
    }
    R.Et[j] = Et;
    for (auto& c : R.Et[j].idx) c = pinv[c];
    R.Et[j].cols = D;
  }
  R.TS = std::min<int64_t>((std::max<int64_t>(smax, 1) + nb - 1) / nb * nb, D);
  return R;
}

double abs_row_sum_max(const Csr& A) {
  double mx = 0;
  for (int64_t i = 0; i < A.n; ++i) {
    double s = 0;
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) s += std::fabs(A.val[e]);
    mx = std::max(mx, s);
  }
  return mx;
}

// Gauss-Legendre nodes on [-1, 1] by Newton's method on P_n (three-term
// recurrence), weights 2 / ((1 - t^2) P_n'(t)^2).  Returned as complex with
// zero imaginary part for uniformity with the pole arrays; ascending.
std::vector<std::complex<double>> gauss_legendre(int n, std::vector<double>* w) {
  std::vector<std::complex<double>> t(n);
  w->assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1; }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) {
        // one more evaluation of the derivative at the converged node
        p0 = 1; p1 = x;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        break;
      }
    }
    t[n - 1 - i] = x;
    (*w)[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return t;
}

// Sec. 2.1: circle centre c = (alpha+beta)/2, radius r = (beta-alpha)/2,
// nodes nu(theta) = c + r e^{i theta}; a rule with nodes theta_l and weights
// h_l on the upper half circle gives zeta_l = nu(theta_l),
// omega_l = -r e^{i theta_l} h_l / (2 pi)  (eq. (2.2) with dnu = i r e^{i theta}).
void make_poles(Poles& P, double alpha, double beta, int n_c, int rule, const double* zeta,
                const double* omega) {
  if (!(alpha < beta) || !std::isfinite(alpha) || !std::isfinite(beta))
    throw Error(ST_EINVAL, "need finite alpha < beta");
  if (n_c < 1 || n_c > 64) throw Error(ST_EINVAL, "need 1 <= n_c <= 64");
  P.alpha = alpha;
  P.beta = beta;
  P.n_c = n_c;
  P.zeta.assign(n_c, 0);
  P.omega.assign(n_c, 0);
  const double c = 0.5 * (alpha + beta), r = 0.5 * (beta - alpha);
  if (rule == 0 || rule == 1) {
    std::vector<double> th(n_c), h(n_c);
    if (rule == 1) {
      for (int l = 0; l < n_c; ++l) {
        th[l] = (l + 0.5) * M_PI / n_c;
        h[l] = M_PI / n_c;
      }
    } else {
      std::vector<double> w;
      auto t = gauss_legendre(n_c, &w);
      for (int l = 0; l < n_c; ++l) {
        th[l] = 0.5 * M_PI * (1.0 + t[l].real());
        h[l] = 0.5 * M_PI * w[l];
      }
    }
    for (int l = 0; l < n_c; ++l) {
      const std::complex<double> e = std::polar(1.0, th[l]);
      P.zeta[l] = c + r * e;
      P.omega[l] = -r * e * h[l] / (2.0 * M_PI);
    }
  } else if (rule == 2) {
    if (!zeta || !omega) throw Error(ST_EINVAL, "explicit rule needs zeta and omega");
    for (int l = 0; l < n_c; ++l) {
      P.zeta[l] = {zeta[2 * l], zeta[2 * l + 1]};
      P.omega[l] = {omega[2 * l], omega[2 * l + 1]};
      if (!(P.zeta[l].imag() > 0)) throw Error(ST_EINVAL, "explicit poles need Im > 0");
    }
  } else {
    throw Error(ST_EINVAL, "unknown quadrature rule");
  }
  P.set = true;
}

Partition make_partition(const Csr& A, const Csr& M, int p, const int32_t* part) {
  const int64_t n = A.n;
  if (p < 1) throw Error(ST_EINVAL, "need p >= 1");
  if (!part) throw Error(ST_EINVAL, "null partition");
  Partition P;
  P.p = p;
  P.part.assign(part, part + n);
  P.interior.assign(p, {});
  std::vector<int32_t> pos(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t q = part[i];
    if (q < -1 || q >= p) throw Error(ST_EINVAL, "partition value out of range");
    if (q >= 0) {
      pos[i] = (int32_t)P.interior[q].size();
      P.interior[q].push_back((int32_t)i);
    } else {
      pos[i] = (int32_t)P.iface.size();
      P.iface.push_back((int32_t)i);
    }
  }
  for (int j = 0; j < p; ++j)
    if (P.interior[j].empty()) throw Error(ST_EINVAL, "empty subdomain");
  if (P.iface.empty()) throw Error(ST_EINVAL, "empty interface");
  const int64_t s = (int64_t)P.iface.size();
  // direct coupling check and adjacency
  P.adj.assign(p, {});
  for (const Csr* X : {&A, &M})
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = X->ptr[i]; e < X->ptr[i + 1]; ++e) {
        const int32_t j = X->idx[e];
        const int32_t pi = part[i], pj = part[j];
        if (pi >= 0 && pj >= 0 && pi != pj && X->val[e] != 0.0)
          throw Error(ST_EINVAL, "two subdomains are coupled directly, not through the interface");
        if (pi >= 0 && pj < 0) P.adj[pi].push_back(pos[j]);
      }
  for (auto& a : P.adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  P.m_diag = true;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = M.ptr[i]; e < M.ptr[i + 1]; ++e)
      if (M.idx[e] != i && M.val[e] != 0.0) P.m_diag = false;
  // local pair-CSR blocks
  auto merged_row = [&](int64_t i, auto&& keep, auto&& local, std::vector<int32_t>& cols,
                        std::vector<double>& av, std::vector<double>& mv) {
    std::map<int32_t, std::pair<double, double>> acc;
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
      if (keep(A.idx[e])) acc[local(A.idx[e])].first += A.val[e];
    for (int64_t e = M.ptr[i]; e < M.ptr[i + 1]; ++e)
      if (keep(M.idx[e])) acc[local(M.idx[e])].second += M.val[e];
    for (auto& kv : acc) {
      cols.push_back(kv.first);
      av.push_back(kv.second.first);
      mv.push_back(kv.second.second);
    }
  };
  P.Bloc.resize(p);
  P.Eloc.resize(p);
  P.EtLoc.resize(p);
  P.m_e_zero = true;
  for (int j = 0; j < p; ++j) {
    const auto& I = P.interior[j];
    std::map<int32_t, int32_t> apos;
    for (size_t a = 0; a < P.adj[j].size(); ++a) apos[P.adj[j][a]] = (int32_t)a;
    PairCsr& B = P.Bloc[j];
    PairCsr& E = P.Eloc[j];
    B.rows = B.cols = (int64_t)I.size();
    E.rows = (int64_t)I.size();
    E.cols = (int64_t)P.adj[j].size();
    B.ptr.assign(1, 0);
    E.ptr.assign(1, 0);
    for (int32_t g : I) {
      merged_row(
          g, [&](int32_t c) { return part[c] == j; }, [&](int32_t c) { return pos[c]; }, B.idx,
          B.a, B.m);
      B.ptr.push_back((int64_t)B.idx.size());
      merged_row(
          g, [&](int32_t c) { return part[c] < 0; }, [&](int32_t c) { return apos[pos[c]]; },
          E.idx, E.a, E.m);
      E.ptr.push_back((int64_t)E.idx.size());
    }
    for (double v : E.m)
      if (v != 0.0) P.m_e_zero = false;
    // transpose of E
    PairCsr& Et = P.EtLoc[j];
    Et.rows = E.cols;
    Et.cols = E.rows;
    Et.ptr.assign(E.cols + 1, 0);
    for (int32_t c : E.idx) Et.ptr[c + 1]++;
    for (int64_t a = 0; a < E.cols; ++a) Et.ptr[a + 1] += Et.ptr[a];
    Et.idx.assign(E.idx.size(), 0);
    Et.a.assign(E.idx.size(), 0);
    Et.m.assign(E.idx.size(), 0);
    std::vector<int64_t> fillp(Et.ptr.begin(), Et.ptr.end() - 1);
    for (int64_t r = 0; r < E.rows; ++r)
      for (int64_t e = E.ptr[r]; e < E.ptr[r + 1]; ++e) {
        const int64_t d = fillp[E.idx[e]]++;
        Et.idx[d] = (int32_t)r;
        Et.a[d] = E.a[e];
        Et.m[d] = E.m[e];
      }
    P.d_max = std::max<int64_t>(P.d_max, (int64_t)I.size());
    P.sj_max = std::max<int64_t>(P.sj_max, (int64_t)P.adj[j].size());
  }
  PairCsr& C = P.Cloc;
  C.rows = C.cols = s;
  C.ptr.assign(1, 0);
  for (int32_t g : P.iface) {
    merged_row(
        g, [&](int32_t c) { return part[c] < 0; }, [&](int32_t c) { return pos[c]; }, C.idx,
        C.a, C.m);
    C.ptr.push_back((int64_t)C.idx.size());
  }
  // greedy colouring: subdomains sharing an adjacent interface node differ
  std::vector<std::vector<int>> touch(s);
  for (int j = 0; j < p; ++j)
    for (int32_t a : P.adj[j]) touch[a].push_back(j);
  std::vector<int> color(p, -1);
  int ncol = 0;
  for (int j = 0; j < p; ++j) {
    std::vector<char> used(ncol + 1, 0);
    for (int32_t a : P.adj[j])
      for (int q : touch[a])
        if (color[q] >= 0) used[color[q]] = 1;
    int c = 0;
    while (used[c]) ++c;
    color[j] = c;
    ncol = std::max(ncol, c + 1);
  }
  P.colors.assign(ncol, {});
  for (int j = 0; j < p; ++j) P.colors[color[j]].push_back(j);
  return P;
}

}  // namespace rfd
