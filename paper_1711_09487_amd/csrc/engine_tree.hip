// The interface filter on the two-level S(zeta) (nested.hpp): block LU of the
// group blocks and the top Schur complement, the blocked solve, and the
// FP32 + FP64-refinement application of eq. (3.5).
#include <algorithm>

#include "dense.hpp"
#include "engine_impl.hpp"

namespace rfd {

namespace {
// two planes (re, then im) of `items` matrices of ld x cols
template <typename T>
DMat<T> planes(DevBuf& b, int64_t ld, int64_t cols, int64_t items) {
  const int64_t bs = ld * cols;
  b.alloc(std::max<size_t>(b.bytes, (size_t)(2 * bs * items) * sizeof(T)));
  T* re = b.as<T>();
  return DMat<T>{re, re + bs * items, ld, bs};
}
}  // namespace

void Engine::set_interface_groups(int L, const int32_t* group) {
  d_->join_prepare();
  EngineImpl& e = *d_;
  e.factored = false;
  for (DevBuf* b : {&e.S64, &e.S32, &e.Sinv32, &e.Sinv64, &e.Swide, &e.Swork, &e.Ssum, &e.Tgg64,
                    &e.TgT64, &e.Ttt64, &e.Txc64, &e.Tgg32, &e.TgT32, &e.Txc32, &e.Ttt32, &e.Tinvg,
                    &e.Tinvt, &e.Twide, &e.Twork, &e.Tgt})
    b->release();
  if (L <= 0) {
    e.tree = TreeDev{};
    return;
  }
  const TreeHost h = build_tree(*e.P, e.SJ, L, group);
  e.tree.upload(h);
}

int64_t EngineImpl::tree_pole_bytes(int64_t MP, int md) const {
  const TreeDev& t = tree;
  const int64_t G = t.NGP, TG = t.TGP, TP = t.TP, L = t.L;
  const bool f32 = md == 1;
  const int64_t e64 = 16, e32 = 8;  // complex element bytes
  int64_t b = (G * G * L + G * TG * L * 2 + TP * TP) * e64;           // S_gg, S_gT, X_g, S_TT
  if (f32) b += (G * G * L + G * TG * L * 2 + TP * TP) * e32;          // FP32 copies
  b += TG * TG * L * (f32 ? e32 : e64);                                // top updates
  b += ((int64_t)NB * 2 * (G * L + TP) + 256 * 2 * TP) * (f32 ? e32 : e64);  // inverses
  b += (G * L + TP) * MP * (f32 ? 2 * e64 + e32 : e64);                // right-hand sides
  b += TG * MP * L * 2 * e64;                                           // U, gathered top rows
  return b;
}

// Block LU of the window's S(zeta_l): each S_gg, X_g = S_gg^{-1} S_gT, the
// top complement S_TT - sum_g S_gT^T X_g, and its LU (with wide leaves for
// the solves).  FP32 factors (s_mode 1) are FP32 copies; the FP64 blocks stay.
void EngineImpl::tree_factor(hipStream_t st, int nc) {
  const TreeDev& tr = tree;
  const int64_t G = tr.NGP, TG = tr.TGP, TP = tr.TP;
  const int ni = nc * tr.L;
  auto top_wide = [&](auto* tag, auto C, auto Ci) {
    using T = std::remove_pointer_t<decltype(tag)>;
    TLW = (TP % 256 == 0 && TP > 256) ? 256 : ((TP % 128 == 0 && TP > 128) ? 128 : 0);
    if (!TLW) return;
    DMat<T> w2 = planes<T>(Twide, TLW, 2 * TP, nc);
    const int64_t mw = (int64_t)(TLW / 2) * (TLW / 2) * std::max<int64_t>(TP / TLW, nc);
    Twork.alloc(std::max<size_t>(Twork.bytes, (size_t)(2 * mw) * sizeof(T)));
    DMat<T> wk{Twork.as<T>(), Twork.as<T>() + mw, TLW / 2, 0};
    merge_inverses<T>(st, C, Ci, TP, nc, w2, TLW, wk);
  };
  if (s_mode == 1) {
    DMat<double> Sgg{Tgg64.as<double>(), Tgg64.as<double>() + G * G * ni, G, G * G};
    DMat<double> SgT{TgT64.as<double>(), TgT64.as<double>() + G * TG * ni, G, G * TG};
    DMat<double> Stt{Ttt64.as<double>(), Ttt64.as<double>() + TP * TP * nc, TP, TP * TP};
    DMat<float> A = planes<float>(Tgg32, G, G, ni);
    DMat<float> Ai = planes<float>(Tinvg, NB, 2 * G, ni);
    convert<float, double>(st, Sgg, A, G, G, ni);
    lu_nopiv<float>(st, A, G, ni, Ai, flags.as<unsigned>(), 1e-30);
    DMat<float> B = planes<float>(TgT32, G, TG, ni);
    DMat<float> X = planes<float>(Txc32, G, TG, ni);
    convert<float, double>(st, SgT, B, G, TG, ni);
    convert<float, float>(st, B, X, G, TG, ni);
    lu_solve<float>(st, A, Ai, nullptr, G, X, TG, ni);
    DMat<float> Gt = planes<float>(Tgt, TG, TG, ni);
    gemm<float>(st, true, false, TG, TG, G, 1.f, B, X, 0.f, Gt, ni);
    DMat<float> C = planes<float>(Ttt32, TP, TP, nc);
    convert<float, double>(st, Stt, C, TP, TP, nc);
    tree_tt_update<float>(st, C, Gt, nc, tr);
    DMat<float> Ci = planes<float>(Tinvt, NB, 2 * TP, nc);
    lu_nopiv<float>(st, C, TP, nc, Ci, flags.as<unsigned>(), 1e-30);
    top_wide((float*)nullptr, C, Ci);
  } else {
    DMat<double> A{Tgg64.as<double>(), Tgg64.as<double>() + G * G * ni, G, G * G};
    DMat<double> B{TgT64.as<double>(), TgT64.as<double>() + G * TG * ni, G, G * TG};
    DMat<double> C{Ttt64.as<double>(), Ttt64.as<double>() + TP * TP * nc, TP, TP * TP};
    DMat<double> Ai = planes<double>(Tinvg, NB, 2 * G, ni);
    lu_nopiv<double>(st, A, G, ni, Ai, flags.as<unsigned>(), 1e-300);
    DMat<double> X = planes<double>(Txc64, G, TG, ni);
    convert<double, double>(st, B, X, G, TG, ni);
    lu_solve<double>(st, A, Ai, nullptr, G, X, TG, ni);
    DMat<double> Gt = planes<double>(Tgt, TG, TG, ni);
    gemm<double>(st, true, false, TG, TG, G, 1.0, B, X, 0.0, Gt, ni);
    tree_tt_update<double>(st, C, Gt, nc, tr);
    DMat<double> Ci = planes<double>(Tinvt, NB, 2 * TP, nc);
    lu_nopiv<double>(st, C, TP, nc, Ci, flags.as<unsigned>(), 1e-300);
    top_wide((double*)nullptr, C, Ci);
  }
  // the top updates are large at the 63^3 size and not needed again
  if (Tgt.bytes > (size_t(1) << 30)) {
    RFD_HIP(hipStreamSynchronize(st));
    Tgt.release();
  }
}

// R <- S^{-1} R: forward through the groups (Z_g = S_gg^{-1} R_g,
// R_T -= sum_g S_gT^T Z_g), the top solve, then back (R_g = Z_g - X_g R_T[T_g]).
template <typename T>
void EngineImpl::tree_solve(hipStream_t st, DMat<T> RG, DMat<T> RT, int64_t MP, int nc) {
  const TreeDev& tr = tree;
  const int64_t G = tr.NGP, TG = tr.TGP, TP = tr.TP;
  const int ni = nc * tr.L;
  constexpr bool F32 = sizeof(T) == 4;
  DevBuf& bA = F32 ? Tgg32 : Tgg64;
  DevBuf& bB = F32 ? TgT32 : TgT64;
  DevBuf& bX = F32 ? Txc32 : Txc64;
  DevBuf& bC = F32 ? Ttt32 : Ttt64;
  DMat<T> A{bA.as<T>(), bA.as<T>() + G * G * ni, G, G * G};
  DMat<T> B{bB.as<T>(), bB.as<T>() + G * TG * ni, G, G * TG};
  DMat<T> X{bX.as<T>(), bX.as<T>() + G * TG * ni, G, G * TG};
  DMat<T> C{bC.as<T>(), bC.as<T>() + TP * TP * nc, TP, TP * TP};
  DMat<T> Ai{Tinvg.as<T>(), Tinvg.as<T>() + (int64_t)NB * 2 * G * ni, NB, (int64_t)NB * 2 * G};
  DMat<T> Ci{Tinvt.as<T>(), Tinvt.as<T>() + (int64_t)NB * 2 * TP * nc, NB, (int64_t)NB * 2 * TP};
  lu_solve<T>(st, A, Ai, nullptr, G, RG, MP, ni);
  DMat<T> U = planes<T>(TU, TG, MP, ni);
  gemm<T>(st, true, false, TG, MP, G, T(1), B, RG, T(0), U, ni);
  tree_top_subtract<T>(st, RT, U, MP, nc, tr);
  if (TLW) {
    const int64_t per = (int64_t)TLW * 2 * TP;
    DMat<T> w2{Twide.as<T>(), Twide.as<T>() + per * nc, TLW, per};
    const int64_t wp = (int64_t)TLW * MP;
    Twork.alloc(std::max<size_t>(Twork.bytes, (size_t)(2 * wp * nc) * sizeof(T)));
    DMat<T> wk{Twork.as<T>(), Twork.as<T>() + wp * nc, TLW, wp};
    lu_solve<T>(st, C, Ci, nullptr, TP, RT, MP, nc, 3, w2, TLW, wk);
  } else {
    lu_solve<T>(st, C, Ci, nullptr, TP, RT, MP, nc);
  }
  DMat<T> XTg = planes<T>(TXTg, TG, MP, ni);
  tree_gather_top<T>(st, RT, XTg, MP, nc, tr);
  gemm<T>(st, false, false, G, MP, TG, T(-1), X, XTg, T(1), RG, ni);
}

// W (+)= 2 Re sum_l omega_l S(zeta_l)^{-1} Y over the window's poles.  FP32
// factors: FP32 solves corrected by FP64 residuals R = Y - S X formed from the
// FP64 blocks (R_g = Y_g - S_gg X_g - S_gT X_T[T_g],
// R_T = Y_T - S_TT X_T - sum_g S_gT^T X_g).
void EngineImpl::tree_apply(hipStream_t st, const double* Y, int64_t ldy, int m, double* Wout,
                            int64_t ldw, bool add) {
  const TreeDev& tr = tree;
  const int nc = winn;
  const double* om = omega.as<double>() + 2 * (int64_t)win0;
  const int64_t G = tr.NGP, TG = tr.TGP, TP = tr.TP, MP = round_up(m, NB);
  const int ni = nc * tr.L;
  // sized for FP64 so that the FP32 solve and the FP64 residual share them
  TU.alloc(std::max<size_t>(TU.bytes, (size_t)(2 * TG * MP * ni) * sizeof(double)));
  TXTg.alloc(std::max<size_t>(TXTg.bytes, (size_t)(2 * TG * MP * ni) * sizeof(double)));
  DMat<double> RG = planes<double>(TRG, G, MP, ni), RT = planes<double>(TRT, TP, MP, nc);
  timer.begin(st, 4);
  if (s_mode == 1) {
    DMat<double> XG = planes<double>(TXG, G, MP, ni), XT = planes<double>(TXT, TP, MP, nc);
    DMat<float> RG3 = planes<float>(TRG32, G, MP, ni), RT3 = planes<float>(TRT32, TP, MP, nc);
    DMat<double> Sgg{Tgg64.as<double>(), Tgg64.as<double>() + G * G * ni, G, G * G};
    DMat<double> SgT{TgT64.as<double>(), TgT64.as<double>() + G * TG * ni, G, G * TG};
    DMat<double> Stt{Ttt64.as<double>(), Ttt64.as<double>() + TP * TP * nc, TP, TP * TP};
    zero_scalar(st, 1);
    DMat<double> Ym{const_cast<double*>(Y), nullptr, ldy, 0};
    absmax<double>(st, Ym, s, m, 1, scal.as<double>() + 1);
    const double ymax = read_scalar(st, 1);
    tree_broadcast(st, Y, ldy, m, RG, RT, MP, nc, tr);
    fill<double>(st, XG, G, MP, ni, 0.0);
    fill<double>(st, XT, TP, MP, nc, 0.0);
    int sw = 0;
    for (;; ++sw) {
      convert<float, double>(st, RG, RG3, G, MP, ni);
      convert<float, double>(st, RT, RT3, TP, MP, nc);
      tree_solve<float>(st, RG3, RT3, MP, nc);
      add_to<double, float>(st, RG3, XG, G, MP, ni);
      add_to<double, float>(st, RT3, XT, TP, MP, nc);
      tree_broadcast(st, Y, ldy, m, RG, RT, MP, nc, tr);
      DMat<double> U{TU.as<double>(), TU.as<double>() + TG * MP * ni, TG, TG * MP};
      DMat<double> XTg{TXTg.as<double>(), TXTg.as<double>() + TG * MP * ni, TG, TG * MP};
      gemm<double>(st, false, false, G, MP, G, -1.0, Sgg, XG, 1.0, RG, ni);
      tree_gather_top<double>(st, XT, XTg, MP, nc, tr);
      gemm<double>(st, false, false, G, MP, TG, -1.0, SgT, XTg, 1.0, RG, ni);
      gemm<double>(st, false, false, TP, MP, TP, -1.0, Stt, XT, 1.0, RT, nc);
      gemm<double>(st, true, false, TG, MP, G, 1.0, SgT, XG, 0.0, U, ni);
      tree_top_subtract<double>(st, RT, U, MP, nc, tr);
      zero_scalar(st, 0);
      absmax<double>(st, RG, G, MP, ni, scal.as<double>());
      absmax<double>(st, RT, TP, MP, nc, scal.as<double>());
      const double r = read_scalar(st, 0);
      if (!(r == r)) throw Error(ST_EBREAKDOWN, "non-finite residual in the filter solves");
      if (r <= tol * ymax) break;
      if (sw + 1 >= sweeps)
        throw Error(ST_ENOCONV, "filter refinement did not converge (residual " +
                                    std::to_string(r / ymax) + ")");
    }
    timer.sweeps_filter = std::max(timer.sweeps_filter, sw + 1);
    tree_accumulate(st, XG, XT, om, nc, Wout, ldw, m, add, tr);
  } else {
    tree_broadcast(st, Y, ldy, m, RG, RT, MP, nc, tr);
    tree_solve<double>(st, RG, RT, MP, nc);
    tree_accumulate(st, RG, RT, om, nc, Wout, ldw, m, add, tr);
  }
  timer.end(st);
}

template void EngineImpl::tree_solve<float>(hipStream_t, DMat<float>, DMat<float>, int64_t, int);
template void EngineImpl::tree_solve<double>(hipStream_t, DMat<double>, DMat<double>, int64_t,
                                             int);

}  // namespace rfd
