// Instantiation of the kernel tables for one element type (included by the
// per-type translation units so that they compile in parallel).
#pragma once
#include "d2_kernels.hpp"

namespace d2k {

constexpr int clog2(int v) { return v <= 1 ? 0 : 1 + clog2(v / 2); }

template <typename T, int MP, int R, bool PLAIN>
void add_kernels(KernTable<T>& t) {
  constexpr int a = clog2(MP) - 3, b = clog2(R);
  if constexpr (PLAIN) {
    // launches that form no support terms
    t.bap[0][a][b] = &k_iter_ba<T, MP, R, false, kVarPlain>;
    t.bap[1][a][b] = &k_iter_ba<T, MP, R, true, kVarPlain>;
    if constexpr (sizeof(T) == 4) {
      t.bapn[0][a][b] = &k_iter_ba<T, MP, R, false, kVarPlain, kCpolStream>;
      t.bapn[1][a][b] = &k_iter_ba<T, MP, R, true, kVarPlain, kCpolStream>;
    }
    t.auxm[0][a][b] = &k_aux<T, MP, R, kRho>;
    t.auxm[1][a][b] = &k_aux<T, MP, R, kA0>;
    t.auxm[2][a][b] = &k_aux<T, MP, R, kBF>;
  } else {
    t.ba[0][a][b] = &k_iter_ba<T, MP, R, false>;
    t.ba[1][a][b] = &k_iter_ba<T, MP, R, true>;
    if constexpr (sizeof(T) == 4)
      t.ban[a][b] = &k_iter_ba<T, MP, R, false, kVarNone, kCpolStream>;
    if constexpr (sizeof(T) == 4 && (MP == 16 || MP == 32)) {
      t.sup[0][a][b] = &k_sup_mfma<MP, R, 0>;
      t.sup[1][a][b] = &k_sup_mfma<MP, R, kCpolStream>;
    }
    if constexpr (sizeof(T) == 4 && MP == 32) t.cst[b] = &k_cost_mfma<R>;
    if constexpr (sizeof(T) == 4) t.cstv[a][b] = &k_cost_valu<MP, R>;
    t.aux[a][b] = &k_aux<T, MP, R>;
    t.asg[a][b] = &k_assign<T, MP, R>;
  }
}

// Tiles up to 2048 entries: R * (64 / MP) columns of MP rows, m_k <= 64.
// PLAIN: the kernels without support terms and the auxiliary kernels fixed
// to one mode (a translation unit of their own).  Row paddings MP in
// [LO, HI] only, so that one type's kernels compile in parallel units.
template <typename T, bool PLAIN, int LO = 8, int HI = 64>
void fill_table(KernTable<T>& t) {
  if constexpr (LO <= 8 && 8 <= HI) {
    add_kernels<T, 8, 1, PLAIN>(t);  add_kernels<T, 8, 2, PLAIN>(t);
    add_kernels<T, 8, 4, PLAIN>(t);  add_kernels<T, 8, 8, PLAIN>(t);
  }
  if constexpr (LO <= 16 && 16 <= HI) {
    add_kernels<T, 16, 1, PLAIN>(t); add_kernels<T, 16, 2, PLAIN>(t);
    add_kernels<T, 16, 4, PLAIN>(t); add_kernels<T, 16, 8, PLAIN>(t);
    add_kernels<T, 16, 16, PLAIN>(t);
  }
  if constexpr (LO <= 32 && 32 <= HI) {
    add_kernels<T, 32, 1, PLAIN>(t); add_kernels<T, 32, 2, PLAIN>(t);
    add_kernels<T, 32, 4, PLAIN>(t); add_kernels<T, 32, 8, PLAIN>(t);
    add_kernels<T, 32, 16, PLAIN>(t); add_kernels<T, 32, 32, PLAIN>(t);
  }
  if constexpr (LO <= 64 && 64 <= HI) {
    add_kernels<T, 64, 1, PLAIN>(t); add_kernels<T, 64, 2, PLAIN>(t);
    add_kernels<T, 64, 4, PLAIN>(t); add_kernels<T, 64, 8, PLAIN>(t);
    add_kernels<T, 64, 16, PLAIN>(t); add_kernels<T, 64, 32, PLAIN>(t);
  }
}

}  // namespace d2k
