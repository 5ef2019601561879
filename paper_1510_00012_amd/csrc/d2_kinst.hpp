// Instantiation of the kernel tables for one element type (included by the
// per-type translation units so that they compile in parallel).
#pragma once
#include "d2_kernels.hpp"

namespace d2k {

constexpr int clog2(int v) { return v <= 1 ? 0 : 1 + clog2(v / 2); }

template <typename T, int MP, int R> void add_kernels(KernTable<T>& t) {
  constexpr int a = clog2(MP) - 3, b = clog2(R);
  t.ba[0][a][b] = &k_iter_ba<T, MP, R, false>;
  t.ba[1][a][b] = &k_iter_ba<T, MP, R, true>;
  if constexpr (sizeof(T) == 4 && (MP == 16 || MP == 32))
    t.bax[a][b] = &k_iter_ba<T, MP, R, false, kVarSupport>;
  if constexpr (sizeof(T) == 4 && MP == 32)
    t.bcx[b] = &k_iter_ba<T, MP, R, false, kVarCost>;
  t.aux[a][b] = &k_aux<T, MP, R>;
  t.asg[a][b] = &k_assign<T, MP, R>;
}

// Tiles up to 2048 entries: R * (64 / MP) columns of MP rows, m_k <= 64.
template <typename T> void fill_table(KernTable<T>& t) {
  add_kernels<T, 8, 1>(t);  add_kernels<T, 8, 2>(t);
  add_kernels<T, 8, 4>(t);  add_kernels<T, 8, 8>(t);
  add_kernels<T, 16, 1>(t); add_kernels<T, 16, 2>(t);
  add_kernels<T, 16, 4>(t); add_kernels<T, 16, 8>(t);
  add_kernels<T, 16, 16>(t);
  add_kernels<T, 32, 1>(t); add_kernels<T, 32, 2>(t);
  add_kernels<T, 32, 4>(t); add_kernels<T, 32, 8>(t);
  add_kernels<T, 32, 16>(t); add_kernels<T, 32, 32>(t);
  add_kernels<T, 64, 1>(t); add_kernels<T, 64, 2>(t);
  add_kernels<T, 64, 4>(t); add_kernels<T, 64, 8>(t);
  add_kernels<T, 64, 16>(t); add_kernels<T, 64, 32>(t);
}

}  // namespace d2k
