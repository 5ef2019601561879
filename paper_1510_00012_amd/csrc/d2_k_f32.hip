// FP32 kernel instantiations (row paddings 8 and 16) and the per-cluster
// finalisation kernels.
#include "d2_kinst.hpp"

void d2k_fill_f32(d2k::KernTable<float>* t) {
  d2k::fill_table<float, false, 8, 16>(*t);
}

void d2k_fill_fin(d2k::FinFn* f) {
  f[0] = &d2k::k_fin<8>;
  f[1] = &d2k::k_fin<16>;
  f[2] = &d2k::k_fin<32>;
  f[3] = &d2k::k_fin<64>;
}
