// FP32 kernel instantiations, row paddings 32 and 64.
#include "d2_kinst.hpp"

void d2k_fill_f32w(d2k::KernTable<float>* t) {
  d2k::fill_table<float, false, 32, 64>(*t);
}
