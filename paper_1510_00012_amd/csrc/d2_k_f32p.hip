// FP32 plan-update kernels for the launches that form no support terms.
#include "d2_kinst.hpp"

void d2k_fill_f32p(d2k::KernTable<float>* t) {
  d2k::fill_table<float, true>(*t);
}
