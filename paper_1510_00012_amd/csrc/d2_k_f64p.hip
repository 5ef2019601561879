// FP64 plan-update kernels for the launches that form no support terms.
#include "d2_kinst.hpp"

void d2k_fill_f64p(d2k::KernTable<double>* t) {
  d2k::fill_table<double, true>(*t);
}
