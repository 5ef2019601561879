// FP64 kernel instantiations, row paddings 32 and 64.
#include "d2_kinst.hpp"

void d2k_fill_f64w(d2k::KernTable<double>* t) {
  d2k::fill_table<double, false, 32, 64>(*t);
}
