// FP64 kernel instantiations, row paddings 8 and 16.
#include "d2_kinst.hpp"

void d2k_fill_f64(d2k::KernTable<double>* t) {
  d2k::fill_table<double, false, 8, 16>(*t);
}
