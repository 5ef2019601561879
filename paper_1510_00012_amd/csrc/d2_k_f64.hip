// FP64 kernel instantiations.
#include "d2_kinst.hpp"

void d2k_fill_f64(d2k::KernTable<double>* t) {
  d2k::fill_table<double, false>(*t);
}
