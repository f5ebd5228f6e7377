// FP64 instances of the multi-rhs half Dslash (vectors complex128, FP64 links).
#include "dslash_kernel.hpp"

dslash::DslashFn dslash_fn_f64(bool epi, int rt, int spb, bool nt, int lds) {
  if (rt > 8) return nullptr;  // FP64 tiles above 8 spill
  return dslash::pick_all<double, double2, 18>(epi, rt, spb, nt, lds);
}
