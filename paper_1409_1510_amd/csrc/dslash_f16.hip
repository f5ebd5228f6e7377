// Instances of the multi-rhs half Dslash with FP16 link storage and FP32 arithmetic/vectors.
#include "dslash_kernel.hpp"

dslash::DslashFn dslash_fn_f16(bool epi, bool r14, int rt, int spb, bool nt, int lds) {
  return r14 ? dslash::pick_all<float, __half2, true>(epi, rt, spb, nt, lds)
             : dslash::pick_all<float, __half2, false>(epi, rt, spb, nt, lds);
}
