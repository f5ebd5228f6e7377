// FP32 instances of the multi-rhs half Dslash (vectors complex64, FP32 links, 18 or 14 reals).
#include "dslash_kernel.hpp"

dslash::DslashFn dslash_fn_f32(bool epi, bool r14, int rt, int spb, bool nt, int lds) {
  return r14 ? dslash::pick_all<float, float2, true>(epi, rt, spb, nt, lds)
             : dslash::pick_all<float, float2, false>(epi, rt, spb, nt, lds);
}
