// FP32 instances of the multi-rhs half Dslash (vectors complex64, FP32 links, Naik stored with 18
// or 14 reals; the 13- and 9-real formats are instantiated in dslash_f32c.hip).
#include "dslash_kernel.hpp"

dslash::DslashFn dslash_fn_f32c(bool epi, int recon, int rt, int spb, bool nt, int lds);

dslash::DslashFn dslash_fn_f32(bool epi, int recon, int rt, int spb, bool nt, int lds) {
  if (recon == 18) return dslash::pick_all<float, float2, 18>(epi, rt, spb, nt, lds);
  if (recon == 14) return dslash::pick_all<float, float2, 14>(epi, rt, spb, nt, lds);
  return dslash_fn_f32c(epi, recon, rt, spb, nt, lds);
}
