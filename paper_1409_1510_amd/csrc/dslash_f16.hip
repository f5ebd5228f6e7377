// Instances of the multi-rhs half Dslash with FP16 link storage and FP32 arithmetic/vectors, Naik
// stored with 18 or 14 reals (13 and 9: dslash_f16c.hip).
#include "dslash_kernel.hpp"

dslash::DslashFn dslash_fn_f16c(bool epi, int recon, int rt, int spb, bool nt, int lds);

dslash::DslashFn dslash_fn_f16(bool epi, int recon, int rt, int spb, bool nt, int lds) {
  if (recon == 18) return dslash::pick_all<float, __half2, 18>(epi, rt, spb, nt, lds);
  if (recon == 14) return dslash::pick_all<float, __half2, 14>(epi, rt, spb, nt, lds);
  return dslash_fn_f16c(epi, recon, rt, spb, nt, lds);
}
