// FP32 instances of the multi-rhs half Dslash with the Naik links stored in 13 or 9 reals.
#include "dslash_kernel.hpp"

dslash::DslashFn dslash_fn_f32c(bool epi, int recon, int rt, int spb, bool nt, int lds) {
  if (recon == 13) return dslash::pick_all<float, float2, 13>(epi, rt, spb, nt, lds);
  if (recon == 9) return dslash::pick_all<float, float2, 9>(epi, rt, spb, nt, lds);
  return nullptr;
}
