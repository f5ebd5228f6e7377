// Learned gauge-covariant preconditioner (placeholder until the network kernels land).
#include "cg_state.hpp"
#include "internal.hpp"

struct NNState {};

void nn_free_state(hisq_ctx *ctx) {
  delete ctx->nn;
  ctx->nn = nullptr;
}

int fcg_nn_solve(hisq_ctx *ctx, double, int, const void *, void *, const hisq_cg_params *,
                 hisq_cg_stats *, CGState *, CGState *, double *) {
  return set_err(ctx, HISQ_ERR_STATE, "hisq_cg_mrhs: no network initialised");
}
