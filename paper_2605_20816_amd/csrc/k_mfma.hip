// k_mfma.hip -- BF16 matrix-core objective/gradient path.
#include "pd_host.h"

pd_status pd_bf16_objective_grad(pd_ctx *ctx, const pd_problem *, int, const double *const *,
                                 double *, double *const *, hipStream_t) {
  return pd_fail(ctx, PD_ERR_UNSUPPORTED, "PD_BF16: not built yet");
}
