// k_mfma.hip -- BF16 matrix-core objective/gradient path.
#include "pd_host.h"

pd_status pd_bf16_objective_grad(pd_ctx *ctx, const pd_problem *, int, const double *const *,
                                 double *, double *const *, hipStream_t) {
  return pd_fail(ctx, PD_ERR_UNSUPPORTED, "PD_BF16: not built yet");
}

void pd_bf16_plan_eval(pd_ctx *, const EvalPlan &P, hipStream_t s, bool center) {
  pd_plan_eval(P, true, s, center);
}

pd_status pd_warm_start(pd_ctx *ctx, const pd_problem *, int, double *const *, const void *, int,
                        hipStream_t) {
  return pd_fail(ctx, PD_ERR_UNSUPPORTED, "PD_INIT_MLP: not built yet");
}

void pd_bf16_profile_stages(pd_ctx *, const EvalPlan &P, int reps, hipStream_t s, hipEvent_t *ev) {
  for (int r = 0; r < reps; ++r) pd_launch_prep(P.prec, P.d_maps, P.d_offP, P.n, P.offP[P.n], s);
  (void)hipEventRecord(ev[1], s);
  for (int r = 0; r < reps; ++r) pd_launch_lse(P.prec, P.dmax, P.d_maps, P.d_offA, P.n, P.offA[P.n], s);
  (void)hipEventRecord(ev[2], s);
  for (int r = 0; r < reps; ++r) pd_launch_grad(P.prec, P.dmax, P.d_maps, P.d_offB, P.n, P.offB[P.n], s);
  (void)hipEventRecord(ev[3], s);
}
