// fit.hip -- device L-BFGS driver (pd_fit).
#include "pd_host.h"

void pd_fit_release(pd_ctx *) {}

extern "C" pd_status pd_fit(pd_ctx *ctx, const pd_problem *, int32_t, double *const *,
                            const pd_fit_opts *, pd_fit_report *, void *) {
  return pd_fail(ctx, PD_ERR_UNSUPPORTED, "pd_fit: not built yet");
}
