// newton.hip -- inexact Newton ascent of Phi with Hessian-vector products
// (eq. hess of Proposition 4.4) and conjugate gradients, on the device.
//
// Gauge theta_N = 0 (on that subspace the Hessian of -Phi is positive definite,
// Proposition 4.11).  Per iteration, for every map still iterating:
//   g = grad(-Phi) with the last grain's row zeroed;
//   truncated CG on H d = -g from d = 0 (H the Hessian of -Phi, products from
//   pd_hessian_vec's kernels with the last row zeroed): stop after cg_max
//   steps, when ||r|| <= eta ||g||, eta = min(0.5, sqrt(||g||)) (the forcing
//   term of Eisenstat and Walker), or at non-positive curvature (d = -g if that
//   happens at the first step);
//   step halving from t = 1 until -Phi(x + t d) <= -Phi(x) + 1e-4 t g.d.
// All vector work and every decision run in one-block-per-map kernels with
// fixed-order sums; the host launches the phases and reads the per-map state
// back between them only to learn when a phase has finished everywhere.  The
// map's own flags gate the evaluation and Hessian-vector kernels, so a map that
// has stopped costs nothing.  Accuracy of every evaluated point comes from the
// certified arg-max inside the objective launch (exact FP64 accuracy).
#include "pd_host.h"

#include <math.h>
#include <string.h>

#include <chrono>
#include <string>

namespace {

// Per-map state (device).  Vectors are N x K FP64.
struct NtMap {
  double *x, *g, *d, *r, *p, *hp, *xt, *gt;
  const double *phi_t;      // Phi at xt (evaluation plan)
  const int64_t *part_c;    // certified-correct counts per row-segment item
  int64_t *fb_count;        // canonical-pass correct count
  double *cert;             // rounding bound slot
  int32_t *unc_count;       // uncertain-pixel count
  int c_items, nk, K;
  int64_t n_px;             // pixels
  // gates of the plans (1 = run): newton (iterating), cg (CG running), ls (line search)
  int32_t newton, cg, ls;
  int32_t status, iters, evals, hvps, cg_k, halvings;
  double f, gn, ginf, eta, rr, gd, t, acc;
  int64_t ncorr;
  int32_t hit;              // set when the map reaches the target (host times it)
};

constexpr int NT_BLOCK = 256;
enum { OP_INIT = 0, OP_CG_START, OP_CG_STEP, OP_LS_START, OP_LS_CHECK };

// Fixed-order block sum of one value per thread (tree over NT_BLOCK slots).
__device__ inline double nt_bsum(double v, double *red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = NT_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}
__device__ inline double nt_bmax(double v, double *red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = NT_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  return red[0];
}

// Number of correct pixels of the last evaluation (certified counts + canonical
// pass), then the slots cleared for the next evaluation.
__device__ inline int64_t nt_take_count(NtMap &S, double *red) {
  __shared__ long long cred[NT_BLOCK];
  long long c = 0;
  for (int t = threadIdx.x; t < S.c_items; t += NT_BLOCK) c += S.part_c[t];
  __syncthreads();
  cred[threadIdx.x] = c;
  __syncthreads();
  for (int w = NT_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) cred[threadIdx.x] += cred[threadIdx.x + w];
    __syncthreads();
  }
  const int64_t tot = cred[0] + *S.fb_count;
  __syncthreads();
  if (threadIdx.x == 0) {
    *S.cert = 0.0;
    *S.unc_count = 0;
    *S.fb_count = 0;
  }
  (void)red;
  return tot;
}

// g = -gt with the last row zeroed; returns (||g||^2, ||g||_inf) through red.
__device__ inline void nt_take_grad(NtMap &S, double *red, double &g2, double &ginf) {
  const int last = S.nk - S.K;
  double a = 0.0, m = 0.0;
  for (int e = threadIdx.x; e < S.nk; e += NT_BLOCK) {
    const double v = e >= last ? 0.0 : -S.gt[e];
    S.g[e] = v;
    a = fma(v, v, a);
    m = fmax(m, fabs(v));
  }
  g2 = nt_bsum(a, red);
  ginf = nt_bmax(m, red);
}

// The stop tests at an accepted point (or the start): target, gradient, budget.
__device__ inline void nt_stop_tests(NtMap &S, int max_iter, double gtol, double target) {
  if (S.acc >= target) {
    S.status = 0;
    S.hit = 1;
    S.newton = 0;
  } else if (!(S.gn > 0.0) || S.ginf <= gtol) {
    S.status = isfinite(S.gn) ? 2 : 4;
    S.newton = 0;
  } else if (S.iters >= max_iter) {
    S.status = 1;
    S.newton = 0;
  }
}

__global__ __launch_bounds__(NT_BLOCK) void k_newton(NtMap *__restrict__ maps, int op, int cg_max,
                                                     int max_iter, double gtol, int max_halvings,
                                                     double target) {
  NtMap &S = maps[blockIdx.x];
  __shared__ double red[NT_BLOCK];
  const int nk = S.nk, last = nk - S.K;
  if (op == OP_INIT) {
    // start: xt = x was evaluated (all gates open); x is already in the gauge
    const int64_t nc = nt_take_count(S, red);
    double g2, ginf;
    nt_take_grad(S, red, g2, ginf);
    if (threadIdx.x == 0) {
      S.evals = 1;
      S.ncorr = nc;
      S.acc = (double)nc / (double)S.n_px;
      S.f = -*S.phi_t;
      S.gn = sqrt(g2);
      S.ginf = ginf;
      S.ls = 0;
      S.newton = 1;
      if (!isfinite(S.f)) {
        S.status = 4;
        S.newton = 0;
      } else {
        nt_stop_tests(S, max_iter, gtol, target);
      }
    }
    return;
  }
  if (op == OP_CG_START) {
    if (!S.newton) return;
    double a = 0.0;
    for (int e = threadIdx.x; e < nk; e += NT_BLOCK) {
      const double v = -S.g[e];
      S.d[e] = 0.0;
      S.r[e] = v;
      S.p[e] = v;
      a = fma(v, v, a);
    }
    const double rr = nt_bsum(a, red);
    if (threadIdx.x == 0) {
      S.rr = rr;
      S.eta = fmin(0.5, sqrt(S.gn));
      S.cg_k = 0;
      S.cg = 1;
    }
    return;
  }
  if (op == OP_CG_STEP) {
    if (!S.cg) return;
    double a = 0.0;
    for (int e = threadIdx.x; e < last; e += NT_BLOCK) a = fma(S.p[e], S.hp[e], a);
    const double pHp = nt_bsum(a, red);
    if (!(pHp > 0.0)) {
      // non-positive curvature: keep d (d = -g at the first step)
      if (S.cg_k == 0)
        for (int e = threadIdx.x; e < nk; e += NT_BLOCK) S.d[e] = -S.g[e];
      __syncthreads();
      if (threadIdx.x == 0) {
        S.cg_k += 1;
        S.hvps += 1;
        S.cg = 0;
      }
      return;
    }
    const double alpha = S.rr / pHp;
    double b = 0.0;
    for (int e = threadIdx.x; e < nk; e += NT_BLOCK) {
      const double hp = e >= last ? 0.0 : S.hp[e];
      S.d[e] = fma(alpha, S.p[e], S.d[e]);
      const double rn = fma(-alpha, hp, S.r[e]);
      S.r[e] = rn;
      b = fma(rn, rn, b);
    }
    const double rr_new = nt_bsum(b, red);
    const bool done = sqrt(rr_new) <= S.eta * S.gn || S.cg_k + 1 >= cg_max;
    if (!done) {
      const double beta = rr_new / S.rr;
      for (int e = threadIdx.x; e < nk; e += NT_BLOCK) S.p[e] = fma(beta, S.p[e], S.r[e]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      S.cg_k += 1;
      S.hvps += 1;
      S.rr = rr_new;
      if (done) S.cg = 0;
    }
    return;
  }
  if (op == OP_LS_START) {
    if (!S.newton) return;
    double a = 0.0;
    for (int e = threadIdx.x; e < nk; e += NT_BLOCK) {
      a = fma(S.g[e], S.d[e], a);
      S.xt[e] = S.x[e] + S.d[e];
    }
    const double gd = nt_bsum(a, red);
    if (threadIdx.x == 0) {
      S.gd = gd;
      S.t = 1.0;
      S.halvings = 0;
      S.ls = 1;
    }
    return;
  }
  if (op == OP_LS_CHECK) {
    if (!S.ls) return;
    const int64_t nc = nt_take_count(S, red);
    const double fx = -*S.phi_t;
    const bool ok = fx <= S.f + 1e-4 * S.t * S.gd;  // false for NaN
    if (ok) {
      for (int e = threadIdx.x; e < nk; e += NT_BLOCK) S.x[e] = S.xt[e];
      double g2, ginf;
      nt_take_grad(S, red, g2, ginf);
      if (threadIdx.x == 0) {
        S.evals += 1;
        S.ls = 0;
        S.f = fx;
        S.gn = sqrt(g2);
        S.ginf = ginf;
        S.ncorr = nc;
        S.acc = (double)nc / (double)S.n_px;
        S.iters += 1;
        nt_stop_tests(S, max_iter, gtol, target);
      }
      return;
    }
    const bool fail = S.halvings + 1 >= max_halvings;
    const double t = 0.5 * S.t;
    if (!fail)
      for (int e = threadIdx.x; e < nk; e += NT_BLOCK) S.xt[e] = fma(t, S.d[e], S.x[e]);
    __syncthreads();
    if (threadIdx.x == 0) {
      S.evals += 1;
      S.halvings += 1;
      S.t = t;
      if (fail) {
        S.ls = 0;
        S.status = 3;
        S.newton = 0;
      }
    }
  }
}

// x <- x - x_{N-1} (the gauge theta_N = 0), and xt = x.
__global__ __launch_bounds__(NT_BLOCK) void k_newton_gauge(NtMap *__restrict__ maps) {
  NtMap &S = maps[blockIdx.x];
  __shared__ double lastrow[64];
  const int last = S.nk - S.K;
  if (threadIdx.x < S.K) lastrow[threadIdx.x] = S.x[last + threadIdx.x];
  __syncthreads();
  for (int e = threadIdx.x; e < S.nk; e += NT_BLOCK) {
    const double v = S.x[e] - lastrow[e % S.K];
    S.x[e] = v;
    S.xt[e] = v;
  }
  if (threadIdx.x == 0) {
    *S.cert = 0.0;
    *S.unc_count = 0;
    *S.fb_count = 0;
  }
}

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};
struct HostBuf {
  void *p = nullptr;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
};

}  // namespace

#define NT_HIP(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return pd_fail(ctx, PD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

extern "C" pd_status pd_fit_newton_cg(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                                      double *const *theta_inout, const pd_newton_opts *opts,
                                      pd_newton_report *reports, void *stream) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!probs || n_probs < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 maps");
  if (!theta_inout || !opts || !reports)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_inout, opts and reports must be non-NULL");
  int code;
  if (opts->prec == PD_FP64) code = 0;
  else if (opts->prec == PD_FP32) code = 1;
  else return pd_fail(ctx, PD_ERR_UNSUPPORTED, "pd_fit_newton_cg: PD_FP64 or PD_FP32");
  if (opts->max_iter < 0) return pd_fail(ctx, PD_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (opts->cg_max < 1 || opts->cg_max > 10000)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "cg_max must be in [1, 10000]");
  if (opts->max_halvings < 1 || opts->max_halvings > 60)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "max_halvings must be in [1, 60]");
  if (!(opts->gtol >= 0.0) || !(opts->target_acc == opts->target_acc))
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "gtol must be >= 0 and target_acc a number");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pd_check_problem(ctx, probs[p], p);
    if (st != PD_OK) return st;
    if (!theta_inout[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_inout[" + std::to_string(p) + "] is NULL");
  }
  NT_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int n = n_probs;

  // the objective at trial points (certified accuracy) and the Hessian-vector
  // products at the iterate share one workspace layout
  EvalPlan PE, PH;
  Arena L;
  PE.target_waves = PH.target_waves = pd_tuned_waves(ctx, probs, n, code);
  PE.cert = true;
  PE.onehot_pre = true;
  PE.sort = PH.sort = true;  // no one-hot gradient in the product plan
  pd_plan_layout(PE, L, probs, n, code);
  pd_plan_layout(PH, L, probs, n, code);
  std::vector<size_t> o_cv(n), o_ub(n);
  for (int p = 0; p < n; ++p) {
    const MapDev &M = PH.maps[p];
    o_cv[p] = L.take(sizeof(double) * (size_t)M.rows * M.Npad * M.DP);
    o_ub[p] = L.take(sizeof(double) * (size_t)M.rows * M.W);
  }
  const size_t o_phi = L.take(sizeof(double) * 2 * n);
  pd_status st = pd_reserve(ctx, L.off);
  if (st != PD_OK) return st;

  // state: 7 work vectors per map (x is the caller's buffer)
  size_t vec_total = 0;
  std::vector<size_t> vo(n);
  for (int p = 0; p < n; ++p) {
    vo[p] = vec_total;
    vec_total += 7 * (size_t)PE.maps[p].N * PE.maps[p].K;
  }
  DevBuf vecs, dstate;
  HostBuf hstate;
  NT_HIP(ctx, hipMalloc(&vecs.p, sizeof(double) * vec_total));
  NT_HIP(ctx, hipMalloc(&dstate.p, sizeof(NtMap) * n));
  NT_HIP(ctx, hipHostMalloc(&hstate.p, sizeof(NtMap) * n, hipHostMallocDefault));
  NtMap *dS = (NtMap *)dstate.p;
  NtMap *hS = (NtMap *)hstate.p;

  std::vector<double *> xt(n), gt(n), pv(n), hp(n);
  std::vector<const double *> xs(n);
  for (int p = 0; p < n; ++p) {
    const MapDev &M = PE.maps[p];
    const size_t nk = (size_t)M.N * M.K;
    double *b = (double *)vecs.p + vo[p];
    NtMap &S = hS[p];
    memset(&S, 0, sizeof(S));
    S.x = theta_inout[p];
    S.g = b;
    S.d = b + nk;
    S.r = b + 2 * nk;
    S.p = b + 3 * nk;
    S.hp = b + 4 * nk;
    S.xt = b + 5 * nk;
    S.gt = b + 6 * nk;
    S.nk = (int)nk;
    S.K = M.K;
    S.n_px = (int64_t)M.H * M.W;
    S.status = 1;
    xt[p] = S.xt;
    gt[p] = S.gt;
    pv[p] = S.p;
    hp[p] = S.hp;
    xs[p] = S.x;
  }
  double *phi = (double *)(ctx->ws + o_phi);
  pd_plan_bind(PE, ctx->ws, xt.data(), phi, gt.data(), nullptr, nullptr);
  pd_plan_bind(PH, ctx->ws, xs.data(), phi + n, hp.data(), nullptr, nullptr);
  for (int p = 0; p < n; ++p) {
    MapDev &E = PE.maps[p];
    NtMap &S = hS[p];
    S.phi_t = phi + p;
    S.part_c = E.part_c;
    S.c_items = E.a_items;
    S.fb_count = E.fb_count;
    S.cert = E.cert;
    S.unc_count = E.unc_count;
    S.ls = 1;
    E.gate = &dS[p].ls;
    MapDev &Hm = PH.maps[p];
    Hm.gate = &dS[p].cg;
    Hm.hv_in = S.p;
    Hm.Cv = ctx->ws + o_cv[p];
    Hm.ubar = (double *)(ctx->ws + o_ub[p]);
    Hm.onehot = nullptr;
    Hm.grad_scale = 1.0 / (Hm.eps * Hm.eps * (double)Hm.H * (double)Hm.W);
    Hm.grad_sign = 1.0;
  }
  NT_HIP(ctx, hipMemcpyAsync(dS, hS, sizeof(NtMap) * n, hipMemcpyHostToDevice, s));
  NT_HIP(ctx, pd_plan_upload(ctx, PE, s));
  NT_HIP(ctx, pd_plan_upload(ctx, PH, s));
  pd_plan_tables(PE, s);
  pd_plan_tables(PH, s);
  pd_plan_onehot(PE, s);

  const int mi = opts->max_iter, cgm = opts->cg_max, mh = opts->max_halvings;
  const double gtol = opts->gtol;
  const double target = opts->target_acc;
  auto op = [&](int o) { k_newton<<<n, NT_BLOCK, 0, s>>>(dS, o, cgm, mi, gtol, mh, target); };
  std::vector<double> t_hit(n, -1.0);
  auto sync_state = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(hS, dS, sizeof(NtMap) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
      const double now = std::chrono::duration<double>(clk::now() - t0).count();
      for (int p = 0; p < n; ++p)
        if (hS[p].hit && t_hit[p] < 0) t_hit[p] = now;
    }
    return e;
  };
  auto any = [&](int32_t NtMap::*f) {
    for (int p = 0; p < n; ++p)
      if (hS[p].*f) return true;
    return false;
  };

  k_newton_gauge<<<n, NT_BLOCK, 0, s>>>(dS);
  pd_plan_eval(PE, true, s, true);
  op(OP_INIT);
  NT_HIP(ctx, hipGetLastError());
  NT_HIP(ctx, sync_state());
  while (any(&NtMap::newton)) {
    op(OP_CG_START);
    // C and log-sum-exp at the iterate once; then one product per CG step
    pd_launch_center(PH.d_maps, PH.n, PH.max_k, s);
    pd_launch_prep(PH.prec, PH.d_maps, PH.d_offP, PH.n, PH.offP[PH.n], s);
    pd_launch_lse(PH.prec, PH.dmax, PH.d_maps, PH.d_offA, PH.n, PH.offA[PH.n], s);
    for (int k = 0; k < cgm; ++k) {
      pd_launch_hvp(PH.prec, PH.dmax, PH.d_maps, PH.d_offP, PH.d_offA, PH.d_offB, PH.n,
                    PH.offP[PH.n], PH.offA[PH.n], PH.offB[PH.n], s);
      pd_launch_reduce(PH.d_maps, PH.d_offR, PH.n, PH.offR[PH.n], true, false, s);
      op(OP_CG_STEP);
      NT_HIP(ctx, hipGetLastError());
      NT_HIP(ctx, sync_state());
      if (!any(&NtMap::cg)) break;
    }
    op(OP_LS_START);
    for (int h = 0; h < mh; ++h) {
      pd_plan_eval(PE, true, s, true);
      op(OP_LS_CHECK);
      NT_HIP(ctx, hipGetLastError());
      NT_HIP(ctx, sync_state());
      if (!any(&NtMap::ls)) break;
    }
  }
  const double total = std::chrono::duration<double>(clk::now() - t0).count();
  for (int p = 0; p < n; ++p) {
    const NtMap &S = hS[p];
    pd_newton_report &R = reports[p];
    R.status = S.status;
    R.iters = S.iters;
    R.evals = S.evals;
    R.hvps = S.hvps;
    R.phi = -S.f;
    R.acc = S.acc;
    R.seconds_total = total;
    R.seconds_to_target = t_hit[p];
  }
  return PD_OK;
}
