// warm_api.hip -- C ABI of the warm start: descriptors, moment seed, training
// targets, network forward / backward / Adam, and pd_warm_start (network or
// moment seed, then a scale search along the ray).
#include "pd.h"
#include "pd_host.h"
#include "pd_warm.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#define WARM_HIP(ctx, expr)                                                                \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return pd_fail(ctx, PD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

// scale of theta_hat applied per grain row: out = s * in
__global__ void kw_scale(const double *__restrict__ in, double s, size_t n, double *__restrict__ out) {
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (size_t)gridDim.x * blockDim.x)
    out[j] = s * in[j];
}

struct WarmLayout {
  std::vector<WarmDev> maps;
  std::vector<int32_t> off;  // grain offsets (pass 2 work list)
  size_t o_maps = 0, o_off = 0, end = 0;
  int max_n = 0, total = 0;
};

// Per-map scratch for descriptors; user buffers are bound afterwards.
void warm_layout(WarmLayout &W, Arena &L, const pd_problem *probs, int n) {
  W.maps.assign(n, WarmDev{});
  W.off.assign(n + 1, 0);
  for (int p = 0; p < n; ++p) {
    WarmDev &M = W.maps[p];
    M.H = probs[p].height;
    M.W = probs[p].width;
    M.N = probs[p].n_grains;
    M.d = probs[p].degree;
    M.K = (M.d + 1) * (M.d + 2) / 2;
    M.labels = probs[p].labels;
    W.off[p + 1] = W.off[p] + M.N;
    W.max_n = std::max(W.max_n, M.N);
  }
  W.total = W.off[n];
  W.o_maps = L.take(sizeof(WarmDev) * n);
  W.o_off = L.take(sizeof(int32_t) * (n + 1));
}

// pinned staging of a small host block, ordered on stream s
hipError_t upload(pd_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t s) {
  char *stage;
  int slot;
  hipError_t e = pd_stage_acquire(ctx, bytes, &stage, &slot);
  if (e != hipSuccess) return e;
  memcpy(stage, src, bytes);
  return pd_stage_copy(ctx, slot, dst, bytes, s);
}

hipError_t warm_upload(pd_ctx *ctx, WarmLayout &W, char *base, hipStream_t s) {
  const int n = (int)W.maps.size();
  std::vector<char> blob(W.o_off - W.o_maps + sizeof(int32_t) * (n + 1));
  memcpy(blob.data(), W.maps.data(), sizeof(WarmDev) * n);
  memcpy(blob.data() + (W.o_off - W.o_maps), W.off.data(), sizeof(int32_t) * (n + 1));
  return upload(ctx, base + W.o_maps, blob.data(), blob.size(), s);
}

pd_status check_maps(pd_ctx *ctx, const pd_problem *probs, int n) {
  if (!probs || n < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 maps");
  for (int p = 0; p < n; ++p) {
    pd_status st = pd_check_problem(ctx, probs[p], p);
    if (st != PD_OK) return st;
  }
  return PD_OK;
}

// Scale search state of one map (bracketing in u = log2 s, then golden section).
struct ScaleSearch {
  static constexpr double STEP = 2.0;
  static constexpr int BRACKET_MAX = 12;
  static constexpr int GOLDEN_ITERS = 6;
  double u0 = 0.0;
  int phase = 0;  // 0: f(a); 1: f(b); 2: bracketing; 3: golden first x1; 4: golden x2; 5: golden; 6: done
  double a = 0, b = 0, fa = 0, fb = 0, step = 0, lo = 0, mid = 0, fmid = 0, hi = 0;
  int n_br = 0, n_gold = 0;
  double left = 0, right = 0, x1 = 0, x2 = 0, f1 = 0, f2 = 0;
  bool last_was_x1 = false;
  std::vector<std::pair<double, double>> seen;  // (u, f)
  double next = 0.0;                            // u to evaluate next

  static double val(double f) { return f == f ? f : -INFINITY; }
  void start(double s0) {
    u0 = log2(s0);
    a = u0;
    b = u0 + STEP;
    phase = 0;
    next = a;
  }
  void begin_golden() {
    left = std::min(lo, hi);
    right = std::max(lo, hi);
    x1 = right - GOLDEN * (right - left);
    x2 = left + GOLDEN * (right - left);
    phase = 3;
    next = x1;
  }
  static constexpr double GOLDEN = 0.6180339887498949;
  // feed f(next); sets `next` or phase 6
  void feed(double f) {
    f = val(f);
    seen.emplace_back(next, f);
    switch (phase) {
      case 0:
        fa = f;
        phase = 1;
        next = b;
        return;
      case 1:
        fb = f;
        if (fb >= fa) {
          step = STEP;
          lo = a;
          mid = b;
          fmid = fb;
        } else {
          step = -STEP;
          lo = b;
          mid = a;
          fmid = fa;
        }
        hi = mid + step;
        n_br = 0;
        phase = 2;
        next = hi;
        return;
      case 2:
        ++n_br;
        if (!(f > fmid) || n_br >= BRACKET_MAX) {
          if (f > fmid) {  // budget reached while still increasing
            lo = mid;
            mid = hi;
            fmid = f;
            hi = mid + step;
          }
          begin_golden();
          return;
        }
        lo = mid;
        mid = hi;
        fmid = f;
        hi = mid + step;
        next = hi;
        return;
      case 3:
        f1 = f;
        phase = 4;
        next = x2;
        return;
      case 4:
        f2 = f;
        n_gold = 2;
        break;
      case 5:
        if (last_was_x1) f1 = f;
        else f2 = f;
        ++n_gold;
        break;
      default:
        return;
    }
    if (n_gold >= GOLDEN_ITERS) {
      phase = 6;
      return;
    }
    phase = 5;
    if (f1 >= f2) {
      right = x2;
      x2 = x1;
      f2 = f1;
      x1 = right - GOLDEN * (right - left);
      last_was_x1 = true;
      next = x1;
    } else {
      left = x1;
      x1 = x2;
      f1 = f2;
      x2 = left + GOLDEN * (right - left);
      last_was_x1 = false;
      next = x2;
    }
  }
  // best evaluated point: largest f, ties to the point closest to u0
  std::pair<double, double> best() const {
    std::pair<double, double> bst = seen.front();
    for (const auto &q : seen)
      if (q.second > bst.second ||
          (q.second == bst.second && fabs(q.first - u0) < fabs(bst.first - u0)))
        bst = q;
    return bst;
  }
};

}  // namespace

// Context buffer for the warm-start scratch (separate from the evaluation
// workspace, which the scale search uses through pd_objective_grad).
static pd_status reserve_aux(pd_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->aux_cap) return PD_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, std::string("hipDeviceSynchronize: ") + hipGetErrorString(e));
  if (ctx->aux) (void)hipFree(ctx->aux);
  ctx->aux = nullptr;
  ctx->aux_cap = 0;
  const size_t want = bytes + bytes / 4 + (1 << 20);
  e = hipMalloc((void **)&ctx->aux, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return pd_fail(ctx, PD_ERR_OOM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  ctx->aux_cap = want;
  return PD_OK;
}

// Descriptor scratch of every map (isum, bbox, frame, desc) in the arena.
struct DescRegions {
  std::vector<size_t> isum, bbox, frame, desc, theta_h;
};

static void desc_regions(DescRegions &R, Arena &L, const WarmLayout &W, bool want_theta_h) {
  const int n = (int)W.maps.size();
  R.isum.resize(n);
  R.bbox.resize(n);
  R.frame.resize(n);
  R.desc.resize(n);
  R.theta_h.resize(n);
  for (int p = 0; p < n; ++p) {
    const WarmDev &M = W.maps[p];
    R.isum[p] = L.take(sizeof(long long) * 6 * M.N);
    R.bbox[p] = L.take(sizeof(int32_t) * 4 * M.N);
    R.frame[p] = L.take(sizeof(double) * PD_FRAME_DIM * M.N);
    R.desc[p] = L.take(sizeof(float) * PD_DESC_DIM * M.N);
    R.theta_h[p] = want_theta_h ? L.take(sizeof(double) * M.N * M.K) : 0;
  }
}

static void desc_bind(WarmLayout &W, const DescRegions &R, char *base) {
  for (size_t p = 0; p < W.maps.size(); ++p) {
    WarmDev &M = W.maps[p];
    M.isum = (long long *)(base + R.isum[p]);
    M.bbox = (int32_t *)(base + R.bbox[p]);
    M.frame = (double *)(base + R.frame[p]);
    M.desc = (float *)(base + R.desc[p]);
    M.theta_h = R.theta_h[p] ? (double *)(base + R.theta_h[p]) : nullptr;
  }
}

static void launch_desc(const WarmLayout &W, char *base, hipStream_t s) {
  const WarmDev *dW = (const WarmDev *)(base + W.o_maps);
  const int32_t *doff = (const int32_t *)(base + W.o_off);
  pd_warm_launch_desc(dW, doff, (int)W.maps.size(), W.total, W.max_n, s);
}

extern "C" {

int64_t pd_mlp_num_params(int32_t k_out) {
  if (k_out < 1) return 0;
  return (int64_t)pd_mlp_params(k_out);
}

pd_status pd_descriptors(pd_ctx *ctx, const pd_problem *probs, int32_t n, float *const *desc_out,
                         double *const *frame_out, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  pd_status st = check_maps(ctx, probs, n);
  if (st != PD_OK) return st;
  if (!desc_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "desc_out is NULL");
  for (int p = 0; p < n; ++p)
    if (!desc_out[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "desc_out entry is NULL");
  WARM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  WarmLayout W;
  Arena L;
  warm_layout(W, L, probs, n);
  DescRegions R;
  desc_regions(R, L, W, false);
  st = reserve_aux(ctx, L.off);
  if (st != PD_OK) return st;
  desc_bind(W, R, ctx->aux);
  for (int p = 0; p < n; ++p) {
    W.maps[p].desc = desc_out[p];
    if (frame_out && frame_out[p]) W.maps[p].frame = frame_out[p];
  }
  WARM_HIP(ctx, warm_upload(ctx, W, ctx->aux, s));
  launch_desc(W, ctx->aux, s);
  WARM_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_heuristic(pd_ctx *ctx, const pd_problem *probs, int32_t n, double *const *theta_out,
                       void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  pd_status st = check_maps(ctx, probs, n);
  if (st != PD_OK) return st;
  if (!theta_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_out is NULL");
  for (int p = 0; p < n; ++p)
    if (!theta_out[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_out entry is NULL");
  WARM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  WarmLayout W;
  Arena L;
  warm_layout(W, L, probs, n);
  DescRegions R;
  desc_regions(R, L, W, false);
  st = reserve_aux(ctx, L.off);
  if (st != PD_OK) return st;
  desc_bind(W, R, ctx->aux);
  for (int p = 0; p < n; ++p) W.maps[p].theta_h = theta_out[p];
  WARM_HIP(ctx, warm_upload(ctx, W, ctx->aux, s));
  launch_desc(W, ctx->aux, s);
  pd_warm_launch_heuristic((const WarmDev *)(ctx->aux + W.o_maps), n, s);
  WARM_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_warm_targets(pd_ctx *ctx, const pd_problem *probs, int32_t n,
                          const double *const *theta_fit, float *const *target_out,
                          double *lambda_out, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  pd_status st = check_maps(ctx, probs, n);
  if (st != PD_OK) return st;
  if (!theta_fit || !target_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_fit and target_out must be non-NULL");
  for (int p = 0; p < n; ++p)
    if (!theta_fit[p] || !target_out[p])
      return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_fit / target_out entry is NULL");
  WARM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  WarmLayout W;
  Arena L;
  warm_layout(W, L, probs, n);
  DescRegions R;
  desc_regions(R, L, W, false);
  st = reserve_aux(ctx, L.off);
  if (st != PD_OK) return st;
  desc_bind(W, R, ctx->aux);
  for (int p = 0; p < n; ++p) {
    W.maps[p].theta_fit = theta_fit[p];
    W.maps[p].target = target_out[p];
    W.maps[p].lambda = lambda_out ? lambda_out + p : nullptr;
  }
  WARM_HIP(ctx, warm_upload(ctx, W, ctx->aux, s));
  launch_desc(W, ctx->aux, s);
  const WarmDev *dW = (const WarmDev *)(ctx->aux + W.o_maps);
  pd_warm_launch_targets(dW, n, s);
  WARM_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_mlp_forward(pd_ctx *ctx, int32_t k_out, const float *params, const float *x,
                         int32_t batch, pd_precision prec, float *y_out, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (k_out < 1 || k_out > 4096) return pd_fail(ctx, PD_ERR_INVALID_ARG, "k_out must be in [1, 4096]");
  if (batch < 0) return pd_fail(ctx, PD_ERR_INVALID_ARG, "batch must be >= 0");
  if (!params || !x || !y_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "params, x and y_out must be non-NULL");
  if (prec != PD_FP32 && prec != PD_BF16)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "network precision must be PD_FP32 or PD_BF16");
  if (batch == 0) return PD_OK;
  WARM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (prec == PD_BF16) {
    pd_status st = reserve_aux(ctx, pd_mlp_bf16_ws(k_out, batch));
    if (st != PD_OK) return st;
    pd_mlp_launch_bf16(params, k_out, x, batch, ctx->aux, y_out, k_out, s);
  } else {
    const size_t act = (size_t)batch * PD_MLP_HID;
    pd_status st = reserve_aux(ctx, 4 * act * sizeof(float) + 1024);
    if (st != PD_OK) return st;
    float *z1 = (float *)ctx->aux, *h1 = z1 + act, *z2 = h1 + act, *h2 = z2 + act;
    pd_mlp_launch_forward(params, k_out, x, batch, z1, h1, z2, h2, y_out, s);
  }
  WARM_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_mlp_backward(pd_ctx *ctx, int32_t k_out, const float *params, const float *x,
                          const float *target, int32_t batch, double *loss_out, float *grad_out,
                          void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (k_out < 1 || k_out > 4096) return pd_fail(ctx, PD_ERR_INVALID_ARG, "k_out must be in [1, 4096]");
  if (batch < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "batch must be >= 1");
  if (!params || !x || !target || !loss_out || !grad_out)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "params, x, target, loss_out and grad_out must be non-NULL");
  WARM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  pd_status st = reserve_aux(ctx, pd_mlp_backward_ws(k_out, batch));
  if (st != PD_OK) return st;
  pd_mlp_launch_backward(params, k_out, x, target, batch, ctx->aux, loss_out, grad_out, s);
  WARM_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_mlp_adam(pd_ctx *ctx, int64_t n_params, float *params, const float *grad, float *m,
                      float *v, int32_t step, float lr, float beta1, float beta2, float eps,
                      void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (n_params < 0) return pd_fail(ctx, PD_ERR_INVALID_ARG, "n_params must be >= 0");
  if (!params || !grad || !m || !v) return pd_fail(ctx, PD_ERR_INVALID_ARG, "buffers must be non-NULL");
  if (step < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "step must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f && lr >= 0.f))
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "need 0 <= beta < 1, eps > 0, lr >= 0");
  if (n_params == 0) return PD_OK;
  WARM_HIP(ctx, hipSetDevice(ctx->device));
  pd_mlp_launch_adam(params, grad, m, v, (size_t)n_params, step, lr, beta1, beta2, eps,
                     (hipStream_t)stream);
  WARM_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_warm_start(pd_ctx *ctx, const pd_problem *probs, int32_t n, const pd_mlp *mlp,
                        double *const *theta_out, pd_precision prec, double *scale_out,
                        void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  pd_status st = check_maps(ctx, probs, n);
  if (st != PD_OK) return st;
  if (!theta_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_out is NULL");
  for (int p = 0; p < n; ++p)
    if (!theta_out[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta_out entry is NULL");
  if (prec != PD_FP64 && prec != PD_FP32 && prec != PD_BF16)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "unknown precision");
  st = pd_validate(ctx, probs, n, stream);
  if (st != PD_OK) return st;
  WARM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  // ---- layout: maps grouped by degree so each network runs once on one batch
  WarmLayout W;
  Arena L;
  warm_layout(W, L, probs, n);
  DescRegions R;
  desc_regions(R, L, W, true);
  std::vector<size_t> o_hat(n), o_out(n);
  std::vector<size_t> o_desc_deg(PD_MAX_DEGREE + 1, 0), o_y_deg(PD_MAX_DEGREE + 1, 0);
  std::vector<int> rows_deg(PD_MAX_DEGREE + 1, 0);
  std::vector<int> row0(n, 0);
  for (int p = 0; p < n; ++p) {
    const int d = W.maps[p].d;
    row0[p] = rows_deg[d];
    rows_deg[d] += W.maps[p].N;
  }
  size_t bf_ws = 0;
  for (int d = 1; d <= PD_MAX_DEGREE; ++d) {
    if (!rows_deg[d]) continue;
    const int K = (d + 1) * (d + 2) / 2;
    o_desc_deg[d] = L.take(sizeof(float) * PD_DESC_DIM * rows_deg[d]);
    o_y_deg[d] = L.take(sizeof(float) * K * rows_deg[d]);
    bf_ws = std::max(bf_ws, pd_mlp_bf16_ws(K, rows_deg[d]));
  }
  const size_t o_bf = L.take(bf_ws);
  for (int p = 0; p < n; ++p) {
    o_hat[p] = L.take(sizeof(double) * W.maps[p].N * W.maps[p].K);
    o_out[p] = L.take(sizeof(double) * W.maps[p].N * W.maps[p].K);
  }
  const size_t o_phi = L.take(sizeof(double) * n);
  st = reserve_aux(ctx, L.off);
  if (st != PD_OK) return st;
  char *base = ctx->aux;
  desc_bind(W, R, base);
  for (int p = 0; p < n; ++p) {
    WarmDev &M = W.maps[p];
    const int d = M.d;
    const bool net = mlp && mlp->params[d];
    M.desc = (float *)(base + o_desc_deg[d]) + (size_t)row0[p] * PD_DESC_DIM;
    M.mlp_out = net ? (float *)(base + o_y_deg[d]) + (size_t)row0[p] * M.K : nullptr;
    M.out_stride = M.K;
    M.theta_out = (double *)(base + o_hat[p]);
  }
  WARM_HIP(ctx, warm_upload(ctx, W, base, s));
  launch_desc(W, base, s);
  const WarmDev *dW = (const WarmDev *)(base + W.o_maps);
  pd_warm_launch_heuristic(dW, n, s);
  for (int d = 1; d <= PD_MAX_DEGREE; ++d) {
    if (!rows_deg[d] || !(mlp && mlp->params[d])) continue;
    const int K = (d + 1) * (d + 2) / 2;
    pd_mlp_launch_bf16(mlp->params[d], K, (const float *)(base + o_desc_deg[d]), rows_deg[d],
                       base + o_bf, (float *)(base + o_y_deg[d]), K, s);
  }
  pd_warm_launch_apply(dW, n, s);
  WARM_HIP(ctx, hipGetLastError());

  // ---- scale search, all maps advanced together (one evaluation per map per round)
  const pd_precision eprec = prec == PD_FP64 ? PD_FP64 : PD_FP32;
  std::vector<ScaleSearch> S(n);
  for (int p = 0; p < n; ++p) {
    const pd_problem &q = probs[p];
    S[p].start(q.eps * std::max(q.height, q.width) / (28.0 * sqrt((double)q.n_grains)));
  }
  double *phi_d = (double *)(base + o_phi);
  double *phi_h = nullptr;
  WARM_HIP(ctx, hipHostMalloc((void **)&phi_h, sizeof(double) * n, hipHostMallocDefault));
  std::vector<int> live;
  std::vector<pd_problem> sub_p;
  std::vector<const double *> sub_t;
  pd_status rs = PD_OK;
  for (int round = 0; round < 64; ++round) {
    live.clear();
    for (int p = 0; p < n; ++p)
      if (S[p].phase != 6) live.push_back(p);
    if (live.empty()) break;
    sub_p.clear();
    sub_t.clear();
    for (int p : live) {
      const size_t NK = (size_t)W.maps[p].N * W.maps[p].K;
      double *trial = (double *)(base + o_out[p]);
      kw_scale<<<(int)std::min<size_t>(256, (NK + 255) / 256), 256, 0, s>>>(
          (const double *)(base + o_hat[p]), pow(2.0, S[p].next), NK, trial);
      sub_p.push_back(probs[p]);
      sub_t.push_back(trial);
    }
    rs = pd_objective_grad(ctx, sub_p.data(), (int)live.size(), sub_t.data(), phi_d, nullptr,
                           eprec, stream);
    if (rs != PD_OK) break;
    hipError_t e = hipMemcpyAsync(phi_h, phi_d, sizeof(double) * live.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      rs = pd_fail(ctx, PD_ERR_HIP, std::string("scale search: ") + hipGetErrorString(e));
      break;
    }
    for (size_t k = 0; k < live.size(); ++k) S[live[k]].feed(phi_h[k]);
  }
  (void)hipHostFree(phi_h);
  if (rs != PD_OK) return rs;
  for (int p = 0; p < n; ++p) {
    const auto bst = S[p].best();
    const double phi0 = -log((double)probs[p].n_grains);
    const bool fallback = !(bst.second >= phi0);
    const double sc = fallback ? 0.0 : pow(2.0, bst.first);
    const size_t NK = (size_t)W.maps[p].N * W.maps[p].K;
    kw_scale<<<(int)std::min<size_t>(256, (NK + 255) / 256), 256, 0, s>>>(
        (const double *)(base + o_hat[p]), sc, NK, theta_out[p]);
    if (scale_out) scale_out[p] = sc;
  }
  WARM_HIP(ctx, hipGetLastError());
  WARM_HIP(ctx, hipStreamSynchronize(s));
  return PD_OK;
}

}  // extern "C"
