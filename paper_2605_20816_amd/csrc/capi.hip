// capi.hip -- C ABI of libpd: context, argument checks, workspace planning and
// the launches of pd_features, pd_validate, pd_objective_grad and pd_assign.
#include "pd.h"
#include "pd_host.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

pd_status pd_fail(pd_ctx *c, pd_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

static bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

pd_status pd_check_problem(pd_ctx *ctx, const pd_problem &p, int idx) {
  char buf[256];
  if (p.height < 1 || p.width < 1) {
    snprintf(buf, sizeof buf, "map %d: height and width must be >= 1 (got %d x %d)", idx,
             p.height, p.width);
    return pd_fail(ctx, PD_ERR_INVALID_ARG, buf);
  }
  if ((long long)p.height * p.width > (1LL << 31) - 1) {
    snprintf(buf, sizeof buf, "map %d: more than 2^31-1 pixels", idx);
    return pd_fail(ctx, PD_ERR_INVALID_ARG, buf);
  }
  if (p.n_grains < 2) {
    snprintf(buf, sizeof buf, "map %d: n_grains must be >= 2 (got %d)", idx, p.n_grains);
    return pd_fail(ctx, PD_ERR_INVALID_ARG, buf);
  }
  if (p.n_grains > (1 << 20)) {
    snprintf(buf, sizeof buf, "map %d: n_grains above 2^20 is not supported", idx);
    return pd_fail(ctx, PD_ERR_UNSUPPORTED, buf);
  }
  if (p.degree < 1 || p.degree > PD_MAX_DEGREE) {
    snprintf(buf, sizeof buf, "map %d: degree must be in [1, %d] (got %d)", idx, PD_MAX_DEGREE,
             p.degree);
    return pd_fail(ctx, PD_ERR_INVALID_ARG, buf);
  }
  if (!finite_pos(p.eps)) {
    snprintf(buf, sizeof buf, "map %d: eps must be finite and > 0", idx);
    return pd_fail(ctx, PD_ERR_INVALID_ARG, buf);
  }
  if (p.labels == nullptr) {
    snprintf(buf, sizeof buf, "map %d: labels is NULL", idx);
    return pd_fail(ctx, PD_ERR_INVALID_ARG, buf);
  }
  return PD_OK;
}

pd_status pd_reserve(pd_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->ws_cap) return PD_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, std::string("hipDeviceSynchronize: ") + hipGetErrorString(e));
  if (ctx->ws) (void)hipFree(ctx->ws);
  ctx->ws = nullptr;
  ctx->ws_cap = 0;
  const size_t want = bytes + bytes / 4 + (1 << 20);
  e = hipMalloc((void **)&ctx->ws, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return pd_fail(ctx, PD_ERR_OOM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  ctx->ws_cap = want;
  return PD_OK;
}

// Tile of the gradient kernel: about `target_waves` waves per map, each over at
// least 64 pixels, as wide as the map allows (the per-row fold into the K
// moments is amortised over the tile width, and each tile reads its rows' row
// coefficients once: tiles narrower than the map read them once per column tile).
static void choose_tiles(int H, int W, int Npad, int target_waves, int &tr, int &tc) {
  const long long groups = Npad / PD_WAVE;
  long long px = (long long)H * W * groups / target_waves;
  if (px < 64) px = 64;
  tc = (int)std::min<long long>(std::min(W, 64 * PD_WAVE), px);  // at most 64 segments
  long long rows = px / tc;
  if (rows > H) rows = H;
  if (rows < 1) rows = 1;  // also for an empty row range (no tiles then)
  tr = (int)rows;
}

void pd_plan_layout(EvalPlan &P, Arena &L, const pd_problem *probs, int n, int prec,
                    const int32_t *rows) {
  P.n = n;
  P.prec = prec;
  P.maps.assign(n, MapDev{});
  P.reg.assign(n, MapRegions{});
  P.offA.assign(n + 1, 0);
  P.offB.assign(n + 1, 0);
  P.offP.assign(n + 1, 0);
  P.offR.assign(n + 1, 0);
  P.off16P.assign(n + 1, 0);
  P.off16A.assign(n + 1, 0);
  P.off16B.assign(n + 1, 0);
  P.off16R.assign(n + 1, 0);
  P.max_hw = 0;
  P.max_k = 0;
  int max_d = 1;
  for (int p = 0; p < n; ++p) max_d = std::max(max_d, probs[p].degree);
  const size_t tsz = prec == 0 ? 8 : 4;  // FP32 tables for the FP32 and BF16 paths
  for (int p = 0; p < n; ++p) {
    const pd_problem &q = probs[p];
    MapDev &M = P.maps[p];
    MapRegions &R = P.reg[p];
    M.H = q.height;
    M.W = q.width;
    M.N = q.n_grains;
    M.d = q.degree;
    M.K = (q.degree + 1) * (q.degree + 2) / 2;
    M.DP = q.degree + 1;
    M.Npad = (q.n_grains + PD_WAVE - 1) / PD_WAVE * PD_WAVE;
    M.segs = (q.width + PD_WAVE - 1) / PD_WAVE;
    M.row0 = rows ? rows[2 * p] : 0;
    M.rows = rows ? rows[2 * p + 1] - rows[2 * p] : q.height;
    M.eps = q.eps;
    M.grad_scale = 1.0 / (q.eps * (double)q.height * (double)q.width);
    M.grad_sign = 1.0;
    M.labels = q.labels;
    choose_tiles(M.rows, M.W, M.Npad, P.target_waves, M.tile_rows, M.tile_cols);
    M.tiles_r = (M.rows + M.tile_rows - 1) / M.tile_rows;
    M.tiles_c = (M.W + M.tile_cols - 1) / M.tile_cols;
    // row-segment items, padded to whole blocks so a block never spans two maps
    M.a_items = (M.rows * M.segs + PD_WAVES_PER_BLOCK - 1) / PD_WAVES_PER_BLOCK * PD_WAVES_PER_BLOCK;
    // gradient work list: super-tiles of 4 tiles (block-summed partials) for
    // degree <= 4, else one tile per partial (a property of the map alone, so a
    // map's result does not depend on its batch)
    M.st_size = q.degree <= 4 ? PD_WAVES_PER_BLOCK : 1;
    M.stiles = (M.tiles_r * M.tiles_c + M.st_size - 1) / M.st_size;
    M.b_items = (M.stiles * M.st_size * (M.Npad / PD_WAVE) + PD_WAVES_PER_BLOCK - 1) /
                PD_WAVES_PER_BLOCK * PD_WAVES_PER_BLOCK;
    M.r_items = (M.N * M.K + 15) / 16;  // gradient-reduction blocks of 16 outputs
    const long long n_px = (long long)M.rows * M.W;  // evaluated pixels
    const bool mf = prec == 2;
    // BF16 matrix-core path: 32-pixel tiles inside one row (ceil(W / 32) per
    // row); k16_lse blocks = row segments of 16 tiles; k16_grad waves = pixel
    // chunks x 64-grain groups
    const int tw = (M.W + 31) / 32;
    M.n32 = (int)((n_px + 31) / 32 * 32);
    M.tiles32 = M.rows * tw;
    M.a16_items = M.rows * ((tw + 15) / 16);
    M.ggroups = (M.Npad + 32 * PD_MF_GROUP_TILES - 1) / (32 * PD_MF_GROUP_TILES);
    {
      // about target_waves / 2 waves of k16_grad (4 grain groups per block), in
      // chunks of whole rows (its gradient partials are per row)
      long long ct = (long long)M.tiles32 * ((M.ggroups + 3) / 4 * 4) / std::max(1, P.target_waves / 2);
      long long cr = (ct + tw / 2) / tw;
      if (cr > M.rows) cr = M.rows;
      if (cr < 1) cr = 1;
      M.chunk_tiles = (int)cr * tw;
      M.chunks = (M.rows + (int)cr - 1) / (int)cr;  // 0 for no rows
    }
    M.b16_items = M.chunks * ((M.ggroups + 3) / 4);  // k16_grad blocks
    R.tx64 = L.take(sizeof(double) * M.W * M.DP);
    R.ty64 = L.take(sizeof(double) * M.H * M.DP);
    R.txT = L.take(tsz * M.W * M.DP);
    R.tyT = L.take(tsz * M.H * M.DP);
    R.thc = L.take(sizeof(double) * M.N * M.K);
    // FP64 row coefficients and log-sum-exp in both VALU modes
    // (the BF16 path needs the coefficients only for the certified arg-max of a fit)
    R.C = L.take(mf && !P.cert ? 0 : sizeof(double) * (size_t)M.rows * M.Npad * M.DP);
    R.lse = L.take(mf ? 0 : sizeof(double) * n_px);
    R.rpix = L.take(mf ? sizeof(float) * (size_t)M.n32 : tsz * n_px);
    R.part_l = L.take(sizeof(double) * std::max(M.a_items, 4 * M.a16_items));
    R.part_g = L.take(mf ? 0 : sizeof(double) * (size_t)M.stiles * M.Npad * M.K);
    R.part_d = L.take(mf || !P.with_diag ? 0 : sizeof(double) * (size_t)M.stiles * M.Npad * M.K);
    R.part_c = L.take(sizeof(int64_t) * (mf ? std::max(M.a_items, 4 * M.a16_items) : M.a_items));
    const bool cert = P.cert;
    R.cert = L.take(cert ? 32 : 0);  // bound (8), uncertain count (4), canonical count (8)
    R.unc_list = L.take(cert ? sizeof(int32_t) * n_px : 0);
    R.btile = L.take(cert && mf ? sizeof(float) * (size_t)(M.Npad / 32) : 0);
    R.onehot = L.take(mf ? 0 : sizeof(double) * (size_t)M.N * M.K);
    M.mask_words = (M.Npad / PD_WAVE + 31) / 32;  // far-field mask: at most 4 words
    R.nearmask_on = !mf && M.mask_words <= 4;
    R.nearmask = L.take(R.nearmask_on ? sizeof(uint32_t) * (size_t)M.rows * M.segs * M.mask_words : 0);
    R.sorted = P.sort && M.N <= PD_ORDER_MAX;
    R.order = L.take(R.sorted ? sizeof(int32_t) * M.N : 0);
    R.pos = L.take(R.sorted ? sizeof(int32_t) * M.N : 0);
    R.order_sums = L.take(R.sorted ? 3 * sizeof(int64_t) * M.N : 0);
    R.T3 = L.take(mf ? 3 * 8 * sizeof(uint16_t) * (size_t)M.rows * M.Npad : 0);
    R.lse32 = L.take(mf ? sizeof(float) * M.n32 : 0);
    R.part_g32 = L.take(mf ? sizeof(float) * 8 * (size_t)M.rows * M.Npad : 0);
    P.offA[p + 1] = P.offA[p] + M.a_items;
    P.offB[p + 1] = P.offB[p] + M.b_items;
    P.offP[p + 1] = P.offP[p] + (int)(((long long)M.rows * M.Npad + PD_BLOCK - 1) / PD_BLOCK);
    P.offR[p + 1] = P.offR[p] + M.r_items;
    P.off16P[p + 1] = P.off16P[p] + (int)(((long long)M.rows * M.Npad + PD_BLOCK - 1) / PD_BLOCK);
    P.off16A[p + 1] = P.off16A[p] + M.a16_items;
    P.off16B[p + 1] = P.off16B[p] + M.b16_items;
    P.off16R[p + 1] = P.off16R[p] + (M.N + 7) / 8;
    M.a_off = P.offA[p];
    M.b_off = P.offB[p];
    M.r_off = P.offR[p];
    P.max_hw = std::max(P.max_hw, std::max(M.H, M.W));
    P.max_k = std::max(P.max_k, M.K);
    P.max_px = std::max(P.max_px, (long long)M.H * M.W);
    P.max_n = std::max(P.max_n, M.N);
  }
  P.dmax = pd_dmax_bucket(max_d);
  P.o_maps = L.take(sizeof(MapDev) * n);
  P.o_off = L.take(sizeof(int32_t) * 8 * (n + 1));
}

void pd_plan_bind(EvalPlan &P, char *base, const double *const *theta, double *phi_out,
                  double *const *grad_out, int32_t *const *labels_out, int64_t *n_correct) {
  P.any_grad = false;
  for (int p = 0; p < P.n; ++p) {
    MapDev &M = P.maps[p];
    const MapRegions &R = P.reg[p];
    M.tx64 = (double *)(base + R.tx64);
    M.ty64 = (double *)(base + R.ty64);
    M.txT = base + R.txT;
    M.tyT = base + R.tyT;
    M.T3 = base + R.T3;
    M.lse32 = (float *)(base + R.lse32);
    M.part_g32 = (float *)(base + R.part_g32);
    M.thc = (double *)(base + R.thc);
    M.C = base + R.C;
    M.lse = base + R.lse;
    M.rpix = base + R.rpix;
    M.part_l = (double *)(base + R.part_l);
    M.part_g = (double *)(base + R.part_g);
    M.part_c = (int64_t *)(base + R.part_c);
    if (P.cert) {
      M.cert = (double *)(base + R.cert);
      M.unc_count = (int32_t *)(base + R.cert + 8);
      M.fb_count = (int64_t *)(base + R.cert + 16);
      M.unc_list = (int32_t *)(base + R.unc_list);
      M.btile = (float *)(base + R.btile);
    } else {
      M.cert = nullptr;
      M.unc_count = nullptr;
      M.fb_count = nullptr;
      M.unc_list = nullptr;
      M.btile = nullptr;
    }
    M.onehot = P.onehot_pre && P.prec != 2 ? (double *)(base + R.onehot) : nullptr;
    M.order = R.sorted ? (const int32_t *)(base + R.order) : nullptr;
    M.pos = R.sorted ? (const int32_t *)(base + R.pos) : nullptr;
    M.order_sums = R.sorted ? (void *)(base + R.order_sums) : nullptr;
    // the far-field mask comes from the objective kernel (not from the fused
    // certified objective of FP32 fits above degree 4, nor from the BF16 kernels)
    M.nearmask = R.nearmask_on ? (uint32_t *)(base + R.nearmask) : nullptr;
    M.part_d = P.with_diag ? (double *)(base + R.part_d) : nullptr;
    M.diag = nullptr;
    M.want_diag = nullptr;
    M.theta = theta ? theta[p] : nullptr;
    M.phi = phi_out ? phi_out + p : nullptr;
    M.grad = grad_out ? grad_out[p] : nullptr;
    M.labels_out = labels_out ? labels_out[p] : nullptr;
    M.n_correct = n_correct ? n_correct + p : nullptr;
    if (M.grad) P.any_grad = true;
  }
  P.d_maps = (MapDev *)(base + P.o_maps);
  int32_t *off = (int32_t *)(base + P.o_off);
  P.d_offA = off;
  P.d_offB = off + (P.n + 1);
  P.d_offP = off + 2 * (P.n + 1);
  P.d_offR = off + 3 * (P.n + 1);
  P.d_off16P = off + 4 * (P.n + 1);
  P.d_off16A = off + 5 * (P.n + 1);
  P.d_off16B = off + 6 * (P.n + 1);
  P.d_off16R = off + 7 * (P.n + 1);
}

// A pinned staging buffer of at least `bytes` from the context's ring; the host
// waits only if the copy that last used this slot (PD_STAGE_SLOTS uploads ago)
// is still queued.
hipError_t pd_stage_acquire(pd_ctx *ctx, size_t bytes, char **buf, int *slot_out) {
  hipError_t e;
  const int slot = ctx->stage_next;
  ctx->stage_next = (slot + 1) % PD_STAGE_SLOTS;
  if (ctx->staged[slot]) {
    e = hipEventSynchronize(ctx->staged[slot]);
    if (e != hipSuccess) return e;
  } else {
    e = hipEventCreateWithFlags(&ctx->staged[slot], hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  if (bytes > ctx->stage_cap[slot]) {
    if (ctx->stage[slot]) (void)hipHostFree(ctx->stage[slot]);
    ctx->stage[slot] = nullptr;
    ctx->stage_cap[slot] = 0;
    e = hipHostMalloc((void **)&ctx->stage[slot], bytes * 2, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    ctx->stage_cap[slot] = bytes * 2;
  }
  *buf = ctx->stage[slot];
  *slot_out = slot;
  return hipSuccess;
}

// The stream-ordered copy out of a slot filled after pd_stage_acquire.
hipError_t pd_stage_copy(pd_ctx *ctx, int slot, void *dst, size_t bytes, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(dst, ctx->stage[slot], bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipEventRecord(ctx->staged[slot], s);
}

hipError_t pd_plan_upload(pd_ctx *ctx, EvalPlan &P, hipStream_t s) {
  // maps and the four offset arrays are contiguous in the arena (o_maps, o_off)
  const size_t maps_bytes = sizeof(MapDev) * P.n;
  const size_t gap = P.o_off - P.o_maps;
  const size_t total = gap + sizeof(int32_t) * 8 * (P.n + 1);
  char *stage;
  int slot;
  hipError_t e = pd_stage_acquire(ctx, total, &stage, &slot);
  if (e != hipSuccess) return e;
  memcpy(stage, P.maps.data(), maps_bytes);
  int32_t *o = (int32_t *)(stage + gap);
  for (int k = 0; k <= P.n; ++k) {
    o[k] = P.offA[k];
    o[(P.n + 1) + k] = P.offB[k];
    o[2 * (P.n + 1) + k] = P.offP[k];
    o[3 * (P.n + 1) + k] = P.offR[k];
    o[4 * (P.n + 1) + k] = P.off16P[k];
    o[5 * (P.n + 1) + k] = P.off16A[k];
    o[6 * (P.n + 1) + k] = P.off16B[k];
    o[7 * (P.n + 1) + k] = P.off16R[k];
  }
  return pd_stage_copy(ctx, slot, P.d_maps, total, s);
}

void pd_plan_tables(const EvalPlan &P, hipStream_t s) {
  pd_launch_tables(P.prec, P.d_maps, P.n, P.max_hw, s);
  if (P.sort) pd_launch_order(P.d_maps, P.n, P.max_px, P.max_n, s);
}

void pd_plan_onehot(const EvalPlan &P, hipStream_t s) {
  if (P.prec == 2 || !P.onehot_pre) return;
  pd_launch_onehot(P.dmax, P.d_maps, P.d_offB, P.n, P.offB[P.n], P.d_offR, P.offR[P.n], s);
}

void pd_plan_eval(const EvalPlan &P, bool with_grad, hipStream_t s, bool center,
                  const MapDev *assign_maps) {
  if (center) pd_launch_center(P.d_maps, P.n, P.max_k, s);
  pd_launch_prep(P.prec, P.d_maps, P.d_offP, P.n, P.offP[P.n], s);
  if (P.cert && P.prec != 2) {
    pd_launch_lse_cert(P.prec, P.dmax, P.d_maps, P.d_offA, P.n, P.offA[P.n], s);
    pd_launch_assign_list(P.dmax, P.d_maps, P.n, s);
  } else if (assign_maps) {
    pd_launch_lse_assign(P.prec, P.dmax, P.d_maps, P.d_offA, P.n, P.offA[P.n], assign_maps, s);
  } else {
    pd_launch_lse(P.prec, P.dmax, P.d_maps, P.d_offA, P.n, P.offA[P.n], s);
  }
  if (with_grad)
    pd_launch_grad(P.prec, P.dmax, P.d_maps, P.d_offB, P.n, P.offB[P.n], P.with_diag, !P.onehot_pre, s);
  pd_launch_reduce(P.d_maps, P.d_offR, P.n, P.offR[P.n], with_grad, with_grad && P.with_diag, s);
}

void pd_plan_assign(const EvalPlan &P, hipStream_t s) {
  pd_launch_assign(P.dmax, P.d_maps, P.d_offA, P.n, P.offA[P.n], true, s);
}

static std::tuple<int, int, int, int> tune_key(const pd_problem *probs, int n, int prec) {
  int dmax = 1;
  double pairs = 0.0;
  for (int p = 0; p < n; ++p) {
    dmax = std::max(dmax, probs[p].degree);
    pairs += (double)probs[p].height * probs[p].width * probs[p].n_grains;
  }
  const int lg = (int)floor(log2(std::max(pairs, 1.0)));
  const int nb = n <= 1 ? 1 : (n <= 8 ? 8 : 64);
  return std::make_tuple(prec, pd_dmax_bucket(dmax), lg, nb);
}

static void tune_load(pd_ctx *ctx) {
  if (ctx->tune_loaded) return;
  ctx->tune_loaded = true;
  const char *path = getenv("PD_AUTOTUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  int a, b, c2, d, w;
  while (fscanf(f, "%d %d %d %d %d", &a, &b, &c2, &d, &w) == 5) ctx->tuned[std::make_tuple(a, b, c2, d)] = w;
  fclose(f);
}

// Untuned work decomposition: about 2^18 pixel-grain pairs per gradient wave,
// from 8192 to 65536 waves.  Large maps need the finer split: the gradient
// kernel holds about four waves per SIMD, and with only two or three rounds of
// long waves the last round leaves most of the chip idle (at 2048^2 x 4895
// grains, 8192 waves took 21.2 ms and 65536 waves 17.5 ms per FP64 gradient;
// at a fitted iterate, where far-field skipping makes the waves uneven, 7.9
// against 4.4 ms).
static int default_waves(const pd_problem *probs, int n) {
  double pairs = 0.0;
  for (int p = 0; p < n; ++p) pairs += (double)probs[p].height * probs[p].width * probs[p].n_grains;
  int w = 8192;
  while (w < 65536 && pairs / w > 262144.0) w *= 2;
  return w;
}

int pd_tuned_waves(pd_ctx *ctx, const pd_problem *probs, int n, int prec) {
  tune_load(ctx);
  auto it = ctx->tuned.find(tune_key(probs, n, prec));
  if (it != ctx->tuned.end()) return it->second;
  return default_waves(probs, n);
}

#define PD_HIP(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return pd_fail(ctx, PD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

static pd_status precision_code(pd_ctx *ctx, pd_precision prec, int &code) {
  if (prec == PD_FP64) code = 0;
  else if (prec == PD_FP32) code = 1;
  else if (prec == PD_BF16) code = 2;
  else return pd_fail(ctx, PD_ERR_INVALID_ARG, "unknown precision");
  return PD_OK;
}

pd_status pd_plan_place(pd_ctx *ctx, EvalPlan &P, const Arena &L, const PlanMemory &mem,
                        const double *const *theta, double *phi_out, double *const *grad_out,
                        hipStream_t s) {
  char *base = mem.base;
  if (base == nullptr) {
    pd_status st = pd_reserve(ctx, L.off);
    if (st != PD_OK) return st;
    base = ctx->ws;
  } else if (L.off > mem.cap) {
    return pd_fail(ctx, PD_ERR_UNSUPPORTED,
                   "this evaluation needs " + std::to_string(L.off) +
                       " bytes of scratch; the fixed buffer holds " + std::to_string(mem.cap));
  }
  pd_plan_bind(P, base, theta, phi_out, grad_out, nullptr, nullptr);
  const hipError_t e = mem.base ? pd_plan_upload_by_kernel(P, s) : pd_plan_upload(ctx, P, s);
  if (e != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, std::string("plan upload: ") + hipGetErrorString(e));
  return PD_OK;
}

pd_status pd_objective_grad_impl(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                                 const int32_t *rows, const double *const *theta,
                                 double *phi_out, double *const *grad_out, pd_precision prec,
                                 int32_t flags, void *stream, const PlanMemory &mem) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  int code = 0;
  if (precision_code(ctx, prec, code) != PD_OK) return PD_ERR_INVALID_ARG;
  if (!probs || n_probs < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 maps");
  if (!theta) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta is NULL");
  if (!phi_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "phi_out is NULL");
  if (flags & ~PD_EVAL_ONEHOT_PRECOMPUTED) return pd_fail(ctx, PD_ERR_INVALID_ARG, "unknown flags");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pd_check_problem(ctx, probs[p], p);
    if (st != PD_OK) return st;
    if (!theta[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta[" + std::to_string(p) + "] is NULL");
    if (rows && !(0 <= rows[2 * p] && rows[2 * p] <= rows[2 * p + 1] && rows[2 * p + 1] <= probs[p].height))
      return pd_fail(ctx, PD_ERR_INVALID_ARG,
                     "map " + std::to_string(p) + ": rows must satisfy 0 <= begin <= end <= height");
  }
  PD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (code == 2)
    return pd_bf16_objective_grad(ctx, probs, n_probs, rows, theta, phi_out, grad_out, s, mem);
  EvalPlan P;
  Arena L;
  P.target_waves = pd_tuned_waves(ctx, probs, n_probs, code);
  P.onehot_pre = (flags & PD_EVAL_ONEHOT_PRECOMPUTED) != 0;
  P.sort = P.onehot_pre;
  pd_plan_layout(P, L, probs, n_probs, code, rows);
  pd_status st = pd_plan_place(ctx, P, L, mem, theta, phi_out, grad_out, s);
  if (st != PD_OK) return st;
  pd_plan_tables(P, s);
  if (P.any_grad) pd_plan_onehot(P, s);
  pd_plan_eval(P, P.any_grad, s, true);
  PD_HIP(ctx, hipGetLastError());
  return PD_OK;
}

extern "C" {

pd_status pd_create(int device, pd_ctx **out) {
  if (out == nullptr) return PD_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    (void)hipGetLastError();
    return PD_ERR_HIP;
  }
  if (device < 0 || device >= count) return PD_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return PD_ERR_HIP;
  pd_ctx *c = new pd_ctx();
  c->device = device;
  const pd_status st = pd_noalloc_setup(c);
  if (st != PD_OK) {
    delete c;
    return st;
  }
  *out = c;
  return PD_OK;
}

void pd_destroy(pd_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->aux) (void)hipFree(ctx->aux);
  for (int k = 0; k < PD_STAGE_SLOTS; ++k) {
    if (ctx->staged[k]) (void)hipEventSynchronize(ctx->staged[k]);
    if (ctx->stage[k]) (void)hipHostFree(ctx->stage[k]);
    if (ctx->staged[k]) (void)hipEventDestroy(ctx->staged[k]);
  }
  pd_fit_release(ctx);
  delete ctx;
}

const char *pd_last_error(const pd_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t pd_num_features(int32_t degree) {
  if (degree < 0 || degree > PD_MAX_DEGREE) return 0;
  return (degree + 1) * (degree + 2) / 2;
}

pd_status pd_features(pd_ctx *ctx, int32_t height, int32_t width, int32_t degree,
                      pd_precision out_prec, void *out, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  int code = 0;
  if (precision_code(ctx, out_prec, code) != PD_OK) return PD_ERR_INVALID_ARG;
  if (out == nullptr) return pd_fail(ctx, PD_ERR_INVALID_ARG, "out is NULL");
  pd_problem q{height, width, (const int32_t *)out, 2, degree, 1.0};
  pd_status st = pd_check_problem(ctx, q, 0);
  if (st != PD_OK) return st;
  PD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  EvalPlan P;
  Arena L;
  pd_plan_layout(P, L, &q, 1, 0);
  st = pd_reserve(ctx, L.off);
  if (st != PD_OK) return st;
  pd_plan_bind(P, ctx->ws, nullptr, nullptr, nullptr, nullptr, nullptr);
  PD_HIP(ctx, pd_plan_upload(ctx, P, s));
  pd_plan_tables(P, s);
  pd_launch_features_out(P.d_maps, code, out, (long long)height * width, s);
  PD_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_validate(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!probs || n_probs < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 maps");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pd_check_problem(ctx, probs[p], p);
    if (st != PD_OK) return st;
  }
  PD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  EvalPlan P;
  Arena L;
  pd_plan_layout(P, L, probs, n_probs, 0);
  const size_t o_bad = L.take(sizeof(int32_t) * n_probs);
  pd_status st = pd_reserve(ctx, L.off);
  if (st != PD_OK) return st;
  pd_plan_bind(P, ctx->ws, nullptr, nullptr, nullptr, nullptr, nullptr);
  int32_t *bad = (int32_t *)(ctx->ws + o_bad);
  PD_HIP(ctx, pd_plan_upload(ctx, P, s));
  PD_HIP(ctx, hipMemsetAsync(bad, 0, sizeof(int32_t) * n_probs, s));
  pd_launch_validate(P.d_maps, n_probs, bad, s);
  PD_HIP(ctx, hipGetLastError());
  std::vector<int32_t> hb(n_probs);
  PD_HIP(ctx, hipMemcpyAsync(hb.data(), bad, sizeof(int32_t) * n_probs, hipMemcpyDeviceToHost, s));
  PD_HIP(ctx, hipStreamSynchronize(s));
  for (int p = 0; p < n_probs; ++p)
    if (hb[p])
      return pd_fail(ctx, PD_ERR_INVALID_ARG,
                     "map " + std::to_string(p) + ": a label lies outside [0, n_grains)");
  return PD_OK;
}

pd_status pd_objective_grad(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                            const double *const *theta, double *phi_out,
                            double *const *grad_out, pd_precision prec, void *stream) {
  return pd_objective_grad_impl(ctx, probs, n_probs, nullptr, theta, phi_out, grad_out, prec, 0,
                                stream, PlanMemory{});
}

pd_status pd_objective_grad_rows(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                                 const int32_t *rows, const double *const *theta,
                                 double *phi_out, double *const *grad_out, pd_precision prec,
                                 int32_t flags, void *stream) {
  if (ctx && !rows) return pd_fail(ctx, PD_ERR_INVALID_ARG, "rows is NULL");
  return pd_objective_grad_impl(ctx, probs, n_probs, rows, theta, phi_out, grad_out, prec, flags,
                                stream, PlanMemory{});
}

pd_status pd_hessian_diag(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                          const double *const *theta, double *const *diag_out,
                          pd_precision prec, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  int code = 0;
  if (precision_code(ctx, prec, code) != PD_OK) return PD_ERR_INVALID_ARG;
  if (code == 2) return pd_fail(ctx, PD_ERR_UNSUPPORTED, "pd_hessian_diag: PD_FP64 or PD_FP32");
  if (!probs || n_probs < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 maps");
  if (!theta || !diag_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta and diag_out must be non-NULL");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pd_check_problem(ctx, probs[p], p);
    if (st != PD_OK) return st;
    if (!theta[p] || !diag_out[p])
      return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta / diag_out entry " + std::to_string(p) + " is NULL");
  }
  PD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  EvalPlan P;
  Arena L;
  P.with_diag = true;
  P.target_waves = pd_tuned_waves(ctx, probs, n_probs, code);
  pd_plan_layout(P, L, probs, n_probs, code);
  std::vector<size_t> o_g(n_probs);
  for (int p = 0; p < n_probs; ++p) o_g[p] = L.take(sizeof(double) * P.maps[p].N * P.maps[p].K);
  const size_t o_phi = L.take(sizeof(double) * n_probs);
  const size_t o_flag = L.take(sizeof(int32_t));
  pd_status st = pd_reserve(ctx, L.off);
  if (st != PD_OK) return st;
  std::vector<double *> g(n_probs);
  for (int p = 0; p < n_probs; ++p) g[p] = (double *)(ctx->ws + o_g[p]);
  pd_plan_bind(P, ctx->ws, theta, (double *)(ctx->ws + o_phi), g.data(), nullptr, nullptr);
  int32_t *flag = (int32_t *)(ctx->ws + o_flag);
  for (int p = 0; p < n_probs; ++p) {
    P.maps[p].diag = diag_out[p];
    P.maps[p].want_diag = flag;
  }
  PD_HIP(ctx, hipMemsetD32Async((hipDeviceptr_t)flag, 1, 1, s));
  PD_HIP(ctx, pd_plan_upload(ctx, P, s));
  pd_plan_tables(P, s);
  pd_plan_eval(P, true, s, true);
  PD_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_hessian_vec(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                         const double *const *theta, const double *const *v,
                         double *const *hv_out, pd_precision prec, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  int code = 0;
  if (precision_code(ctx, prec, code) != PD_OK) return PD_ERR_INVALID_ARG;
  if (code == 2) return pd_fail(ctx, PD_ERR_UNSUPPORTED, "pd_hessian_vec: PD_FP64 or PD_FP32");
  if (!probs || n_probs < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 maps");
  if (!theta || !v || !hv_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta, v and hv_out must be non-NULL");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pd_check_problem(ctx, probs[p], p);
    if (st != PD_OK) return st;
    if (!theta[p] || !v[p] || !hv_out[p])
      return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta / v / hv_out entry " + std::to_string(p) + " is NULL");
  }
  PD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  EvalPlan P;
  Arena L;
  P.target_waves = pd_tuned_waves(ctx, probs, n_probs, code);
  pd_plan_layout(P, L, probs, n_probs, code);
  std::vector<size_t> o_cv(n_probs), o_ub(n_probs);
  for (int p = 0; p < n_probs; ++p) {
    const MapDev &M = P.maps[p];
    o_cv[p] = L.take(sizeof(double) * (size_t)M.rows * M.Npad * M.DP);
    o_ub[p] = L.take(sizeof(double) * (size_t)M.rows * M.W);
  }
  const size_t o_phi = L.take(sizeof(double) * n_probs);
  pd_status st = pd_reserve(ctx, L.off);
  if (st != PD_OK) return st;
  pd_plan_bind(P, ctx->ws, theta, (double *)(ctx->ws + o_phi), hv_out, nullptr, nullptr);
  for (int p = 0; p < n_probs; ++p) {
    MapDev &M = P.maps[p];
    M.hv_in = v[p];
    M.Cv = ctx->ws + o_cv[p];
    M.ubar = (double *)(ctx->ws + o_ub[p]);
    M.onehot = nullptr;
    // the reduction writes scale * sum_x p_i (u_i - ubar) psi: 1 / (eps^2 n)
    M.grad_scale = 1.0 / (M.eps * M.eps * (double)M.H * (double)M.W);
    M.grad_sign = 1.0;
  }
  PD_HIP(ctx, pd_plan_upload(ctx, P, s));
  pd_plan_tables(P, s);
  pd_launch_center(P.d_maps, P.n, P.max_k, s);
  pd_launch_prep(P.prec, P.d_maps, P.d_offP, P.n, P.offP[P.n], s);
  pd_launch_lse(P.prec, P.dmax, P.d_maps, P.d_offA, P.n, P.offA[P.n], s);
  pd_launch_hvp(P.prec, P.dmax, P.d_maps, P.d_offP, P.d_offA, P.d_offB, P.n, P.offP[P.n],
                P.offA[P.n], P.offB[P.n], s);
  pd_launch_reduce(P.d_maps, P.d_offR, P.n, P.offR[P.n], true, false, s);
  PD_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_assign(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                    const double *const *theta, int32_t *const *labels_out,
                    int64_t *n_correct_out, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!probs || n_probs < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 maps");
  if (!theta) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta is NULL");
  if (!n_correct_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "n_correct_out is NULL");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pd_check_problem(ctx, probs[p], p);
    if (st != PD_OK) return st;
    if (!theta[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta[" + std::to_string(p) + "] is NULL");
  }
  PD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  EvalPlan P;
  Arena L;
  pd_plan_layout(P, L, probs, n_probs, 0);
  pd_status st = pd_reserve(ctx, L.off);
  if (st != PD_OK) return st;
  pd_plan_bind(P, ctx->ws, theta, nullptr, nullptr, labels_out, n_correct_out);
  PD_HIP(ctx, pd_plan_upload(ctx, P, s));
  pd_plan_tables(P, s);
  pd_plan_assign(P, s);
  PD_HIP(ctx, hipGetLastError());
  return PD_OK;
}

pd_status pd_profile_eval(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                          const double *const *theta, pd_precision prec, int32_t reps,
                          double *ms_out, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  int code = 0;
  if (precision_code(ctx, prec, code) != PD_OK) return PD_ERR_INVALID_ARG;
  if (!probs || n_probs < 1 || !theta || !ms_out || reps < 1)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "pd_profile_eval: bad arguments");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pd_check_problem(ctx, probs[p], p);
    if (st != PD_OK) return st;
    if (!theta[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta entry is NULL");
  }
  PD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  EvalPlan P;
  Arena L;
  P.onehot_pre = true;  // as in a fit
  P.sort = true;
  // the FP64/FP32 objective stage times the certified kernel a fit runs
  P.cert = code != 2;
  P.target_waves = pd_tuned_waves(ctx, probs, n_probs, code);
  pd_plan_layout(P, L, probs, n_probs, code);
  const size_t o_phi = L.take(sizeof(double) * n_probs);
  std::vector<size_t> o_g(n_probs);
  for (int p = 0; p < n_probs; ++p)
    o_g[p] = L.take(sizeof(double) * (size_t)P.maps[p].N * P.maps[p].K);
  pd_status st = pd_reserve(ctx, L.off);
  if (st != PD_OK) return st;
  std::vector<double *> g(n_probs);
  for (int p = 0; p < n_probs; ++p) g[p] = (double *)(ctx->ws + o_g[p]);
  pd_plan_bind(P, ctx->ws, theta, (double *)(ctx->ws + o_phi), g.data(), nullptr, nullptr);
  PD_HIP(ctx, pd_plan_upload(ctx, P, s));
  // certificate slots (bound, uncertain count, canonical count) start at zero;
  // the timed repetitions below add to them, and nothing reads them after
  if (P.cert)
    for (int p = 0; p < n_probs; ++p) PD_HIP(ctx, hipMemsetAsync(P.maps[p].cert, 0, 32, s));
  hipEvent_t ev[PD_NUM_STAGES + 1];
  for (auto &e : ev) PD_HIP(ctx, hipEventCreate(&e));
  // one untimed evaluation first (loads the kernels' code on first use)
  pd_plan_tables(P, s);
  pd_plan_onehot(P, s);
  if (code == 2) pd_bf16_plan_eval(ctx, P, s, true);
  else pd_plan_eval(P, true, s, true);
  PD_HIP(ctx, hipEventRecord(ev[0], s));
  // the tables stage includes the per-plan indicator moments
  for (int r = 0; r < reps; ++r) {
    pd_plan_tables(P, s);
    pd_plan_onehot(P, s);
  }
  PD_HIP(ctx, hipEventRecord(ev[1], s));
  for (int r = 0; r < reps; ++r) pd_launch_center(P.d_maps, P.n, P.max_k, s);
  PD_HIP(ctx, hipEventRecord(ev[2], s));
  if (code == 2) {
    for (int p = 0; p < n_probs; ++p)
      if (probs[p].degree > 6) return pd_fail(ctx, PD_ERR_UNSUPPORTED, "PD_BF16 supports degree <= 6");
    pd_bf16_profile_stages(ctx, P, reps, s, ev + 2);
  } else {
    for (int r = 0; r < reps; ++r) pd_launch_prep(P.prec, P.d_maps, P.d_offP, P.n, P.offP[P.n], s);
    PD_HIP(ctx, hipEventRecord(ev[3], s));
    for (int r = 0; r < reps; ++r)
      pd_launch_lse_cert(P.prec, P.dmax, P.d_maps, P.d_offA, P.n, P.offA[P.n], s);
    PD_HIP(ctx, hipEventRecord(ev[4], s));
    for (int r = 0; r < reps; ++r)
      pd_launch_grad(P.prec, P.dmax, P.d_maps, P.d_offB, P.n, P.offB[P.n], false, !P.onehot_pre, s);
    PD_HIP(ctx, hipEventRecord(ev[5], s));
  }
  for (int r = 0; r < reps; ++r) {
    if (code == 2) pd_bf16_launch(P, 3, s);
    else pd_launch_reduce(P.d_maps, P.d_offR, P.n, P.offR[P.n], true, false, s);
  }
  PD_HIP(ctx, hipEventRecord(ev[6], s));
  PD_HIP(ctx, hipGetLastError());
  PD_HIP(ctx, hipEventSynchronize(ev[6]));
  for (int k = 0; k < PD_NUM_STAGES; ++k) {
    float ms = 0.f;
    PD_HIP(ctx, hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
    ms_out[k] = (double)ms / reps;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  return PD_OK;
}

pd_status pd_autotune(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                      const double *const *theta, pd_precision prec, int32_t *best_waves_out,
                      void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  int code = 0;
  if (precision_code(ctx, prec, code) != PD_OK) return PD_ERR_INVALID_ARG;
  if (!probs || n_probs < 1 || !theta) return pd_fail(ctx, PD_ERR_INVALID_ARG, "pd_autotune: bad arguments");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pd_check_problem(ctx, probs[p], p);
    if (st != PD_OK) return st;
    if (!theta[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta entry is NULL");
    if (code == 2 && probs[p].degree > 6)
      return pd_fail(ctx, PD_ERR_UNSUPPORTED, "PD_BF16 supports degree <= 6");
  }
  PD_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  tune_load(ctx);
  // candidates timed over five evaluations each; the untuned default is kept
  // unless another is more than 2% faster, so timing noise does not flip the
  // tiling (and with it the rounding of the gradient sums) from run to run
  static const int cand[] = {1024, 2048, 4096, 8192, 16384, 32768, 65536};
  const int kDefault = default_waves(probs, n_probs);
  float best_ms = 1e30f, default_ms = 1e30f;
  int best = kDefault;
  hipEvent_t e0, e1;
  PD_HIP(ctx, hipEventCreate(&e0));
  PD_HIP(ctx, hipEventCreate(&e1));
  for (int w : cand) {
    EvalPlan P;
    Arena L;
    P.onehot_pre = true;  // as in a fit
  P.sort = true;
    P.target_waves = w;
    pd_plan_layout(P, L, probs, n_probs, code);
    const size_t o_phi = L.take(sizeof(double) * n_probs);
    std::vector<size_t> o_g(n_probs);
    for (int p = 0; p < n_probs; ++p)
      o_g[p] = L.take(sizeof(double) * (size_t)P.maps[p].N * P.maps[p].K);
    pd_status st = pd_reserve(ctx, L.off);
    if (st != PD_OK) return st;
    std::vector<double *> g(n_probs);
    for (int p = 0; p < n_probs; ++p) g[p] = (double *)(ctx->ws + o_g[p]);
    pd_plan_bind(P, ctx->ws, theta, (double *)(ctx->ws + o_phi), g.data(), nullptr, nullptr);
    PD_HIP(ctx, pd_plan_upload(ctx, P, s));
    pd_plan_tables(P, s);
    pd_plan_onehot(P, s);
    auto run = [&]() {
      if (code == 2) pd_bf16_plan_eval(ctx, P, s, true);
      else pd_plan_eval(P, true, s, true);
    };
    run();  // warm-up
    PD_HIP(ctx, hipEventRecord(e0, s));
    for (int r = 0; r < 5; ++r) run();
    PD_HIP(ctx, hipEventRecord(e1, s));
    PD_HIP(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    PD_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
    if (w == kDefault) default_ms = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = w;
    }
  }
  if (default_ms <= 1.02f * best_ms) best = kDefault;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const auto key = tune_key(probs, n_probs, code);
  ctx->tuned[key] = best;
  if (const char *path = getenv("PD_AUTOTUNE_CACHE")) {
    if (FILE *f = fopen(path, "a")) {
      fprintf(f, "%d %d %d %d %d\n", std::get<0>(key), std::get<1>(key), std::get<2>(key),
              std::get<3>(key), best);
      fclose(f);
    }
  }
  if (best_waves_out) *best_waves_out = best;
  return PD_OK;
}

}  // extern "C"
