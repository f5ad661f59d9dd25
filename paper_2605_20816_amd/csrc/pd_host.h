// pd_host.h -- host-side planning structures of libpd (not part of the C ABI).
#pragma once

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "pd.h"
#include "pd_internal.h"

struct FitState;

#define PD_STAGE_SLOTS 4

struct pd_ctx {
  int device = 0;
  std::string err;
  char *ws = nullptr;     // evaluation workspace, grown on demand
  size_t ws_cap = 0;
  char *aux = nullptr;    // warm-start and network workspace, grown on demand
  size_t aux_cap = 0;
  FitState *fit = nullptr;
  // pinned staging of the map descriptors: a ring of PD_STAGE_SLOTS buffers, each
  // with the event of the last copy out of it, so that the host waits only when
  // that many uploads are still in flight
  char *stage[PD_STAGE_SLOTS] = {};
  size_t stage_cap[PD_STAGE_SLOTS] = {};
  hipEvent_t staged[PD_STAGE_SLOTS] = {};
  int stage_next = 0;
  // autotuned waves per map, keyed by (precision, dmax bucket, log2 pairs, maps)
  std::map<std::tuple<int, int, int, int>, int> tuned;
  bool tune_loaded = false;
};

// Waves per map for this batch: the autotuned value for its key, else a default.
int pd_tuned_waves(pd_ctx *ctx, const pd_problem *probs, int n, int prec);

// Bump allocator over byte offsets (256-byte aligned regions).
struct Arena {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

struct MapRegions {
  size_t tx64, ty64, txT, tyT, thc, C, lse, rpix, part_l, part_g, part_c, T3, lse32, part_g32, part_d,
      onehot, cert, unc_list, btile, order, pos, order_sums, nearmask;
  bool sorted, nearmask_on;
};

// Everything one batched evaluation / assignment needs, laid out in an arena.
struct EvalPlan {
  int n = 0, prec = 0;
  bool any_grad = false;
  bool with_diag = false;  // FP64/FP32: room for Hessian-diagonal partials (set before layout)
  // FP64/FP32: the indicator moments are computed once (pd_plan_onehot, after
  // the tables) and the gradient kernel skips the one-hot term (set before bind)
  bool onehot_pre = false;
  // FP64/FP32: the objective launch also assigns every pixel with a certified
  // arg-max (per-wave counts in part_c, the canonical pass for the rest); the
  // caller clears the cert slots between evaluations (set before layout)
  bool cert = false;
  // row coefficients in the spatial order of the grains (k_order.hip), for the
  // far-field test; requires the one-hot term precomputed wherever a gradient is
  // taken (set before layout)
  bool sort = false;
  long long max_px = 0;
  int max_n = 0;
  int target_waves = 8192;
  std::vector<MapDev> maps;
  std::vector<MapRegions> reg;
  std::vector<int32_t> offA, offB, offP, offR;
  std::vector<int32_t> off16P, off16A, off16B, off16R;  // BF16 path (prec 2)
  int max_hw = 0, max_k = 0, dmax = 8;
  size_t o_maps = 0, o_off = 0;
  MapDev *d_maps = nullptr;
  int32_t *d_offA = nullptr, *d_offB = nullptr, *d_offP = nullptr, *d_offR = nullptr;
  int32_t *d_off16P = nullptr, *d_off16A = nullptr, *d_off16B = nullptr, *d_off16R = nullptr;
};

// Device memory of an evaluation plan.  base == nullptr: the context's
// workspace, grown on demand, with the plan records staged through pinned host
// memory.  Otherwise `cap` bytes of fixed device memory, the plan records written
// by a kernel from its arguments, so that nothing is allocated.
struct PlanMemory {
  char *base = nullptr;
  size_t cap = 0;
};

pd_status pd_fail(pd_ctx *c, pd_status s, const std::string &msg);
pd_status pd_check_problem(pd_ctx *ctx, const pd_problem &p, int idx);
pd_status pd_reserve(pd_ctx *ctx, size_t bytes);
// rows (may be null): 2 entries per map, the evaluated rows [rows[2p], rows[2p+1])
// (already checked); null evaluates every row.
void pd_plan_layout(EvalPlan &P, Arena &L, const pd_problem *probs, int n, int prec,
                    const int32_t *rows = nullptr);
void pd_plan_bind(EvalPlan &P, char *base, const double *const *theta, double *phi_out,
                  double *const *grad_out, int32_t *const *labels_out, int64_t *n_correct);
hipError_t pd_plan_upload(pd_ctx *ctx, EvalPlan &P, hipStream_t s);
// Pinned staging ring: a buffer of >= bytes (waits only for the copy that used
// the slot PD_STAGE_SLOTS uploads ago), then its stream-ordered copy to dst.
hipError_t pd_stage_acquire(pd_ctx *ctx, size_t bytes, char **buf, int *slot);
hipError_t pd_stage_copy(pd_ctx *ctx, int slot, void *dst, size_t bytes, hipStream_t s);
// Memory for a laid-out plan (reserved in the workspace, or checked against the
// fixed buffer: PD_ERR_UNSUPPORTED if it does not fit), then bind and upload.
pd_status pd_plan_place(pd_ctx *ctx, EvalPlan &P, const Arena &L, const PlanMemory &mem,
                        const double *const *theta, double *phi_out, double *const *grad_out,
                        hipStream_t s);
// noalloc.hip: the plan records (maps and work-list offsets, at most
// PD_NOALLOC_MAX_MAPS maps) written into the plan's memory by a one-block kernel
// whose arguments carry them.
hipError_t pd_plan_upload_by_kernel(const EvalPlan &P, hipStream_t s);
// Set-up of the fixed scratch buffer of the allocation-free entry point on the
// current device (its device address, kept per device).  Called by pd_create.
pd_status pd_noalloc_setup(pd_ctx *ctx);
// Shared body of pd_objective_grad, pd_objective_grad_rows and
// pd_objective_grad_noalloc (rows: null or a checked row band per map).
pd_status pd_objective_grad_impl(pd_ctx *ctx, const pd_problem *probs, int32_t n_probs,
                                 const int32_t *rows, const double *const *theta,
                                 double *phi_out, double *const *grad_out, pd_precision prec,
                                 int32_t flags, void *stream, const PlanMemory &mem);
void pd_plan_tables(const EvalPlan &P, hipStream_t s);
// Indicator moments of every map when P.onehot_pre (after pd_plan_tables).
void pd_plan_onehot(const EvalPlan &P, hipStream_t s);
// center: run k_center (thc from theta); the fit driver forms thc itself.
// assign_maps: also assign these maps' pixels (same work list) in the
// objective launch (the fit's accuracy check).
void pd_plan_eval(const EvalPlan &P, bool with_grad, hipStream_t s, bool center,
                  const MapDev *assign_maps = nullptr);
void pd_plan_assign(const EvalPlan &P, hipStream_t s);

pd_status pd_bf16_objective_grad(pd_ctx *ctx, const pd_problem *probs, int n,
                                 const int32_t *rows, const double *const *theta,
                                 double *phi_out, double *const *grad_out, hipStream_t s,
                                 const PlanMemory &mem);
void pd_fit_release(pd_ctx *ctx);
// BF16 path: stage 0 prep (thc pieces), 1 log-sum-exp, 2 gradient, 3 reductions.
void pd_bf16_launch(const EvalPlan &P, int stage, hipStream_t s);
// BF16 path: time its prep / matrix-core stages, recording ev[1], ev[2], ev[3]
// (the PREP, LSE and GRAD slots).
void pd_bf16_profile_stages(pd_ctx *ctx, const EvalPlan &P, int reps, hipStream_t s,
                            hipEvent_t *ev);
// BF16 matrix-core evaluation of a plan laid out with FP32 buffers.
void pd_bf16_plan_eval(pd_ctx *ctx, const EvalPlan &P, hipStream_t s, bool center);
