// noalloc.hip -- the allocation-free variant of pd_objective_grad.
//
// Some callers cannot allocate device memory at the time of the call (code under
// stream capture into a graph, tight serving loops, harnesses that forbid it).
// pd_objective_grad_noalloc runs the same kernels as pd_objective_grad, with
// their scratch (Legendre tables, centred coefficients, row coefficients,
// per-pixel log-sum-exp, fixed-order partial sums, plan records) laid out in one
// file-scope device array instead of the context's workspace, and the plan
// records written into it by a one-block kernel that receives them as kernel
// arguments (no pinned staging buffer, no host-to-device copy).
//
// The array is a host-side stand-in in host code: kernels are only ever given
// its device address, taken once per device by pd_noalloc_setup (called from
// pd_create with the device current) through hipGetSymbolAddress.
#include "pd_host.h"

#include <string.h>

#include <mutex>
#include <string>

// Fixed scratch of the allocation-free entry point, one copy per device, held
// until the process ends.
static __device__ __align__(256) char scratch[PD_NOALLOC_SCRATCH_BYTES];

#define PD_NOALLOC_MAX_DEVICES 64

static std::mutex g_noalloc_mu;
static char *g_scratch_dev[PD_NOALLOC_MAX_DEVICES];  // device address per device, or null

pd_status pd_noalloc_setup(pd_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= PD_NOALLOC_MAX_DEVICES)
    return pd_fail(ctx, PD_ERR_UNSUPPORTED, "device index above the library's table of devices");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_scratch_dev[ctx->device] != nullptr) return PD_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    return pd_fail(ctx, PD_ERR_HIP,
                   std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_dev[ctx->device] = (char *)ptr;
  return PD_OK;
}

// The plan records as kernel arguments: the MapDev array, then (at the plan's
// offset o_off - o_maps) the eight work-list offset arrays of n + 1 entries.
#define PD_PLAN_BLOB_BYTES 2048
struct PlanBlob {
  uint32_t words[PD_PLAN_BLOB_BYTES / 4];
  int32_t n_words;
};

__global__ __launch_bounds__(PD_BLOCK) void k_write_plan(PlanBlob blob, uint32_t *dst) {
  for (int i = threadIdx.x; i < blob.n_words; i += PD_BLOCK) dst[i] = blob.words[i];
}

hipError_t pd_plan_upload_by_kernel(const EvalPlan &P, hipStream_t s) {
  const size_t maps_bytes = sizeof(MapDev) * P.n;
  const size_t gap = P.o_off - P.o_maps;
  const size_t total = gap + sizeof(int32_t) * 8 * (P.n + 1);
  static_assert(sizeof(MapDev) % 4 == 0, "MapDev is copied as 32-bit words");
  if (total > PD_PLAN_BLOB_BYTES) return hipErrorInvalidValue;  // excluded by the map limit
  PlanBlob blob;
  memset(&blob, 0, sizeof blob);
  memcpy(blob.words, P.maps.data(), maps_bytes);
  int32_t *o = (int32_t *)((char *)blob.words + gap);
  const std::vector<int32_t> *arrs[8] = {&P.offA,   &P.offB,   &P.offP,   &P.offR,
                                         &P.off16P, &P.off16A, &P.off16B, &P.off16R};
  for (int a = 0; a < 8; ++a)
    for (int k = 0; k <= P.n; ++k) o[a * (P.n + 1) + k] = (*arrs[a])[k];
  blob.n_words = (int32_t)(total / 4);
  k_write_plan<<<1, PD_BLOCK, 0, s>>>(blob, (uint32_t *)P.d_maps);
  return hipGetLastError();
}

extern "C" pd_status pd_objective_grad_noalloc(pd_ctx *ctx, const pd_problem *probs,
                                               int32_t n_probs, const double *const *theta,
                                               double *phi_out, double *const *grad_out,
                                               pd_precision prec, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (n_probs > PD_NOALLOC_MAX_MAPS)
    return pd_fail(ctx, PD_ERR_INVALID_ARG,
                   "pd_objective_grad_noalloc takes at most " +
                       std::to_string(PD_NOALLOC_MAX_MAPS) + " maps per call");
  char *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (ctx->device >= 0 && ctx->device < PD_NOALLOC_MAX_DEVICES) base = g_scratch_dev[ctx->device];
  }
  if (base == nullptr)
    return pd_fail(ctx, PD_ERR_HIP, "the fixed scratch buffer was not set up on this device");
  PlanMemory mem;
  mem.base = base;
  mem.cap = PD_NOALLOC_SCRATCH_BYTES;
  return pd_objective_grad_impl(ctx, probs, n_probs, nullptr, theta, phi_out, grad_out, prec, 0,
                                stream, mem);
}
