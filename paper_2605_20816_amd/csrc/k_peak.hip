// k_peak.hip -- microbenchmarks of the units that bound the evaluation kernels:
// FP32 FMA (built, like everything here, without packed FP32), the hardware
// base-2 exponential v_exp_f32, four FP32 FMAs per exponential (whether the two
// overlap), FP64 FMA, and the BF16 matrix-core product of the BF16 path
// (v_mfma_f32_32x32x16_bf16).  Every thread runs PK_CHAINS independent
// dependency chains and the grid holds many waves per SIMD, so issue rate, not
// latency, limits the loop; the results are summed into out so nothing is
// removed as dead code.
#include "pd_host.h"

#include <vector>

#define PK_CHAINS 8
#define PK_BLOCKS 4096
#define PK_THREADS 256

typedef __bf16 pk_bf16x8 __attribute__((ext_vector_type(8)));
typedef float pk_f32x16 __attribute__((ext_vector_type(16)));

// KIND 0: FP32 FMA; 1: exp2; 2: 4 FMA + 1 exp2 per chain step; 3: FP64 FMA;
// 4: BF16 MFMA 32x32x16 (4 independent accumulators per wave).
template <int KIND>
__global__ __launch_bounds__(PK_THREADS) void k_peak(float *out, int iters, float m, float c) {
  const int gid = blockIdx.x * PK_THREADS + threadIdx.x;
  float r = 0.f;
  if constexpr (KIND == 0 || KIND == 1 || KIND == 2) {
    float a[PK_CHAINS];
#pragma unroll
    for (int j = 0; j < PK_CHAINS; ++j) a[j] = 0.25f + 1e-6f * (float)(threadIdx.x + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < PK_CHAINS; ++j) {
        if constexpr (KIND == 0) {
          a[j] = __builtin_fmaf(a[j], m, c);
        } else if constexpr (KIND == 1) {
          a[j] = __builtin_amdgcn_exp2f(-a[j]);  // the negation is an input modifier
        } else {
          a[j] = __builtin_fmaf(a[j], m, c);
          a[j] = __builtin_fmaf(a[j], m, c);
          a[j] = __builtin_fmaf(a[j], m, c);
          a[j] = __builtin_fmaf(a[j], m, c);
          a[j] = __builtin_amdgcn_exp2f(-a[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < PK_CHAINS; ++j) r += a[j];
  } else if constexpr (KIND == 3) {
    double a[PK_CHAINS];
#pragma unroll
    for (int j = 0; j < PK_CHAINS; ++j) a[j] = 0.25 + 1e-6 * (double)(threadIdx.x + j);
    const double md = m, cd = c;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int j = 0; j < PK_CHAINS; ++j) a[j] = __builtin_fma(a[j], md, cd);
#pragma unroll
    for (int j = 0; j < PK_CHAINS; ++j) r += (float)a[j];
  } else {
    pk_bf16x8 A, B;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      A[e] = (__bf16)(m * (float)(threadIdx.x % 7 + e));
      B[e] = (__bf16)(c * (float)(threadIdx.x % 5 + e));
    }
    pk_f32x16 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[q][e] = 0.f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[q], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 16; ++e) r += acc[q][e];
  }
  out[gid] = r;
}

extern "C" pd_status pd_probe_peak(pd_ctx *ctx, int32_t kind, double *rate_out, void *stream) {
  if (!ctx || !rate_out || kind < 0 || kind > 4)
    return ctx ? pd_fail(ctx, PD_ERR_INVALID_ARG, "pd_probe_peak: bad arguments") : PD_ERR_INVALID_ARG;
  ctx->err.clear();
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, hipGetErrorString(e));
  pd_status st = pd_reserve(ctx, sizeof(float) * PK_BLOCKS * PK_THREADS);
  if (st != PD_OK) return st;
  float *out = (float *)ctx->ws;
  hipStream_t s = (hipStream_t)stream;
  // iterations per thread, sized to about a millisecond per launch
  static const int iters_of[5] = {4096, 1024, 512, 2048, 256};
  const int iters = iters_of[kind];
  auto launch = [&]() {
    switch (kind) {
      case 0: k_peak<0><<<PK_BLOCKS, PK_THREADS, 0, s>>>(out, iters, 0.5f, 0.25f); break;
      case 1: k_peak<1><<<PK_BLOCKS, PK_THREADS, 0, s>>>(out, iters, 0.5f, 0.25f); break;
      case 2: k_peak<2><<<PK_BLOCKS, PK_THREADS, 0, s>>>(out, iters, 0.5f, 0.25f); break;
      case 3: k_peak<3><<<PK_BLOCKS, PK_THREADS, 0, s>>>(out, iters, 0.5f, 0.25f); break;
      default: k_peak<4><<<PK_BLOCKS, PK_THREADS, 0, s>>>(out, iters, 0.5f, 0.25f); break;
    }
  };
  hipEvent_t e0, e1;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, hipGetErrorString(e));
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return pd_fail(ctx, PD_ERR_HIP, hipGetErrorString(e));
  }
  launch();  // warm-up
  float best = 1e30f;
  for (int r = 0; r < 5 && e == hipSuccess; ++r) {
    (void)hipEventRecord(e0, s);
    launch();
    (void)hipEventRecord(e1, s);
    e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms < best) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, hipGetErrorString(e));
  const double threads = (double)PK_BLOCKS * PK_THREADS;
  double ops;
  if (kind == 0 || kind == 3) ops = 2.0 * threads * PK_CHAINS * iters;      // flops
  else if (kind == 1 || kind == 2) ops = threads * PK_CHAINS * iters;       // exponentials
  else ops = 2.0 * (threads / PD_WAVE) * 4 * iters * (32.0 * 32.0 * 16.0);  // flops
  *rate_out = ops / (best * 1e-3);
  return PD_OK;
}

// ---------------------------------------------------------------------------
// The evaluation kernels' exponentials and logarithms on given arguments, so
// their accuracy can be checked against a reference library on the host.
#include "pd_math.h"

__global__ __launch_bounds__(PK_THREADS) void k_probe_math(int fn, const double *__restrict__ in,
                                                          double *__restrict__ out, long long n) {
  const long long j = (long long)blockIdx.x * PK_THREADS + threadIdx.x;
  if (j >= n) return;
  const double x = in[j];
  double y;
  switch (fn) {
    case 0: y = pd_exp2<double>(x); break;
    case 1: y = (double)pd_exp2<float>((float)x); break;
    case 2: y = pd_log2<double>(x); break;
    default: y = (double)pd_log2<float>((float)x); break;
  }
  out[j] = y;
}

extern "C" pd_status pd_probe_math(pd_ctx *ctx, int32_t fn, const double *in, double *out,
                                   int64_t n, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (fn < 0 || fn > 3) return pd_fail(ctx, PD_ERR_INVALID_ARG, "fn must be 0..3");
  if (n < 0 || (n > 0 && (!in || !out))) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n >= 0 and device in/out");
  if (n == 0) return PD_OK;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) {
    const unsigned blocks = (unsigned)((n + PK_THREADS - 1) / PK_THREADS);
    k_probe_math<<<blocks, PK_THREADS, 0, (hipStream_t)stream>>>(fn, in, out, n);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, std::string("k_probe_math: ") + hipGetErrorString(e));
  return PD_OK;
}
