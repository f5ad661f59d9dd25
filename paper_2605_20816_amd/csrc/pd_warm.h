// pd_warm.h -- device view of one map for the warm-start kernels (descriptors,
// moment seed, training targets, warm start from network outputs) and the
// launchers of the network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pd.h"
#include "pd_internal.h"



struct WarmDev {
  int32_t H, W, N, d, K;
  const int32_t *labels;
  long long *isum;         // N x 6 exact integer pixel sums
  int32_t *bbox;           // N x 4 (r0, r1, c0, c1)
  double *frame;           // N x 8 (y1, y2, r, B11, B12, B22, count, 0)
  float *desc;             // N x 32
  double *theta_h;         // N x K moment seed
  const double *theta_fit; // N x K fitted theta (targets)
  float *target;           // N x K normalised targets
  double *lambda;          // RMS of the centred fitted theta (1 value), may be NULL
  const float *mlp_out;    // N x out_stride network outputs, or NULL
  int32_t out_stride;
  double *theta_out;       // N x K warm start before scaling
};

void pd_warm_launch_desc(const WarmDev *W, const int32_t *off, int n_maps, int total_grains,
                         int max_n, hipStream_t s);
void pd_warm_launch_heuristic(const WarmDev *W, int n_maps, hipStream_t s);
void pd_warm_launch_targets(const WarmDev *W, int n_maps, hipStream_t s);
void pd_warm_launch_apply(const WarmDev *W, int n_maps, hipStream_t s);

// Network of the warm start: 32 -> 256 -> 256 -> kout (GELU after both hidden
// layers).  Parameters are one FP32 buffer [W1 (32 x 256), b1, W2 (256 x 256), b2,
// W3 (256 x kout), b3], weights stored input-major (row k = input k).
#define PD_MLP_HID PD_MLP_WIDTH
size_t pd_mlp_params(int kout);
// FP32 forward; keeps the pre-activations z1, z2 and activations h1, h2 (B x 256
// each) when they are non-NULL.
void pd_mlp_launch_forward(const float *params, int kout, const float *x, int batch, float *z1,
                           float *h1, float *z2, float *h2, float *y, hipStream_t s);
// Loss and full parameter gradient of mean((y - t)^2); ws holds 4 B x 256 floats
// plus B x kout floats plus partial sums (pd_mlp_backward_ws bytes).
size_t pd_mlp_backward_ws(int kout, int batch);
void pd_mlp_launch_backward(const float *params, int kout, const float *x, const float *t,
                            int batch, char *ws, double *loss, float *grad, hipStream_t s);
void pd_mlp_launch_adam(float *params, const float *grad, float *m, float *v, size_t n,
                        int step, float lr, float beta1, float beta2, float eps, hipStream_t s);
// BF16 inference on matrix cores: weights and activations rounded to bf16, FP32
// accumulation; ws holds the bf16 copies (pd_mlp_bf16_ws bytes).
size_t pd_mlp_bf16_ws(int kout, int batch);
void pd_mlp_launch_bf16(const float *params, int kout, const float *x, int batch, char *ws,
                        float *y, int y_stride, hipStream_t s);
