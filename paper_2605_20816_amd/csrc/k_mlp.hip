// k_mlp.hip -- kernels of the warm-start network 32 -> 256 -> 256 -> kout.
//
// Training runs in FP32 on the vector ALUs: one LDS-tiled GEMM kernel (64 x 64
// output tile, 16-deep k-slices, 4 x 4 outputs per thread) covers the forward
// products, the input-gradient products (transposed weights through strides) and
// the weight-gradient products (transposed activations, split over the batch
// into fixed slices whose partial tiles are summed in slice order, so gradients
// are deterministic).  The bias of a layer is the row after its weights in the
// parameter buffer, so [x, 1] times [W; b] gives both the layer and, for the
// gradient, [x, 1]^T dz gives dW and db in one product.
// Inference runs on bf16 matrix cores (v_mfma_f32_32x32x16_bf16, FP32
// accumulation): one wave per 32 x 32 output tile, operands loaded straight from
// bf16 copies of the activations (row-major) and of the transposed weights.
#include "pd_host.h"

#include <math.h>

#include "pd_warm.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#define GT 64   // output tile
#define GK 16   // k-slice

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

struct GemmArgs {
  const float *A;
  long long a_rs, a_cs;   // A[m][k] = A[m * a_rs + k * a_cs]
  const float *B;
  long long b_rs, b_cs;   // B[k][n] = B[k * b_rs + n * b_cs]
  float *C;               // C[m][n] = C[m * ldc + n]; split slice z writes C + z * M * ldc
  int ldc;
  int M, N, Kd;
  int ones_row;           // A's last row (m == M - 1) reads as 1
  int kslice;             // k range of one grid.z slice
  int epi;
  const float *bias;      // EPI_BIAS*: bias[n]
  float *C2;              // EPI_BIAS_GELU: activation out (same layout as C)
  const float *Zaux;      // EPI_GELU_GRAD: pre-activation (same layout as C)
};

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__global__ __launch_bounds__(256) void km_gemm(GemmArgs g) {
  __shared__ float sA[GK][GT + 4];
  __shared__ float sB[GK][GT + 4];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int k_begin = blockIdx.z * g.kslice;
  const int k_end = min(g.Kd, k_begin + g.kslice);
  const int tx = tid % 16, ty = tid / 16;
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int k0 = k_begin; k0 < k_end; k0 += GK) {
    // A tile: 64 rows x 16 k; B tile: 16 k x 64 columns (4 elements per thread each)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = tid + 256 * e;
      const int mm = q / GK, kk = q % GK;
      const int m = m0 + mm, k = k0 + kk;
      float va = 0.f;
      if (m < g.M && k < k_end) {
        if (g.ones_row && m == g.M - 1) va = 1.f;
        else va = g.A[(long long)m * g.a_rs + (long long)k * g.a_cs];
      }
      sA[kk][mm] = va;
      const int kb = q / GT, nn = q % GT;
      const int n = n0 + nn, kB = k0 + kb;
      sB[kb][nn] = (n < g.N && kB < k_end) ? g.B[(long long)kB * g.b_rs + (long long)n * g.b_cs] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sA[kk][ty * 4 + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sB[kk][tx * 4 + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  float *C = g.C + (size_t)blockIdx.z * g.M * g.ldc;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int m = m0 + ty * 4 + a;
    if (m >= g.M) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int n = n0 + tx * 4 + b;
      if (n >= g.N) continue;
      float v = acc[a][b];
      const size_t o = (size_t)m * g.ldc + n;
      if (g.epi == EPI_BIAS || g.epi == EPI_BIAS_GELU) v += g.bias[n];
      if (g.epi == EPI_GELU_GRAD) v *= gelu_grad_f(g.Zaux[o]);
      C[o] = v;
      if (g.epi == EPI_BIAS_GELU) g.C2[o] = gelu_f(v);
    }
  }
}

// out[j] = sum_z part[z * count + j], z ascending
__global__ void km_sum_slices(const float *__restrict__ part, int slices, size_t count,
                              float *__restrict__ out) {
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < count;
       j += (size_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < slices; ++z) s += part[(size_t)z * count + j];
    out[j] = s;
  }
}

// dy = 2 (y - t) / (B K); per-block partial sums of (y - t)^2 in FP64
__global__ __launch_bounds__(256) void km_loss_grad(const float *__restrict__ y,
                                                    const float *__restrict__ t, size_t count,
                                                    float scale, float *__restrict__ dy,
                                                    double *__restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < count;
       j += (size_t)gridDim.x * blockDim.x) {
    const float r = y[j] - t[j];
    dy[j] = 2.0f * r * scale;
    s += (double)r * (double)r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void km_loss_final(const double *__restrict__ part, int n,
                                                     double scale, double *__restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) s += part[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * scale;
}

__global__ void km_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                        float *__restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                        float c1, float c2) {
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (size_t)gridDim.x * blockDim.x) {
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.0f - b1) * gj;
    const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    p[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
  }
}

// ---------------------------------------------------------------- host helpers
size_t pd_mlp_params(int kout) {
  return (size_t)(PD_MLP_IN + 1) * PD_MLP_HID + (size_t)(PD_MLP_HID + 1) * PD_MLP_HID +
         (size_t)(PD_MLP_HID + 1) * kout;
}

static void mlp_offsets(int kout, size_t &o1, size_t &o2, size_t &o3) {
  o1 = 0;
  o2 = (size_t)(PD_MLP_IN + 1) * PD_MLP_HID;
  o3 = o2 + (size_t)(PD_MLP_HID + 1) * PD_MLP_HID;
  (void)kout;
}

// Returns the number of k slices launched (partial tiles written for slices > 1).
static int gemm(const GemmArgs &g0, int slices, hipStream_t s) {
  GemmArgs g = g0;
  g.kslice = (g.Kd + slices - 1) / slices;
  g.kslice = (g.kslice + GK - 1) / GK * GK;
  slices = (g.Kd + g.kslice - 1) / g.kslice;
  dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT, slices);
  km_gemm<<<grid, 256, 0, s>>>(g);
  return slices;
}

// y[B x kout] (ldc kout) of layer l: x[B x in] (row stride in) times [W; b]
static void layer_fwd(const float *x, int B, int in, const float *Wb, int out, float *z,
                      float *h, hipStream_t s) {
  GemmArgs g{};
  g.A = x;
  g.a_rs = in;
  g.a_cs = 1;
  g.B = Wb;
  g.b_rs = out;
  g.b_cs = 1;
  g.C = z;
  g.ldc = out;
  g.M = B;
  g.N = out;
  g.Kd = in;
  g.epi = h ? EPI_BIAS_GELU : EPI_BIAS;
  g.bias = Wb + (size_t)in * out;
  g.C2 = h;
  gemm(g, 1, s);
}

void pd_mlp_launch_forward(const float *params, int kout, const float *x, int batch, float *z1,
                           float *h1, float *z2, float *h2, float *y, hipStream_t s) {
  size_t o1, o2, o3;
  mlp_offsets(kout, o1, o2, o3);
  layer_fwd(x, batch, PD_MLP_IN, params + o1, PD_MLP_HID, z1, h1, s);
  layer_fwd(h1, batch, PD_MLP_HID, params + o2, PD_MLP_HID, z2, h2, s);
  layer_fwd(h2, batch, PD_MLP_HID, params + o3, kout, y, nullptr, s);
}

static int grad_slices(int batch) { return std::max(1, std::min(32, batch / 256)); }

size_t pd_mlp_backward_ws(int kout, int batch) {
  const size_t act = (size_t)batch * PD_MLP_HID * sizeof(float);
  const size_t yb = (size_t)batch * kout * sizeof(float);
  const size_t part = (size_t)grad_slices(batch) * (PD_MLP_HID + 1) * PD_MLP_HID * sizeof(float);
  return 6 * act + 2 * yb + part + 1024 * sizeof(double) + 4096;
}

// dW_aug [(in + 1) x out] = [act, 1]^T dz, written to grad
static void weight_grad(const float *act, int B, int in, const float *dz, int out, float *part,
                        float *grad, hipStream_t s) {
  GemmArgs g{};
  g.A = act;          // A[m][k] = act[k][m]
  g.a_rs = 1;
  g.a_cs = in;
  g.B = dz;
  g.b_rs = out;
  g.b_cs = 1;
  g.C = part;
  g.ldc = out;
  g.M = in + 1;
  g.N = out;
  g.Kd = B;
  g.ones_row = 1;
  g.epi = EPI_STORE;
  const int used = gemm(g, grad_slices(B), s);
  const size_t count = (size_t)(in + 1) * out;
  km_sum_slices<<<(int)std::min<size_t>(1024, (count + 255) / 256), 256, 0, s>>>(part, used, count, grad);
}

// dz_prev [B x in] = (dz [B x out] W^T) * gelu'(z_prev)
static void input_grad(const float *dz, int B, int out, const float *W, int in, const float *zprev,
                       float *dzprev, hipStream_t s) {
  GemmArgs g{};
  g.A = dz;
  g.a_rs = out;
  g.a_cs = 1;
  g.B = W;            // B[k][n] = W[n][k], W is in x out
  g.b_rs = 1;
  g.b_cs = out;
  g.C = dzprev;
  g.ldc = in;
  g.M = B;
  g.N = in;
  g.Kd = out;
  g.epi = EPI_GELU_GRAD;
  g.Zaux = zprev;
  gemm(g, 1, s);
}

void pd_mlp_launch_backward(const float *params, int kout, const float *x, const float *t,
                            int batch, char *ws, double *loss, float *grad, hipStream_t s) {
  size_t o1, o2, o3;
  mlp_offsets(kout, o1, o2, o3);
  const size_t act = (size_t)batch * PD_MLP_HID;
  float *z1 = (float *)ws, *h1 = z1 + act, *z2 = h1 + act, *h2 = z2 + act, *d2 = h2 + act,
        *d1 = d2 + act;
  float *y = d1 + act, *dy = y + (size_t)batch * kout;
  float *part = dy + (size_t)batch * kout;
  double *lpart = (double *)(((uintptr_t)(part + (size_t)grad_slices(batch) * (PD_MLP_HID + 1) *
                                                      PD_MLP_HID) + 255) & ~(uintptr_t)255);
  pd_mlp_launch_forward(params, kout, x, batch, z1, h1, z2, h2, y, s);
  const size_t count = (size_t)batch * kout;
  const int nb = (int)std::min<size_t>(1024, (count + 255) / 256);
  km_loss_grad<<<nb, 256, 0, s>>>(y, t, count, 1.0f / (float)count, dy, lpart);
  km_loss_final<<<1, 256, 0, s>>>(lpart, nb, 1.0 / (double)count, loss);
  weight_grad(h2, batch, PD_MLP_HID, dy, kout, part, grad + o3, s);
  input_grad(dy, batch, kout, params + o3, PD_MLP_HID, z2, d2, s);
  weight_grad(h1, batch, PD_MLP_HID, d2, PD_MLP_HID, part, grad + o2, s);
  input_grad(d2, batch, PD_MLP_HID, params + o2, PD_MLP_HID, z1, d1, s);
  weight_grad(x, batch, PD_MLP_IN, d1, PD_MLP_HID, part, grad + o1, s);
}

void pd_mlp_launch_adam(float *params, const float *grad, float *m, float *v, size_t n, int step,
                        float lr, float beta1, float beta2, float eps, hipStream_t s) {
  const float c1 = 1.0f - powf(beta1, (float)step);
  const float c2 = 1.0f - powf(beta2, (float)step);
  km_adam<<<(int)std::min<size_t>(2048, (n + 255) / 256), 256, 0, s>>>(params, grad, m, v, n, lr,
                                                                       beta1, beta2, eps, c1, c2);
}

// ---------------------------------------------------------------- BF16 inference
// Wt[n][k] = bf16(W[k][n]) for n < out_pad (zero rows beyond out), k < in
__global__ void km_to_bf16_t(const float *__restrict__ W, int in, int out, int out_pad,
                             __bf16 *__restrict__ Wt) {
  const size_t count = (size_t)out_pad * in;
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < count;
       j += (size_t)gridDim.x * blockDim.x) {
    const int n = (int)(j / in), k = (int)(j % in);
    Wt[j] = (__bf16)(n < out ? W[(size_t)k * out + n] : 0.f);
  }
}

// xb[r][k] = bf16(x[r][k]) for r < rows_pad (zero rows beyond batch)
__global__ void km_rows_to_bf16(const float *__restrict__ x, int batch, int rows_pad, int in,
                                __bf16 *__restrict__ xb) {
  const size_t count = (size_t)rows_pad * in;
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < count;
       j += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(j / in);
    xb[j] = (__bf16)(r < batch ? x[j] : 0.f);
  }
}

// One wave per 32 x 32 output tile: out = act(x Wt^T + b).  x: rows_pad x in bf16,
// Wt: out_pad x in bf16.  Hidden layers write bf16 GELU activations (ldo = out_pad);
// the last layer writes FP32 y[r][n] for r < batch, n < out (row stride y_stride).
__global__ __launch_bounds__(256) void km_bf16_layer(const __bf16 *__restrict__ x,
                                                     const __bf16 *__restrict__ Wt,
                                                     const float *__restrict__ bias, int in,
                                                     int out, int out_pad, int tiles_n, int n_tiles,
                                                     __bf16 *__restrict__ hb, float *__restrict__ y,
                                                     int batch, int y_stride) {
  const int wave = blockIdx.x * 4 + threadIdx.x / 64;
  if (wave >= n_tiles) return;
  const int lane = threadIdx.x % 64;
  const int tr = wave / tiles_n, tn = wave % tiles_n;
  const int i = lane % 32, h = lane / 32;
  const __bf16 *pa = x + (size_t)(tr * 32 + i) * in + 8 * h;
  const __bf16 *pb = Wt + (size_t)(tn * 32 + i) * in + 8 * h;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int k0 = 0; k0 < in; k0 += 16) {
    const bf16x8 a = *(const bf16x8 *)(pa + k0);
    const bf16x8 b = *(const bf16x8 *)(pb + k0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  // D[row][col]: col = lane % 32, row = 8 (r / 4) + 4 h + r % 4
  const int col = tn * 32 + i;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = tr * 32 + 8 * (r / 4) + 4 * h + r % 4;
    if (col >= out) continue;
    const float v = acc[r] + bias[col];
    if (hb) hb[(size_t)row * out_pad + col] = (__bf16)gelu_f(v);
    else if (row < batch) y[(size_t)row * y_stride + col] = v;
  }
}

static int round_up(int v, int m) { return (v + m - 1) / m * m; }

size_t pd_mlp_bf16_ws(int kout, int batch) {
  const int rows = round_up(std::max(batch, 1), 32);
  const int kp = round_up(kout, 32);
  size_t b = 0;
  b += (size_t)PD_MLP_HID * PD_MLP_IN + (size_t)PD_MLP_HID * PD_MLP_HID + (size_t)kp * PD_MLP_HID;
  b += (size_t)rows * PD_MLP_IN + 2 * (size_t)rows * PD_MLP_HID;
  return b * sizeof(__bf16) + 4 * 256;
}

static void bf16_layer(const __bf16 *x, int rows, const __bf16 *Wt, const float *bias, int in,
                       int out, int out_pad, __bf16 *hb, float *y, int batch, int y_stride,
                       hipStream_t s) {
  const int tiles_n = out_pad / 32;
  const int n_tiles = (rows / 32) * tiles_n;
  km_bf16_layer<<<(n_tiles + 3) / 4, 256, 0, s>>>(x, Wt, bias, in, out, out_pad, tiles_n, n_tiles,
                                                  hb, y, batch, y_stride);
}

void pd_mlp_launch_bf16(const float *params, int kout, const float *x, int batch, char *ws,
                        float *y, int y_stride, hipStream_t s) {
  size_t o1, o2, o3;
  mlp_offsets(kout, o1, o2, o3);
  const int rows = round_up(batch, 32);
  const int kp = round_up(kout, 32);
  __bf16 *w1 = (__bf16 *)ws;
  __bf16 *w2 = w1 + (size_t)PD_MLP_HID * PD_MLP_IN;
  __bf16 *w3 = w2 + (size_t)PD_MLP_HID * PD_MLP_HID;
  __bf16 *xb = w3 + (size_t)kp * PD_MLP_HID;
  __bf16 *h1 = xb + (size_t)rows * PD_MLP_IN;
  __bf16 *h2 = h1 + (size_t)rows * PD_MLP_HID;
  km_to_bf16_t<<<64, 256, 0, s>>>(params + o1, PD_MLP_IN, PD_MLP_HID, PD_MLP_HID, w1);
  km_to_bf16_t<<<256, 256, 0, s>>>(params + o2, PD_MLP_HID, PD_MLP_HID, PD_MLP_HID, w2);
  km_to_bf16_t<<<64, 256, 0, s>>>(params + o3, PD_MLP_HID, kout, kp, w3);
  km_rows_to_bf16<<<std::min(1024, (rows * PD_MLP_IN + 255) / 256), 256, 0, s>>>(x, batch, rows,
                                                                                 PD_MLP_IN, xb);
  bf16_layer(xb, rows, w1, params + o1 + (size_t)PD_MLP_IN * PD_MLP_HID, PD_MLP_IN, PD_MLP_HID,
             PD_MLP_HID, h1, nullptr, batch, 0, s);
  bf16_layer(h1, rows, w2, params + o2 + (size_t)PD_MLP_HID * PD_MLP_HID, PD_MLP_HID, PD_MLP_HID,
             PD_MLP_HID, h2, nullptr, batch, 0, s);
  bf16_layer(h2, rows, w3, params + o3 + (size_t)PD_MLP_HID * kout, PD_MLP_HID, kout, kp, nullptr,
             y, batch, y_stride, s);
}
