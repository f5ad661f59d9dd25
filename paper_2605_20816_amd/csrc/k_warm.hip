// k_warm.hip -- per-grain descriptors, the moment seed of Section 5.6.2, training
// targets and the assembly of a warm start from network outputs.
//
// Per grain i (pixels G_i, centres x = ((2c+1-W)/W, (2r+1-H)/H), n pixels):
//   frame: centroid y'_i and central second moments B'_i (eq. centroid-guess and
//     cov-guess) from exact integer sums of c, r, c^2, c r, r^2; radius
//     r_i = 2 sqrt(lambda_max(B'_i)) (at least one pixel width); pixel count.
//   descriptor (PD_DESC_DIM = 32 floats): log(N |G_i| / n); the 27 Legendre
//     indicator moments mean_{x in G_i} P_a(x_1) P_b(x_2), 1 <= a + b <= 6, in the
//     degree-graded order (the degree-1 pair is the centroid); N B'_i (three
//     entries, O(1) for cells of typical size); log(N) / 10.
// Moment seed: A'_i = B'_i^{-1} (eq. A-guess; the identity at degree 1),
//   w'_i = sqrt(det A'_i) area(G_i) / pi with area(G_i) = 4 |G_i| / n (the ratio
//   of the grain's area to that of the ellipse of B'_i), the score
//   (x - y')^T A' (x - y') - w' of eq. h-APD in Legendre coefficients
//   (x^2 = (2 P_2(x) + 1) / 3); at degree 1 the common |x|^2 is dropped.
// Grains without pixels get the row (C, 0, ..., 0) with C above every other
//   grain's score on [-1, 1]^2 (|P_a| <= 1 there), so they win no pixel.
// Targets: the fitted theta centred over the non-empty grains (a common shift is
//   a gauge, Lemma 4.2) and divided by its root mean square over those grains and
//   the K coefficients (the scale of a fit is free, Proposition 4.8).
// The per-grain sums use integer atomics (exact) and one wave per grain over its
// bounding box in a fixed order, so descriptors are bitwise reproducible.
#include "pd_host.h"

#include <math.h>

#include "pd_warm.h"

__device__ inline void legendre_d(double t, int d, double *P) {
  P[0] = 1.0;
  if (d >= 1) P[1] = t;
  for (int m = 1; m < d; ++m) P[m + 1] = ((double)(2 * m + 1) * t * P[m] - (double)m * P[m - 1]) / (double)(m + 1);
}

// Block-wide sum of one double per thread (fixed tree order); every thread
// receives the total.
__device__ inline double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

__device__ inline double block_max(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
__global__ void kw_zero(const WarmDev *__restrict__ W, int n_maps) {
  const WarmDev &M = W[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M.N; i += gridDim.x * blockDim.x) {
    for (int q = 0; q < 6; ++q) M.isum[(size_t)i * 6 + q] = 0;
    M.bbox[(size_t)i * 4 + 0] = 0x7fffffff;
    M.bbox[(size_t)i * 4 + 1] = -1;
    M.bbox[(size_t)i * 4 + 2] = 0x7fffffff;
    M.bbox[(size_t)i * 4 + 3] = -1;
  }
}

// integer sums per grain: count, sum c, sum r, sum c^2, sum c r, sum r^2; bounding box
__global__ void kw_pass1(const WarmDev *__restrict__ W, int n_maps) {
  const WarmDev &M = W[blockIdx.y];
  const long long n = (long long)M.H * M.W;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (long long)gridDim.x * blockDim.x) {
    const int g = M.labels[j];
    if (g < 0 || g >= M.N) continue;
    const unsigned long long r = (unsigned long long)(j / M.W), c = (unsigned long long)(j % M.W);
    unsigned long long *s = (unsigned long long *)M.isum + (size_t)g * 6;
    atomicAdd(s + 0, 1ull);
    atomicAdd(s + 1, c);
    atomicAdd(s + 2, r);
    atomicAdd(s + 3, c * c);
    atomicAdd(s + 4, c * r);
    atomicAdd(s + 5, r * r);
    int *bb = M.bbox + (size_t)g * 4;
    atomicMin(bb + 0, (int)r);
    atomicMax(bb + 1, (int)r);
    atomicMin(bb + 2, (int)c);
    atomicMax(bb + 3, (int)c);
  }
}

// one wave per grain: frame (y'1, y'2, r, B11, B12, B22, count) and descriptor
__global__ __launch_bounds__(PD_BLOCK) void kw_pass2(const WarmDev *__restrict__ W,
                                                     const int32_t *__restrict__ off, int n_maps,
                                                     int total) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / PD_WAVE);
  const int lane = threadIdx.x % PD_WAVE;
  const int item = blockIdx.x * PD_WAVES_PER_BLOCK + wave;
  if (item >= total) return;
  const int m = pd_find_map(off, n_maps, item);
  const WarmDev &M = W[m];
  const int i = item - off[m];
  const long long *s = M.isum + (size_t)i * 6;
  const double cnt = (double)s[0];
  double *fr = M.frame + (size_t)i * PD_FRAME_DIM;
  float *ds = M.desc + (size_t)i * PD_DESC_DIM;
  const double Wd = M.W, Hd = M.H;
  if (cnt == 0.0) {  // empty grain: zero descriptor, frame at the origin
    if (lane < PD_DESC_DIM) ds[lane] = 0.f;
    if (lane < PD_FRAME_DIM) fr[lane] = lane == 2 ? 1.0 : 0.0;
    return;
  }
  // x1 = (2c + 1 - W) / W, x2 = (2r + 1 - H) / H
  const double Sc = (double)s[1], Sr = (double)s[2], Scc = (double)s[3], Scr = (double)s[4],
               Srr = (double)s[5];
  const double y1 = (2.0 * Sc + cnt * (1.0 - Wd)) / (cnt * Wd);
  const double y2 = (2.0 * Sr + cnt * (1.0 - Hd)) / (cnt * Hd);
  // central moments of (c, r), then scaled to x units (2/W, 2/H)
  const double mc = Sc / cnt, mr = Sr / cnt;
  const double vcc = Scc / cnt - mc * mc, vcr = Scr / cnt - mc * mr, vrr = Srr / cnt - mr * mr;
  const double B11 = vcc * 4.0 / (Wd * Wd), B12 = vcr * 4.0 / (Wd * Hd), B22 = vrr * 4.0 / (Hd * Hd);
  const double tr = B11 + B22, det = B11 * B22 - B12 * B12;
  const double lmax = 0.5 * tr + sqrt(fmax(0.25 * tr * tr - det, 0.0));
  const double rmin = 2.0 / fmax(Wd, Hd);
  const double rad = fmax(2.0 * sqrt(fmax(lmax, 0.0)), rmin);
  // Legendre indicator moments over the bounding box, fixed order
  const int *bb = M.bbox + (size_t)i * 4;
  const int r0 = bb[0], r1 = bb[1], c0 = bb[2], c1 = bb[3];
  const int bw = c1 - c0 + 1;
  const long long area = (long long)(r1 - r0 + 1) * bw;
  double acc[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) acc[q] = 0.0;
  for (long long e = lane; e < area; e += PD_WAVE) {
    const int r = r0 + (int)(e / bw), c = c0 + (int)(e % bw);
    if (M.labels[(size_t)r * M.W + c] != i) continue;
    double P1[7], P2[7];
    legendre_d((2.0 * c + 1.0 - Wd) / Wd, 6, P1);
    legendre_d((2.0 * r + 1.0 - Hd) / Hd, 6, P2);
    int q = 0;
#pragma unroll
    for (int deg = 1; deg <= 6; ++deg)
#pragma unroll
      for (int b = 0; b <= deg; ++b) acc[q++] += P1[deg - b] * P2[b];
  }
#pragma unroll
  for (int q = 0; q < 27; ++q) acc[q] = pd_wave_sum(acc[q]);
  if (lane == 0) {
    fr[0] = y1;
    fr[1] = y2;
    fr[2] = rad;
    fr[3] = B11;
    fr[4] = B12;
    fr[5] = B22;
    fr[6] = cnt;
    fr[7] = 0.0;
    const double n = Hd * Wd, N = (double)M.N;
    ds[0] = (float)log(cnt * N / n);
    for (int q = 0; q < 27; ++q) ds[1 + q] = (float)(acc[q] / cnt);
    ds[28] = (float)(N * B11);
    ds[29] = (float)(N * B12);
    ds[30] = (float)(N * B22);
    ds[31] = (float)(log(N) / 10.0);
  }
}

// Moment seed of Section 5.6.2 in Legendre coefficients; zero row if empty.
__device__ inline void heuristic_theta(const WarmDev &M, int i, double *th) {
  const double *fr = M.frame + (size_t)i * PD_FRAME_DIM;
  const double y1 = fr[0], y2 = fr[1], B11 = fr[3], B12 = fr[4], B22 = fr[5], cnt = fr[6];
  for (int k = 0; k < M.K; ++k) th[k] = 0.0;
  const double n = (double)M.H * M.W;
  if (cnt == 0.0) return;
  double A11 = 1.0, A12 = 0.0, A22 = 1.0;
  const double det = B11 * B22 - B12 * B12;
  if (M.d >= 2 && det > 1e-300) {  // A' = B'^{-1}
    A11 = B22 / det;
    A12 = -B12 / det;
    A22 = B11 / det;
  }
  const double detA = A11 * A22 - A12 * A12;
  // ratio of the grain's area (4 |G_i| / n on [-1, 1]^2) to the ellipse area of B'
  const double w = sqrt(fmax(detA, 0.0)) * (4.0 * cnt / n) / M_PI;
  const double Ay1 = A11 * y1 + A12 * y2, Ay2 = A12 * y1 + A22 * y2;
  const double yAy = y1 * Ay1 + y2 * Ay2;
  if (M.d == 1) {  // power diagram: |x|^2 is common to all grains (a gauge term)
    th[0] = y1 * y1 + y2 * y2 - w;
    th[1] = -2.0 * y1;
    th[2] = -2.0 * y2;
    return;
  }
  th[0] = yAy - w + (A11 + A22) / 3.0;
  th[1] = -2.0 * Ay1;
  th[2] = -2.0 * Ay2;
  th[3] = 2.0 * A11 / 3.0;
  th[4] = 2.0 * A12;
  th[5] = 2.0 * A22 / 3.0;
}

// Rows of empty grains := (C, 0, ...), C = 1 + max over non-empty grains of
// sum_k |theta_ik| (a bound of |theta_i . psi| on [-1, 1]^2).  One block per map.
__device__ inline void block_fix_empty(const WarmDev &M, double *th, double *red) {
  const int K = M.K;
  double mx = 0.0;
  for (int i = threadIdx.x; i < M.N; i += PD_BLOCK) {
    if (M.frame[(size_t)i * PD_FRAME_DIM + 6] == 0.0) continue;
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += fabs(th[(size_t)i * K + k]);
    mx = fmax(mx, s);
  }
  const double C = 1.0 + block_max(mx, red);
  for (int i = threadIdx.x; i < M.N; i += PD_BLOCK) {
    if (M.frame[(size_t)i * PD_FRAME_DIM + 6] != 0.0) continue;
    th[(size_t)i * K] = C;
    for (int k = 1; k < K; ++k) th[(size_t)i * K + k] = 0.0;
  }
}

__global__ __launch_bounds__(PD_BLOCK) void kw_heuristic(const WarmDev *__restrict__ W) {
  const WarmDev &M = W[blockIdx.x];
  __shared__ double red[PD_BLOCK];
  for (int i = threadIdx.x; i < M.N; i += PD_BLOCK) heuristic_theta(M, i, M.theta_h + (size_t)i * M.K);
  __syncthreads();
  block_fix_empty(M, M.theta_h, red);
}

// Training targets (one block per map): centred over non-empty grains, divided by
// the root mean square; zero rows for empty grains; lambda = that RMS.
__global__ __launch_bounds__(PD_BLOCK) void kw_targets(const WarmDev *__restrict__ W) {
  const WarmDev &M = W[blockIdx.x];
  const int K = M.K;
  __shared__ double red[PD_BLOCK];
  __shared__ double mean[45];
  double ne = 0.0;
  for (int i = threadIdx.x; i < M.N; i += PD_BLOCK) ne += M.frame[(size_t)i * PD_FRAME_DIM + 6] > 0.0 ? 1.0 : 0.0;
  const double n_live = block_sum(ne, red);
  for (int k = 0; k < K; ++k) {
    double sm = 0.0;
    for (int i = threadIdx.x; i < M.N; i += PD_BLOCK)
      if (M.frame[(size_t)i * PD_FRAME_DIM + 6] > 0.0) sm += M.theta_fit[(size_t)i * K + k];
    const double tot = block_sum(sm, red);
    if (threadIdx.x == 0) mean[k] = n_live > 0.0 ? tot / n_live : 0.0;
  }
  __syncthreads();
  double sq = 0.0;
  for (int i = threadIdx.x; i < M.N; i += PD_BLOCK) {
    if (!(M.frame[(size_t)i * PD_FRAME_DIM + 6] > 0.0)) continue;
    for (int k = 0; k < K; ++k) {
      const double a = M.theta_fit[(size_t)i * K + k] - mean[k];
      sq += a * a;
    }
  }
  const double ss = block_sum(sq, red);
  const double rms = (n_live > 0.0 && ss > 0.0) ? sqrt(ss / (n_live * K)) : 1.0;
  if (threadIdx.x == 0 && M.lambda) *M.lambda = rms;
  for (int i = threadIdx.x; i < M.N; i += PD_BLOCK) {
    const bool live = M.frame[(size_t)i * PD_FRAME_DIM + 6] > 0.0;
    for (int k = 0; k < K; ++k)
      M.target[(size_t)i * K + k] = live ? (float)((M.theta_fit[(size_t)i * K + k] - mean[k]) / rms) : 0.f;
  }
}

// Warm start before scaling (one block per map): network outputs (FP32) centred
// over the non-empty grains, or the moment seed without a network; empty grains
// get the row that wins no pixel.
__global__ __launch_bounds__(PD_BLOCK) void kw_apply(const WarmDev *__restrict__ W) {
  const WarmDev &M = W[blockIdx.x];
  const int K = M.K;
  __shared__ double red[PD_BLOCK];
  if (M.mlp_out == nullptr) {
    for (int j = threadIdx.x; j < M.N * K; j += PD_BLOCK) M.theta_out[j] = M.theta_h[j];
    return;  // the seed already carries the empty-grain rows
  }
  double ne = 0.0;
  for (int i = threadIdx.x; i < M.N; i += PD_BLOCK) ne += M.frame[(size_t)i * PD_FRAME_DIM + 6] > 0.0 ? 1.0 : 0.0;
  const double n_live = block_sum(ne, red);
  for (int k = 0; k < K; ++k) {
    double sm = 0.0;
    for (int i = threadIdx.x; i < M.N; i += PD_BLOCK)
      if (M.frame[(size_t)i * PD_FRAME_DIM + 6] > 0.0) sm += (double)M.mlp_out[(size_t)i * M.out_stride + k];
    const double mean = n_live > 0.0 ? block_sum(sm, red) / n_live : 0.0;
    for (int i = threadIdx.x; i < M.N; i += PD_BLOCK)
      M.theta_out[(size_t)i * K + k] = (double)M.mlp_out[(size_t)i * M.out_stride + k] - mean;
  }
  __syncthreads();
  block_fix_empty(M, M.theta_out, red);
}

// ---------------------------------------------------------------------------
void pd_warm_launch_desc(const WarmDev *W, const int32_t *off, int n_maps, int total_grains,
                         int max_n, hipStream_t s) {
  const int gx = std::min(1024, (max_n + 255) / 256);
  kw_zero<<<dim3(gx, n_maps), 256, 0, s>>>(W, n_maps);
  kw_pass1<<<dim3(1024, n_maps), 256, 0, s>>>(W, n_maps);
  kw_pass2<<<(total_grains + PD_WAVES_PER_BLOCK - 1) / PD_WAVES_PER_BLOCK, PD_BLOCK, 0, s>>>(
      W, off, n_maps, total_grains);
}

void pd_warm_launch_heuristic(const WarmDev *W, int n_maps, hipStream_t s) {
  kw_heuristic<<<n_maps, PD_BLOCK, 0, s>>>(W);
}

void pd_warm_launch_targets(const WarmDev *W, int n_maps, hipStream_t s) {
  kw_targets<<<n_maps, PD_BLOCK, 0, s>>>(W);
}

void pd_warm_launch_apply(const WarmDev *W, int n_maps, hipStream_t s) {
  kw_apply<<<n_maps, PD_BLOCK, 0, s>>>(W);
}
