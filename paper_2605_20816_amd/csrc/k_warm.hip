// k_warm.hip -- per-grain descriptors, the moment heuristic start and the
// local/global frame changes of the learned warm start.
//
// Per grain i (pixels G_i, centres x = ((2c+1-W)/W, (2r+1-H)/H)):
//   centroid y'_i and central second moments B'_i (Section 5.6.2, eq.
//   centroid-guess and cov-guess) from exact integer sums of c, r, c^2, c r, r^2;
//   local frame u = (x - y'_i) / r_i with r_i = 2 sqrt(lambda_max(B'_i)) (so an
//   elliptic grain fills [-1, 1]);
//   descriptor (PD_DESC_DIM = 32 floats): log(N |G_i| / n), B'_i / r_i^2 (3),
//   the 27 local Legendre indicator moments mean_{x in G_i} P_a(u_1) P_b(u_2),
//   1 <= a + b <= 6, and log(N) / 10.
// Moment heuristic (Section 5.6.2): A'_i = B'_i^{-1}, w'_i = sqrt(det A'_i)
//   area(G_i) / pi with area(G_i) = 4 |G_i| / n, the grain-to-ellipse area ratio
//   (A' = I at d = 1), converted to Legendre coefficients through
//   x^2 = (2 P_2(x) + 1) / 3; higher-degree coefficients zero.
// Frame change: a polynomial sum_{a+b<=d} c_ab P_a(t_1) P_b(t_2) with
//   t = alpha x + beta per axis is re-expanded in P_a'(x_1) P_b'(x_2) using
//   (alpha x + beta) P_k(x) = alpha ((k+1) P_{k+1} + k P_{k-1}) / (2k+1) + beta P_k
//   inside the three-term recurrence; total degree is preserved.
// The per-grain sums use integer atomics (exact) and one wave per grain over its
// bounding box in a fixed order, so descriptors are bitwise reproducible.
#include "pd_host.h"

#include <math.h>

#include "pd_warm.h"

// 1-D re-expansion: m[a][a'] = coefficient of P_a'(x) in P_a(alpha x + beta), a <= d.
__device__ inline void leg_affine(double alpha, double beta, int d, double (*m)[PD_DMAX + 1]) {
  for (int a = 0; a <= d; ++a)
    for (int k = 0; k <= d; ++k) m[a][k] = 0.0;
  m[0][0] = 1.0;
  if (d >= 1) {
    m[1][0] = beta;
    m[1][1] = alpha;
  }
  for (int a = 1; a < d; ++a) {
    double tp[PD_DMAX + 2];
    for (int k = 0; k <= d + 1; ++k) tp[k] = 0.0;
    for (int k = 0; k <= a; ++k) {  // (alpha x + beta) P_a(t) in the x basis
      const double c = m[a][k];
      if (c == 0.0) continue;
      tp[k] += beta * c;
      tp[k + 1] += alpha * c * (double)(k + 1) / (double)(2 * k + 1);
      if (k >= 1) tp[k - 1] += alpha * c * (double)k / (double)(2 * k + 1);
    }
    for (int k = 0; k <= a + 1; ++k)
      m[a + 1][k] = ((double)(2 * a + 1) * tp[k] - (double)a * m[a - 1][k]) / (double)(a + 1);
  }
}

// out = coefficients in P(x) of sum_ab c_ab P_a(t1) P_b(t2), t_j = al_j x_j + be_j.
__device__ inline void leg_affine_2d(const double *c, int d, double al1, double be1, double al2,
                                     double be2, double *out) {
  double m1[PD_DMAX + 1][PD_DMAX + 1], m2[PD_DMAX + 1][PD_DMAX + 1];
  leg_affine(al1, be1, d, m1);
  leg_affine(al2, be2, d, m2);
  const int K = (d + 1) * (d + 2) / 2;
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  for (int deg = 0; deg <= d; ++deg)
    for (int b = 0; b <= deg; ++b) {
      const int a = deg - b;
      const double cab = c[pd_alpha_index(a, b)];
      if (cab == 0.0) continue;
      for (int a2 = 0; a2 <= a; ++a2)
        for (int b2 = 0; b2 <= b; ++b2) out[pd_alpha_index(a2, b2)] += cab * m1[a][a2] * m2[b][b2];
    }
}

__device__ inline void legendre_d(double t, int d, double *P) {
  P[0] = 1.0;
  if (d >= 1) P[1] = t;
  for (int m = 1; m < d; ++m) P[m + 1] = ((double)(2 * m + 1) * t * P[m] - (double)m * P[m - 1]) / (double)(m + 1);
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
  if (cnt == 0.0) {  // empty grain: neutral descriptor, frame at the origin
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
  // local Legendre moments over the bounding box, fixed order
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
    const double u1 = (((2.0 * c + 1.0 - Wd) / Wd) - y1) / rad;
    const double u2 = (((2.0 * r + 1.0 - Hd) / Hd) - y2) / rad;
    double P1[7], P2[7];
    legendre_d(u1, 6, P1);
    legendre_d(u2, 6, P2);
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
    const double n = Hd * Wd;
    ds[0] = (float)log(cnt * (double)M.N / n);
    ds[1] = (float)(B11 / (rad * rad));
    ds[2] = (float)(B12 / (rad * rad));
    ds[3] = (float)(B22 / (rad * rad));
    for (int q = 0; q < 27; ++q) ds[4 + q] = (float)(acc[q] / cnt);
    ds[31] = (float)(log((double)M.N) / 10.0);
  }
}

// Moment heuristic of Section 5.6.2 in Legendre coefficients (one thread per grain).
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

__global__ void kw_heuristic(const WarmDev *__restrict__ W, int n_maps) {
  const WarmDev &M = W[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M.N; i += gridDim.x * blockDim.x)
    heuristic_theta(M, i, M.theta_h + (size_t)i * M.K);
}

// Training targets (one block per map): the fitted theta is matched to the
// heuristic by a common scale lambda and shift g (least squares over grains),
// Delta_i = (theta_i - g) / lambda - theta'_i, expressed in grain i's local frame.
__global__ __launch_bounds__(PD_BLOCK) void kw_targets(const WarmDev *__restrict__ W) {
  const WarmDev &M = W[blockIdx.x];
  const int K = M.K;
  __shared__ double red[PD_BLOCK];
  __shared__ double mean_t[45], mean_h[45], lam;
  // grain means (fixed-order block sums)
  for (int k = 0; k < K; ++k) {
    for (int pass = 0; pass < 2; ++pass) {
      const double *src = pass ? M.theta_h : M.theta_fit;
      double sm = 0.0;
      for (int i = threadIdx.x; i < M.N; i += PD_BLOCK) sm += src[(size_t)i * K + k];
      red[threadIdx.x] = sm;
      __syncthreads();
      for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      if (threadIdx.x == 0) (pass ? mean_h : mean_t)[k] = red[0] / (double)M.N;
      __syncthreads();
    }
  }
  double num = 0.0, den = 0.0;
  for (int i = threadIdx.x; i < M.N; i += PD_BLOCK)
    for (int k = 0; k < K; ++k) {
      const double a = M.theta_fit[(size_t)i * K + k] - mean_t[k];
      const double b = M.theta_h[(size_t)i * K + k] - mean_h[k];
      num += a * b;
      den += b * b;
    }
  red[threadIdx.x] = num;
  __syncthreads();
  for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double numt = red[0];
  __syncthreads();
  red[threadIdx.x] = den;
  __syncthreads();
  for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lam = (red[0] > 0.0 && numt > 0.0) ? numt / red[0] : 1.0;
    if (M.lambda) *M.lambda = lam;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < M.N; i += PD_BLOCK) {
    double delta[45], loc[45];
    for (int k = 0; k < K; ++k) {
      const double g = mean_t[k] - lam * mean_h[k];
      delta[k] = (M.theta_fit[(size_t)i * K + k] - g) / lam - M.theta_h[(size_t)i * K + k];
    }
    const double *fr = M.frame + (size_t)i * PD_FRAME_DIM;
    // x = y' + r u: re-expand in the Legendre basis of u
    leg_affine_2d(delta, M.d, fr[2], fr[0], fr[2], fr[1], loc);
    for (int k = 0; k < K; ++k) M.target[(size_t)i * K + k] = (float)loc[k];
  }
}

// theta_out_i = theta'_i + (local correction predicted for grain i, taken back to
// the global frame by u = (x - y') / r); theta'_i alone without a network.
__global__ void kw_apply(const WarmDev *__restrict__ W, int n_maps) {
  const WarmDev &M = W[blockIdx.y];
  const int K = M.K;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M.N; i += gridDim.x * blockDim.x) {
    if (M.mlp_out == nullptr || M.frame[(size_t)i * PD_FRAME_DIM + 6] == 0.0) {
      for (int k = 0; k < K; ++k) M.theta_out[(size_t)i * K + k] = M.theta_h[(size_t)i * K + k];
      continue;
    }
    double loc[45], glob[45];
    for (int k = 0; k < K; ++k) loc[k] = (double)M.mlp_out[(size_t)i * M.out_stride + k];
    const double *fr = M.frame + (size_t)i * PD_FRAME_DIM;
    const double r = fr[2];
    leg_affine_2d(loc, M.d, 1.0 / r, -fr[0] / r, 1.0 / r, -fr[1] / r, glob);
    for (int k = 0; k < K; ++k)
      M.theta_out[(size_t)i * K + k] = M.theta_h[(size_t)i * K + k] + glob[k];
  }
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

void pd_warm_launch_heuristic(const WarmDev *W, int n_maps, int max_n, hipStream_t s) {
  kw_heuristic<<<dim3(std::min(1024, (max_n + 255) / 256), n_maps), 256, 0, s>>>(W, n_maps);
}

void pd_warm_launch_targets(const WarmDev *W, int n_maps, hipStream_t s) {
  kw_targets<<<n_maps, PD_BLOCK, 0, s>>>(W);
}

void pd_warm_launch_apply(const WarmDev *W, int n_maps, int max_n, hipStream_t s) {
  kw_apply<<<dim3(std::min(1024, (max_n + 255) / 256), n_maps), 256, 0, s>>>(W, n_maps);
}
