// k_points.hip -- the objective, gradient and hard assignment on unstructured
// point sets in 2-D and 3-D.
//
// Section 2.1 takes the domain as a finite set of points and nothing in the
// method needs a grid or two dimensions; Section 3.3's basis is the tensor
// product of Legendre polynomials, psi_alpha(x) = prod_j P_{alpha_j}(x_j), |alpha|
// <= d.  Without a grid the logit has no separable row form: each pair costs K
// FMAs.  Layout: psi of every point (n x K, FP64, formed once per call), the
// centred base-2 logit coefficients thc = -(log2 e / eps)(theta - mean) (N_pad x
// K), lse and r = 1 - p_G per point, fixed-order partials.
//
//   k_pts_feat    per point: the 1-D values (fused three-term recurrence) and
//                 their products in the degree-graded order
//   k_pts_center  per feature column: grain mean, thc
//   k_pts_lse     wave = 64 points (lanes), loop over grains (thc rows as scalar
//                 loads): online maximum, sum of the other grains' exp2 terms,
//                 lse, r and a per-wave partial of log2 p_G; a grain whose logit
//                 lies PD_SKIP_F64 (PD_SKIP_F32) below every lane's running
//                 maximum adds nothing above rounding and is skipped
//   k_pts_grad    wave = (chunk of points, 64 grains), lanes = grains (thc row
//                 and K accumulators in registers), psi, lse, label and r of each
//                 point as scalar loads; weight p, or -r for the labelled grain
//   k_pts_reduce  Phi and the gradient in a fixed order
//   k_pts_assign  lanes = points, canonical FP64 scores (theta_i0, then one FMA
//                 per feature in index order), smallest index on ties
#include "pd_host.h"
#include "pd_math.h"

#include <math.h>

#include <string>

namespace {

constexpr int PTS_WAVES = PD_WAVES_PER_BLOCK;

// Degree-graded multi-index k of dimension D as (a, b, c) (c = 0 in 2-D).
__host__ __device__ inline void pts_alpha(int D, int d, int kk, int &a, int &b, int &c) {
  int idx = 0;
  for (int k = 0; k <= d; ++k) {
    if (D == 2) {
      for (int bb = 0; bb <= k; ++bb, ++idx)
        if (idx == kk) { a = k - bb; b = bb; c = 0; return; }
    } else {
      for (int cc = 0; cc <= k; ++cc)
        for (int bb = 0; bb <= k - cc; ++bb, ++idx)
          if (idx == kk) { a = k - bb - cc; b = bb; c = cc; return; }
    }
  }
  a = b = c = 0;
}

__device__ inline void pts_legendre(double t, int d, double *P) {
  P[0] = 1.0;
  if (d >= 1) P[1] = t;
  for (int m = 1; m < d; ++m) {
    const double a = (double)(2 * m + 1) * t;
    const double b = (double)m * P[m - 1];
    P[m + 1] = __builtin_fma(a, P[m], -b) / (double)(m + 1);
  }
}

// psi[j*K + k] = (P_a(x_j1) P_b(x_j2)) P_c(x_j3).
__global__ __launch_bounds__(PD_BLOCK) void k_pts_feat(const double *__restrict__ X, long long n,
                                                       int D, int d, int K, double *__restrict__ psi) {
  const long long j = (long long)blockIdx.x * PD_BLOCK + threadIdx.x;
  if (j >= n) return;
  double P[3][PD_POINTS_DMAX2 + 1];
  for (int q = 0; q < D; ++q) pts_legendre(X[j * D + q], d, P[q]);
  for (int k = 0; k < K; ++k) {
    int a, b, c;
    pts_alpha(D, d, k, a, b, c);
    double v = P[0][a] * P[1][b];
    if (D == 3) v = v * P[2][c];
    psi[j * K + k] = v;
  }
}

// grid: K blocks; padded grains get the row (PD_LOGIT_FLOOR, 0, ..., 0) (psi_0 = 1).
__global__ __launch_bounds__(PD_BLOCK) void k_pts_center(const double *__restrict__ theta, int N,
                                                         int Npad, int K, double eps,
                                                         double *__restrict__ thc) {
  const int k = blockIdx.x;
  __shared__ double red[PD_BLOCK];
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += PD_BLOCK) s += theta[(size_t)i * K + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double mean = red[0] / (double)N;
  const double scale = -PD_LOG2E / eps;
  for (int i = threadIdx.x; i < Npad; i += PD_BLOCK)
    thc[(size_t)i * K + k] = i < N ? scale * (theta[(size_t)i * K + k] - mean) : (k == 0 ? PD_LOGIT_FLOOR : 0.0);
}

struct PtsArgs {
  const double *psi, *thc;
  const int32_t *labels;
  long long n;
  int N, Npad;
  double *lse;
  void *r;
  double *part_l;
  double *part_g;
  long long chunk;  // points per gradient wave
  int chunks;
};

template <int K, typename P>
__device__ inline double pts_logit(P t, const double (&p)[K]) {
  // two interleaved chains (psi_0 = 1)
  double v0 = t[0], v1 = 0.0;
#pragma unroll
  for (int k = 1; k < K; k += 2) {
    v0 = pd_fma(t[k], p[k], v0);
    if (k + 1 < K) v1 = pd_fma(t[k + 1], p[k + 1], v1);
  }
  return v0 + v1;
}

template <typename T, int K>
__global__ __launch_bounds__(PD_BLOCK) void k_pts_lse(PtsArgs A) {
  constexpr double SKIP = sizeof(T) == sizeof(double) ? PD_SKIP_F64 : PD_SKIP_F32;
  const int wave = blockIdx.x * PTS_WAVES + threadIdx.x / PD_WAVE;
  const int lane = threadIdx.x % PD_WAVE;
  const long long j0 = (long long)wave * PD_WAVE;
  if (j0 >= A.n) return;
  const long long j = j0 + lane;
  const bool valid = j < A.n;
  const long long jj = valid ? j : A.n - 1;
  double p[K];
  const auto pr = pd_glb(A.psi + jj * K);
#pragma unroll
  for (int k = 0; k < K; ++k) p[k] = pr[k];
  const int g = valid ? pd_glb(A.labels)[j] : -1;
  const auto th = pd_uni(A.thc);
  double mrun = pts_logit<K>(th, p);  // grain 0 sets the reference
  T S = (g == 0) ? (T)0 : (T)1;
  for (int i = 1; i < A.N; ++i) {
    const double s = pts_logit<K>(th + (size_t)i * K, p);
    if (__ballot(!(s <= mrun - SKIP)) == 0) continue;  // far from every lane
    if (s > mrun) {  // a new maximum (rare after the first grains)
      S *= pd_exp2<T>((T)(mrun - s));
      mrun = s;
    }
    const T e = pd_exp2<T>((T)(s - mrun));
    S += (i == g) ? (T)0 : e;
  }
  double ell = 0.0;
  if (valid) {
    const double v = pts_logit<K>(pd_glb(A.thc + (size_t)g * K), p);  // per-lane row
    const T tot = S + pd_exp2<T>((T)(v - mrun));
    const double lse = mrun + (double)pd_log2<T>(tot);
    ell = v - lse;
    pd_glb(A.lse)[j] = lse;
    pd_glb((T *)A.r)[j] = S / tot;
  }
  const double tw = pd_wave_sum(ell);
  if (lane == 0) pd_glb(A.part_l)[wave] = tw;
}

// wave w: grain group w % groups, point chunk w / groups.
template <typename T, int K>
__global__ __launch_bounds__(PD_BLOCK) void k_pts_grad(PtsArgs A) {
  constexpr double SKIP = sizeof(T) == sizeof(double) ? PD_SKIP_F64 : PD_SKIP_F32;
  const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * PTS_WAVES + threadIdx.x / PD_WAVE);
  const int lane = threadIdx.x % PD_WAVE;
  const int groups = A.Npad / PD_WAVE;
  if (wave >= groups * A.chunks) return;
  const int grp = wave % groups, ch = wave / groups;
  const int gbase = grp * PD_WAVE;
  const int i = gbase + lane;
  double t[K], q[K];
  const auto tr = pd_glb(A.thc + (size_t)i * K);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    t[k] = tr[k];
    q[k] = 0.0;
  }
  const long long p0 = (long long)ch * A.chunk;
  const long long p1 = p0 + A.chunk < A.n ? p0 + A.chunk : A.n;
  const auto psu = pd_uni(A.psi);
  const auto lsu = pd_uni(A.lse);
  const auto gsu = pd_uni(A.labels);
  const auto rsu = pd_uni((const T *)A.r);
  for (long long j = p0; j < p1; ++j) {
    const auto pp = psu + j * K;
    double s = t[0] - lsu[j];
    double s1 = 0.0;
#pragma unroll
    for (int k = 1; k < K; k += 2) {
      s = pd_fma(t[k], pp[k], s);
      if (k + 1 < K) s1 = pd_fma(t[k + 1], pp[k + 1], s1);
    }
    s += s1;
    const int g = gsu[j];
    const bool hit = (unsigned)(g - gbase) < (unsigned)PD_WAVE;  // wave-uniform
    if (!hit && __ballot(!(s <= -SKIP)) == 0) continue;  // far from every grain
    const T pv = pd_exp2<T>((T)s);
    const double w = (hit && lane == g - gbase) ? -(double)rsu[j] : (double)pv;
    q[0] += w;
#pragma unroll
    for (int k = 1; k < K; ++k) q[k] = pd_fma(w, pp[k], q[k]);
  }
  const auto out = pd_glb(A.part_g + ((size_t)ch * A.Npad + i) * K);
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = q[k];
}

// Block 0: Phi; blocks 1..: 16 outputs (i, k) x 16 chunk phases each.
__global__ __launch_bounds__(PD_BLOCK) void k_pts_reduce(PtsArgs A, int K, int n_waves,
                                                         double scale, double *phi,
                                                         double *grad) {
  if (blockIdx.x == 0) {
    __shared__ double red[PD_BLOCK];
    double s = 0.0;
    for (int t = threadIdx.x; t < n_waves; t += PD_BLOCK) s += A.part_l[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) *phi = PD_LN2 * red[0] / (double)A.n;
    return;
  }
  if (grad == nullptr) return;
  __shared__ double red2[16][17];
  const int ol = threadIdx.x % 16, ph = threadIdx.x / 16;
  const int o = (blockIdx.x - 1) * 16 + ol;
  const int NK = A.N * K;
  double s = 0.0;
  if (o < NK) {
    const int i = o / K, k = o - i * K;
    for (int c = ph; c < A.chunks; c += 16) s += A.part_g[((size_t)c * A.Npad + i) * K + k];
  }
  red2[ph][ol] = s;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (ph < w) red2[ph][ol] += red2[ph + w][ol];
    __syncthreads();
  }
  if (ph == 0 && o < NK) grad[o] = red2[0][ol] * scale;
}

template <int K>
__global__ __launch_bounds__(PD_BLOCK) void k_pts_assign(const double *__restrict__ psi,
                                                         const double *__restrict__ theta,
                                                         const int32_t *__restrict__ labels,
                                                         long long n, int N,
                                                         int32_t *__restrict__ labels_out,
                                                         long long *__restrict__ part_c) {
  const int wave = blockIdx.x * PTS_WAVES + threadIdx.x / PD_WAVE;
  const int lane = threadIdx.x % PD_WAVE;
  const long long j0 = (long long)wave * PD_WAVE;
  if (j0 >= n) return;
  const long long j = j0 + lane;
  const bool valid = j < n;
  const long long jj = valid ? j : n - 1;
  double p[K];
  const auto pr = pd_glb(psi + jj * K);
#pragma unroll
  for (int k = 0; k < K; ++k) p[k] = pr[k];
  const auto th = pd_uni(theta);
  auto score = [&](int i) {
    const auto t = th + (size_t)i * K;
    double f = t[0];
#pragma unroll
    for (int k = 1; k < K; ++k) f = __builtin_fma(t[k], p[k], f);
    return f;
  };
  int best = 0;
  double fb = score(0);
  bool bad = fb != fb;
  for (int i = 1; i < N; ++i) {
    const double f = score(i);
    bad |= f != f;
    if (f < fb) {
      fb = f;
      best = i;
    }
  }
  const int lab = bad ? -1 : best;
  long long ok = 0;
  if (valid) {
    if (labels_out) pd_glb(labels_out)[j] = lab;
    ok = (labels && lab == pd_glb(labels)[j]) ? 1 : 0;
  }
  const long long wc = pd_wave_sum_i64(ok);
  if (lane == 0) pd_glb(part_c)[wave] = wc;
}

__global__ __launch_bounds__(PD_BLOCK) void k_pts_count(const long long *__restrict__ part_c,
                                                        int n_waves, int64_t *__restrict__ out) {
  __shared__ long long red[PD_BLOCK];
  long long s = 0;
  for (int t = threadIdx.x; t < n_waves; t += PD_BLOCK) s += part_c[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Every feature count a point set can have: 2-D d = 0..7 and 3-D d = 0..4.
#define PTS_DISPATCH_K(kval, CALL)                    \
  switch (kval) {                                     \
    case 1: { constexpr int KK = 1; CALL; } break;    \
    case 3: { constexpr int KK = 3; CALL; } break;    \
    case 4: { constexpr int KK = 4; CALL; } break;    \
    case 6: { constexpr int KK = 6; CALL; } break;    \
    case 10: { constexpr int KK = 10; CALL; } break;  \
    case 15: { constexpr int KK = 15; CALL; } break;  \
    case 20: { constexpr int KK = 20; CALL; } break;  \
    case 21: { constexpr int KK = 21; CALL; } break;  \
    case 28: { constexpr int KK = 28; CALL; } break;  \
    case 35: { constexpr int KK = 35; CALL; } break;  \
    case 36: { constexpr int KK = 36; CALL; } break;  \
    default: break;                                   \
  }

int pts_num_features(int D, int d) {
  return D == 2 ? (d + 1) * (d + 2) / 2 : (d + 1) * (d + 2) * (d + 3) / 6;
}

pd_status pts_check(pd_ctx *ctx, const pd_points &q, int idx) {
  const std::string at = "point set " + std::to_string(idx) + ": ";
  if (q.dim != 2 && q.dim != 3) return pd_fail(ctx, PD_ERR_INVALID_ARG, at + "dim must be 2 or 3");
  const int dmax = q.dim == 2 ? PD_POINTS_DMAX2 : PD_POINTS_DMAX3;
  if (q.degree < 0 || q.degree > dmax)
    return pd_fail(ctx, PD_ERR_UNSUPPORTED, at + "degree must be in [0, " + std::to_string(dmax) + "]");
  if (q.n_points < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, at + "n_points must be >= 1");
  if (q.n_points > ((long long)1 << 40)) return pd_fail(ctx, PD_ERR_INVALID_ARG, at + "n_points too large");
  if (q.n_grains < 2) return pd_fail(ctx, PD_ERR_INVALID_ARG, at + "n_grains must be >= 2");
  if (!(q.eps > 0.0) || !isfinite(q.eps)) return pd_fail(ctx, PD_ERR_INVALID_ARG, at + "eps must be finite and > 0");
  if (!q.coords || !q.labels) return pd_fail(ctx, PD_ERR_INVALID_ARG, at + "coords and labels must be non-NULL");
  return PD_OK;
}

#define PTS_HIP(ctx, expr)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return pd_fail(ctx, PD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

extern "C" int32_t pd_points_num_features(int32_t dim, int32_t degree) {
  if ((dim != 2 && dim != 3) || degree < 0) return 0;
  return pts_num_features(dim, degree);
}

extern "C" pd_status pd_points_objective_grad(pd_ctx *ctx, const pd_points *probs, int32_t n_probs,
                                              const double *const *theta, double *phi_out,
                                              double *const *grad_out, pd_precision prec,
                                              void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (prec != PD_FP64 && prec != PD_FP32)
    return pd_fail(ctx, PD_ERR_UNSUPPORTED, "pd_points_objective_grad: PD_FP64 or PD_FP32");
  if (!probs || n_probs < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 point sets");
  if (!theta || !phi_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta and phi_out must be non-NULL");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pts_check(ctx, probs[p], p);
    if (st != PD_OK) return st;
    if (!theta[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta[" + std::to_string(p) + "] is NULL");
  }
  PTS_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const bool f64 = prec == PD_FP64;
  for (int p = 0; p < n_probs; ++p) {
    const pd_points &q = probs[p];
    const int K = pts_num_features(q.dim, q.degree);
    const int Npad = (q.n_grains + PD_WAVE - 1) / PD_WAVE * PD_WAVE;
    const long long n = q.n_points;
    const int n_waves = (int)((n + PD_WAVE - 1) / PD_WAVE);
    const int groups = Npad / PD_WAVE;
    long long chunks = (8192 + groups - 1) / groups;
    if (chunks > n_waves) chunks = n_waves;
    if (chunks < 1) chunks = 1;
    const long long chunk = (n + chunks - 1) / chunks;
    chunks = (n + chunk - 1) / chunk;
    Arena L;
    const size_t o_psi = L.take(sizeof(double) * (size_t)n * K);
    const size_t o_thc = L.take(sizeof(double) * (size_t)Npad * K);
    const size_t o_lse = L.take(sizeof(double) * (size_t)n);
    const size_t o_r = L.take(sizeof(double) * (size_t)n);
    const size_t o_pl = L.take(sizeof(double) * (size_t)n_waves);
    const size_t o_pg = L.take(grad_out && grad_out[p] ? sizeof(double) * (size_t)chunks * Npad * K : 0);
    pd_status st = pd_reserve(ctx, L.off);
    if (st != PD_OK) return st;
    char *b = ctx->ws;
    PtsArgs A;
    A.psi = (double *)(b + o_psi);
    A.thc = (double *)(b + o_thc);
    A.labels = q.labels;
    A.n = n;
    A.N = q.n_grains;
    A.Npad = Npad;
    A.lse = (double *)(b + o_lse);
    A.r = b + o_r;
    A.part_l = (double *)(b + o_pl);
    A.part_g = (double *)(b + o_pg);
    A.chunk = chunk;
    A.chunks = (int)chunks;
    const unsigned bp = (unsigned)((n + PD_BLOCK - 1) / PD_BLOCK);
    k_pts_feat<<<bp, PD_BLOCK, 0, s>>>(q.coords, n, q.dim, q.degree, K, (double *)A.psi);
    k_pts_center<<<K, PD_BLOCK, 0, s>>>(theta[p], q.n_grains, Npad, K, q.eps, (double *)A.thc);
    const unsigned bl = (unsigned)((n_waves + PTS_WAVES - 1) / PTS_WAVES);
    if (f64) { PTS_DISPATCH_K(K, (k_pts_lse<double, KK><<<bl, PD_BLOCK, 0, s>>>(A))); }
    else { PTS_DISPATCH_K(K, (k_pts_lse<float, KK><<<bl, PD_BLOCK, 0, s>>>(A))); }
    double *g = grad_out ? grad_out[p] : nullptr;
    if (g) {
      const unsigned bg = (unsigned)(((long long)groups * chunks + PTS_WAVES - 1) / PTS_WAVES);
      if (f64) { PTS_DISPATCH_K(K, (k_pts_grad<double, KK><<<bg, PD_BLOCK, 0, s>>>(A))); }
      else { PTS_DISPATCH_K(K, (k_pts_grad<float, KK><<<bg, PD_BLOCK, 0, s>>>(A))); }
    }
    const unsigned br = 1 + (g ? (unsigned)((q.n_grains * K + 15) / 16) : 0);
    k_pts_reduce<<<br, PD_BLOCK, 0, s>>>(A, K, n_waves, 1.0 / (q.eps * (double)n), phi_out + p, g);
    PTS_HIP(ctx, hipGetLastError());
  }
  return PD_OK;
}

extern "C" pd_status pd_points_assign(pd_ctx *ctx, const pd_points *probs, int32_t n_probs,
                                      const double *const *theta, int32_t *const *labels_out,
                                      int64_t *n_correct_out, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!probs || n_probs < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "need n_probs >= 1 point sets");
  if (!theta || !n_correct_out) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta and n_correct_out must be non-NULL");
  for (int p = 0; p < n_probs; ++p) {
    pd_status st = pts_check(ctx, probs[p], p);
    if (st != PD_OK) return st;
    if (!theta[p]) return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta[" + std::to_string(p) + "] is NULL");
  }
  PTS_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  for (int p = 0; p < n_probs; ++p) {
    const pd_points &q = probs[p];
    const int K = pts_num_features(q.dim, q.degree);
    const long long n = q.n_points;
    const int n_waves = (int)((n + PD_WAVE - 1) / PD_WAVE);
    Arena L;
    const size_t o_psi = L.take(sizeof(double) * (size_t)n * K);
    const size_t o_pc = L.take(sizeof(long long) * (size_t)n_waves);
    pd_status st = pd_reserve(ctx, L.off);
    if (st != PD_OK) return st;
    double *psi = (double *)(ctx->ws + o_psi);
    long long *pc = (long long *)(ctx->ws + o_pc);
    const unsigned bp = (unsigned)((n + PD_BLOCK - 1) / PD_BLOCK);
    k_pts_feat<<<bp, PD_BLOCK, 0, s>>>(q.coords, n, q.dim, q.degree, K, psi);
    const unsigned bl = (unsigned)((n_waves + PTS_WAVES - 1) / PTS_WAVES);
    int32_t *lo = labels_out ? labels_out[p] : nullptr;
    PTS_DISPATCH_K(K, (k_pts_assign<KK><<<bl, PD_BLOCK, 0, s>>>(psi, theta[p], q.labels, n, q.n_grains, lo, pc)));
    k_pts_count<<<1, PD_BLOCK, 0, s>>>(pc, n_waves, n_correct_out + p);
    PTS_HIP(ctx, hipGetLastError());
  }
  return PD_OK;
}
