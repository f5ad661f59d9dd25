// recover.hip -- physical parameters (y, w, A) of a fitted degree-1 or degree-2
// diagram (Section 5.6.3; eq. pd-lr-to-phys and apd-lr-to-phys of Section 2.3.1).
//
// The Legendre coefficients of a grain's score are rewritten in monomials
// (P_2(t) = (3t^2 - 1)/2): h(x) = x.A x + c_lin.x + c_0 with
// A = [[c_xx, c_xy/2], [c_xy/2, c_yy]], and read as y = -(1/2) A^{-1} c_lin,
// w = y.A y - c_0.  Adding lambda (x1^2 + x2^2) to every grain is a common shift
// (Lemma 4.2) that leaves every cell as it is and turns each A_i into
// A_i + lambda I; lambda = max(0, margin - min_i lambda_min(A_i)) makes every
// anisotropy positive definite with smallest eigenvalue >= margin.  At degree 1
// the common |x|^2 is the gauge term already dropped: A_i = I, lambda = 0.
#include "pd_host.h"

#include <math.h>

#include <string>

// Monomial coefficients (c0, cx, cy, cxx, cxy, cyy) of grain i (degree 2).
__device__ inline void rc_monomial(const double *th, double (&c)[6]) {
  c[0] = th[0] - 0.5 * th[3] - 0.5 * th[5];
  c[1] = th[1];
  c[2] = th[2];
  c[3] = 1.5 * th[3];
  c[4] = th[4];
  c[5] = 1.5 * th[5];
}

// Smallest eigenvalue of [[a, b], [b, c]]: (a + c)/2 - sqrt(((a - c)/2)^2 + b^2).
__device__ inline double rc_lmin(double a, double b, double c) {
  const double h = 0.5 * (a - c);
  return 0.5 * (a + c) - sqrt(__builtin_fma(h, h, b * b));
}

// One block: pass 1 takes the smallest eigenvalue over the grains (fixed-order
// tree), pass 2 writes (y1, y2, w, A11, A12, A22) per grain and lambda.
__global__ __launch_bounds__(PD_BLOCK) void k_recover(int N, int d, const double *__restrict__ theta,
                                                      double margin, double *__restrict__ out,
                                                      double *__restrict__ lam_out) {
  const int K = d == 1 ? 3 : 6;
  __shared__ double red[PD_BLOCK];
  double lam = 0.0;
  if (d == 2) {
    double lo = INFINITY;
    for (int i = threadIdx.x; i < N; i += PD_BLOCK) {
      double c[6];
      rc_monomial(theta + (size_t)i * K, c);
      lo = fmin(lo, rc_lmin(c[3], 0.5 * c[4], c[5]));
    }
    red[threadIdx.x] = lo;
    __syncthreads();
    for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    lam = fmax(0.0, margin - red[0]);
  }
  for (int i = threadIdx.x; i < N; i += PD_BLOCK) {
    const double *th = theta + (size_t)i * K;
    double *o = out + (size_t)i * PD_PHYS_DIM;
    if (d == 1) {
      const double y1 = -0.5 * th[1], y2 = -0.5 * th[2];
      o[0] = y1;
      o[1] = y2;
      o[2] = y1 * y1 + y2 * y2 - th[0];
      o[3] = 1.0;
      o[4] = 0.0;
      o[5] = 1.0;
      continue;
    }
    double c[6];
    rc_monomial(th, c);
    const double a = c[3] + lam, b = 0.5 * c[4], e = c[5] + lam;
    const double det = a * e - b * b;
    // y = -(1/2) A^{-1} c_lin with A^{-1} = [[e, -b], [-b, a]] / det
    const double y1 = -0.5 * (e * c[1] - b * c[2]) / det;
    const double y2 = -0.5 * (a * c[2] - b * c[1]) / det;
    o[0] = y1;
    o[1] = y2;
    o[2] = a * y1 * y1 + 2.0 * b * y1 * y2 + e * y2 * y2 - c[0];
    o[3] = a;
    o[4] = b;
    o[5] = e;
  }
  if (threadIdx.x == 0) *lam_out = lam;
}

extern "C" pd_status pd_recover_params(pd_ctx *ctx, int32_t n_grains, int32_t degree,
                                       const double *theta, double margin, double *params_out,
                                       double *lambda_out, void *stream) {
  if (!ctx) return PD_ERR_INVALID_ARG;
  ctx->err.clear();
  if (degree != 1 && degree != 2)
    return pd_fail(ctx, PD_ERR_UNSUPPORTED,
                   "physical parameters exist for degree 1 (power) and 2 (anisotropic) diagrams");
  if (n_grains < 1) return pd_fail(ctx, PD_ERR_INVALID_ARG, "n_grains must be >= 1");
  if (!(margin > 0.0) || !isfinite(margin))
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "margin must be finite and > 0");
  if (!theta || !params_out || !lambda_out)
    return pd_fail(ctx, PD_ERR_INVALID_ARG, "theta, params_out and lambda_out must be non-NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) {
    k_recover<<<1, PD_BLOCK, 0, (hipStream_t)stream>>>(n_grains, degree, theta, margin, params_out,
                                                       lambda_out);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, std::string("k_recover: ") + hipGetErrorString(e));
  return PD_OK;
}
