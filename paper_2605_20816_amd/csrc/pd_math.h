// pd_math.h -- device arithmetic shared by the evaluation kernels: base-2
// exponential and logarithm in the evaluation type, fused multiply-add, maximum.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

template <typename T> __device__ inline T pd_exp2(T x);
template <> __device__ inline float pd_exp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
// FP64 2^t for t <= 0 (the only arguments the kernels form: a logit minus a
// running maximum or minus the log-sum-exp).  Range reduction t = n + f with
// n = rint(t), |f| <= 1/2; 2^f = exp(f ln 2) by its Taylor series
// sum_k (ln 2)^k f^k / k! to degree 13 (truncation error below 2^-58 on
// |f| <= 1/2) in Horner form; 2^n applied exactly by ldexp, which also yields
// the subnormal and zero results.  Arguments below -1100 are clamped (the
// result is 0 either way); NaN propagates through the comparison.
__device__ inline double pd_exp2_nonpos(double t) {
  t = (t < -1100.0) ? -1100.0 : t;
  const double n = __builtin_rint(t);
  const double f = t - n;
  double p = 1.3691488853904124e-12;
  p = __builtin_fma(p, f, 2.5678435993488196e-11);
  p = __builtin_fma(p, f, 4.44553827187081e-10);
  p = __builtin_fma(p, f, 7.054911620801121e-09);
  p = __builtin_fma(p, f, 1.0178086009239696e-07);
  p = __builtin_fma(p, f, 1.3215486790144305e-06);
  p = __builtin_fma(p, f, 1.5252733804059838e-05);
  p = __builtin_fma(p, f, 0.00015403530393381606);
  p = __builtin_fma(p, f, 0.0013333558146428441);
  p = __builtin_fma(p, f, 0.009618129107628477);
  p = __builtin_fma(p, f, 0.055504108664821576);
  p = __builtin_fma(p, f, 0.2402265069591007);
  p = __builtin_fma(p, f, 0.6931471805599453);
  p = __builtin_fma(p, f, 1.0);
  return __builtin_ldexp(p, (int)n);
}
template <> __device__ inline double pd_exp2<double>(double x) { return pd_exp2_nonpos(x); }
template <typename T> __device__ inline T pd_log2(T x);
template <> __device__ inline float pd_log2<float>(float x) { return __builtin_amdgcn_logf(x); }
template <> __device__ inline double pd_log2<double>(double x) { return log2(x); }
__device__ inline float pd_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double pd_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float pd_max(float a, float b) { return fmaxf(a, b); }
__device__ inline double pd_max(double a, double b) { return fmax(a, b); }
