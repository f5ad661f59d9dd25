// pd_math.h -- device arithmetic shared by the evaluation kernels: base-2
// exponential and logarithm in the evaluation type, fused multiply-add, maximum.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

template <typename T> __device__ inline T pd_exp2(T x);
template <> __device__ inline float pd_exp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
// FP64 2^t for finite t <= 1023 or NaN (the kernels form a logit minus a running
// reference or minus the log-sum-exp; padded grains and empty references use a
// large finite floor, never -inf, which would give NaN here).  Range reduction
// t = n + f with n = rint(t), |f| <= 1/2; 2^f by the Chebyshev interpolant of
// degree 11 of 2^f on [-1/2, 1/2] (Chebyshev nodes; its monomial coefficients,
// computed in 50-digit arithmetic by exp2_coefficients.py beside this file;
// interpolation error 3.2e-18 relative) in Horner form with FMAs (at most 0.80
// ulp on 20000 sampled arguments, against 50-digit values); 2^n applied exactly
// by ldexp, which also yields the subnormal and zero results.  n is bounded below
// by -2100 before its integer conversion (every result below 2^-1075 is 0); a NaN
// argument makes f, and with it the result, NaN.
__device__ inline double pd_exp2_f64(double t) {
  const double n = __builtin_rint(t);
  const double f = t - n;
  double p = 4.4558179083360645e-10;
  p = __builtin_fma(p, f, 7.074194297288521e-09);
  p = __builtin_fma(p, f, 1.0178057087733941e-07);
  p = __builtin_fma(p, f, 1.3215432535912375e-06);
  p = __builtin_fma(p, f, 1.5252733841556773e-05);
  p = __builtin_fma(p, f, 0.00015403530463724353);
  p = __builtin_fma(p, f, 0.001333355814640647);
  p = __builtin_fma(p, f, 0.009618129107587256);
  p = __builtin_fma(p, f, 0.055504108664821625);
  p = __builtin_fma(p, f, 0.24022650695910158);
  p = __builtin_fma(p, f, 0.6931471805599453);
  p = __builtin_fma(p, f, 1.0);
  return __builtin_ldexp(p, (int)__builtin_fmax(n, -2100.0));
}
template <> __device__ inline double pd_exp2<double>(double x) { return pd_exp2_f64(x); }
template <typename T> __device__ inline T pd_log2(T x);
template <> __device__ inline float pd_log2<float>(float x) { return __builtin_amdgcn_logf(x); }
template <> __device__ inline double pd_log2<double>(double x) { return log2(x); }
__device__ inline float pd_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double pd_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float pd_max(float a, float b) { return fmaxf(a, b); }
__device__ inline double pd_max(double a, double b) { return fmax(a, b); }
