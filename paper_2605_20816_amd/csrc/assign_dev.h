// assign_dev.h -- the hard arg-min assignment F_theta and its accuracy count
// (Section 2.1, 2.2) for one block of four 64-pixel row segments; used by
// k_assign and by the fit's fused objective/assignment launch.
//
// Lanes = pixels of a 64-pixel row segment, loop over grains.  Scores use one
// canonical FP64 operation order,
//   psi_(a,b) = P_a(x1) * P_b(x2)           (one rounded product)
//   f_i = theta_i0;  f_i = fma(theta_ik, psi_k, f_i), k = 1..K-1
// and the scan keeps the first strict minimum (smallest index on ties), so the
// labels are bit-reproducible.  A NaN score marks the pixel -1.
#pragma once
#include "pd_internal.h"

// A block = 4 waves = 4 row segments of one map (each map's item count is a
// multiple of 4).  theta is staged through LDS in chunks of 64 grains and read
// by all lanes at one address (broadcast); grains are scanned in ascending order.
#define AS_CHUNK 64

// Canonical arg-min over every grain for the pixel (r, c) of each thread, with
// theta staged through sth by the whole block (every thread of the block must
// call it; the pixel may differ per thread and need not be valid).  Returns the
// smallest index among the minimal scores; *bad is set if a score is NaN.
template <int D, bool UNI_ROW>
__device__ inline int canonical_argmin(const MapDev &M, int r, int c, double *sth, bool *bad_out) {
  constexpr int K = (D + 1) * (D + 2) / 2;
  constexpr int DP = D + 1;
  const auto px = pd_glb(M.tx64 + (size_t)c * DP);
  double py[DP];
  if (UNI_ROW) {
    const auto pu = pd_uni(M.ty64 + (size_t)r * DP);
#pragma unroll
    for (int b = 0; b < DP; ++b) py[b] = pu[b];
  } else {
    const auto pv = pd_glb(M.ty64 + (size_t)r * DP);
#pragma unroll
    for (int b = 0; b < DP; ++b) py[b] = pv[b];
  }
  double psi[K];
#pragma unroll
  for (int deg = 0; deg <= D; ++deg)
#pragma unroll
    for (int b = 0; b <= deg; ++b) psi[pd_alpha_index(deg - b, b)] = px[deg - b] * py[b];
  const auto th = pd_glb(M.theta);
  double fbest = INFINITY;
  bool bad = false;
  int best = 0;
  for (int i0 = 0; i0 < M.N; i0 += AS_CHUNK) {
    const int cnt = min(AS_CHUNK, M.N - i0);
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * K; e += PD_BLOCK) sth[e] = th[(size_t)i0 * K + e];
    __syncthreads();
    // four grains at a time (independent FMA chains), compared in index order
    int j = 0;
    for (; j + 4 <= cnt; j += 4) {
      double f[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) f[u] = sth[(j + u) * K];
#pragma unroll
      for (int k = 1; k < K; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) f[u] = __builtin_fma(sth[(j + u) * K + k], psi[k], f[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bad |= __builtin_isnan(f[u]);
        if (f[u] < fbest) {
          fbest = f[u];
          best = i0 + j + u;
        }
      }
    }
    for (; j < cnt; ++j) {
      const double *tj = sth + j * K;
      double f = tj[0];
#pragma unroll
      for (int k = 1; k < K; ++k) f = __builtin_fma(tj[k], psi[k], f);
      bad |= __builtin_isnan(f);
      if (f < fbest) {
        fbest = f;
        best = i0 + j;
      }
    }
  }
  *bad_out = bad;
  return best;
}

template <int D>
__device__ inline void assign_block(const MapDev &M, int base, double *sth) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / PD_WAVE);
  const int lane = threadIdx.x % PD_WAVE;
  const int local = base + wave;
  const bool wave_valid = local < M.rows * M.segs;
  const int lr = wave_valid ? local / M.segs : 0;
  const int r = M.row0 + lr;
  const int c = wave_valid ? (local - lr * M.segs) * PD_WAVE + lane : M.W;
  const bool valid = c < M.W;
  const int cc = valid ? c : M.W - 1;
  bool bad = false;
  const int best = canonical_argmin<D, true>(M, r, cc, sth, &bad);
  long long correct = 0;
  if (valid) {
    const int lab = bad ? -1 : best;
    const size_t jx = (size_t)r * M.W + c;
    if (M.labels_out) pd_glb(M.labels_out)[jx] = lab;
    correct = (lab == pd_glb(M.labels)[jx]) ? 1 : 0;
  }
  // one count per block (its four row segments, in wave order)
  __shared__ long long wcnt[PD_WAVES_PER_BLOCK];
  const long long tot = pd_wave_sum_i64(correct);
  if (lane == 0) wcnt[wave] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long b = 0;
#pragma unroll
    for (int w = 0; w < PD_WAVES_PER_BLOCK; ++w) b += wcnt[w];
    pd_glb(M.part_c)[base / PD_WAVES_PER_BLOCK] = b;
  }
}

