// k_mfma.hip -- BF16 matrix-core objective/gradient path (v_mfma_f32_32x32x16_bf16).
//
// Logits in base 2, s_i(x) = thc_i . psi(x) with thc = -(log2 e / eps)(theta -
// mean), factor over the rows of the grid (the separable Legendre basis):
// s_i(r, c) = sum_a C_a(r, i) P_a(x1_c) with C_a(r, i) = sum_b thc_i(a, b) P_b(x2_r),
// a contraction of inner dimension d + 1 <= 8 per pixel row.  At eps = 1e-3 the
// logits reach |s| ~ 1e3..1e4 while the softmax needs them to ~1e-3, i.e. about
// 22 significant bits, so both operands are split into three bf16 pieces (hi +
// mid + lo, each the rounding of the remainder) and the six products of total
// order <= 2 (hh, hm, mh, hl, lh, mm) are accumulated in FP32; the dropped terms
// are below 2^-26 relative.  Since one operand piece fills only half of the
// instruction's 16-deep inner dimension, each instruction takes two of the six
// products: the lanes of the first half carry one piece pair, those of the
// second half another, so a 32 x 32 tile of logits costs three instructions:
//   [Ym | Yh] x [Xh | Xm] = mh + hm,  [Yl | Yh] x [Xh | Xl] = lh + hl,
//   [Yh | Ym] x [Xh | Xm] = hh + mm    (Y: row coefficients, X: P_a(x1)).
// The gradient contraction sum_x (p_i(x) - delta_{i,G(x)}) psi(x) multiplies
// values of size <= 1: p - delta as two FP16 pieces against the two FP16 pieces
// of psi, on v_mfma_f32_32x32x16_f16.  Log-sum-exp in FP32; Phi and grad Phi are
// summed in FP64 in a fixed order.
//
// Operand/accumulator lane layout of the 32x32x16 instruction (lane l, half
// h = l / 32): A[i][k] at lane i + 32 (k / 8), element k % 8; B[k][j] at lane
// j + 32 (k / 8), element k % 8; D[i][j] at lane j + 32 ((i / 4) % 2),
// register 4 (i / 8) + i % 4.
//
// Pixel tiles are 32 consecutive pixels of one row (ceil(W / 32) per row, the
// last one partial), so a tile has one set of row coefficients.
// k16_lse:  block = one row segment of 16 tiles, tile 4 t + w for wave w; the
//           pieces of C for 256 grains at a time are staged in LDS and shared;
//           S = C X^T puts one pixel per lane column and 16 grains per lane, so
//           the online max / sum of exp2 stays in-lane (halves merged at the end).
// k16_grad: wave = (chunk of whole rows, 64 grains); the C pieces of its grains
//           stay in registers while the chunk stays in one row; S^T = X C^T puts
//           one grain per lane column, so p - delta feeds the gradient product
//           directly as its A operand.  The gradient factors over the rows too:
//           per row G_i(r, a) = sum_c (p - delta)_i(r, c) P_a(x1_c) (inner
//           dimension = pixels, 8 columns a), written per row; k16_reduce forms
//           grad_(a, b) = sum_r P_b(x2_r) G_i(r, a) in FP64.
#include "pd_host.h"

#include <math.h>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#define MF_TILES_PER_WAVE 4     // pixel tiles per wave in k16_lse
#define MF_SEG_TILES 16         // tiles per k16_lse block (one row segment)
#define MF_GRAIN_STAGE 256      // grains staged in LDS per step of k16_lse

// Exponents (a, b) of feature k in the degree-graded order (degree <= 8).
__constant__ signed char c_fa[45] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0,
                                     5, 4, 3, 2, 1, 0, 6, 5, 4, 3, 2, 1, 0,
                                     7, 6, 5, 4, 3, 2, 1, 0, 8, 7, 6, 5, 4, 3, 2, 1, 0};
__constant__ signed char c_fb[45] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4,
                                     0, 1, 2, 3, 4, 5, 0, 1, 2, 3, 4, 5, 6,
                                     0, 1, 2, 3, 4, 5, 6, 7, 0, 1, 2, 3, 4, 5, 6, 7, 8};

__device__ inline float bf_to_f(__bf16 h) { return (float)h; }

// Three-piece split of 8 FP32 values.
__device__ inline void split3(const float (&v)[8], bf16x8 &h, bf16x8 &m, bf16x8 &l) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 a = (__bf16)v[e];
    const float r1 = v[e] - bf_to_f(a);
    const __bf16 b = (__bf16)r1;
    const float r2 = r1 - bf_to_f(b);
    h[e] = a;
    m[e] = b;
    l[e] = (__bf16)r2;
  }
}

// The pixel-side operands of one pixel: P_a(x1) for a <= d (zero beyond, and
// for a pixel outside the row), split in three; xa = [h | m] and xb = [h | l]
// by lane half.
__device__ inline void pixel_operands(const MapDev &M, int c, bool valid, int half, bf16x8 &xa,
                                      bf16x8 &xb) {
  const auto tx = pd_glb((const float *)M.txT);
  float v[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) v[a] = (valid && a <= M.d) ? tx[c * M.DP + a] : 0.f;
  bf16x8 h, m, l;
  split3(v, h, m, l);
  xa = half ? m : h;
  xb = half ? l : h;
}

// acc += the six order <= 2 products of the pieces (small terms first): y1 =
// [m | h], y2 = [l | h], y3 = [h | m] on the row-coefficient side.
__device__ inline f32x16 mfma3(const bf16x8 &y1, const bf16x8 &y2, const bf16x8 &y3,
                               const bf16x8 &xa, const bf16x8 &xb, f32x16 acc, bool y_is_a) {
  if (y_is_a) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(y2, xb, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(y1, xa, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(y3, xa, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xb, y2, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, y1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, y3, acc, 0, 0, 0);
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Rounding bounds of grain i's logits for the certified arg-max of a fit.
// cert_bound16: the FP64 row-factorised logits against the canonical scores (as
// for the FP64 objective: 2D + 8 roundings of the row-coefficient form, K + 4 of
// the canonical dot product, relative to sum |thc| resp. (log2 e / eps) sum
// |theta|, with |P_a| <= 1).  mfma_bound16: the matrix-core logits against the
// exact ones, 2^-17 sum |thc| (piece splitting and dropped products below 2^-24
// of sum |thc|, the FP32 tables 2^-24, at most 48 FP32 roundings in the three
// products: < 2^-18.3).
__device__ inline double cert_bound16(const MapDev &M, int i) {
  const double *th = M.thc + (size_t)i * M.K;
  const double *x = M.theta + (size_t)i * M.K;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < M.K; ++k) {
    a += fabs(th[k]);
    b += fabs(x[k]);
  }
  constexpr double u = 0x1p-53;
  return 2.0 * ((2 * M.d + 8) * u * a + (PD_LOG2E / M.eps) * (M.K + 4) * u * b);
}
__device__ inline float mfma_bound16(const MapDev &M, int i) {
  const double *th = M.thc + (size_t)i * M.K;
  double a = 0.0;
  for (int k = 0; k < M.K; ++k) a += fabs(th[k]);
  return (float)(0x1p-17 * a);
}

// Row coefficients C_a(r, i) = sum_b thc_i(a, b) P_b(x2_r) in FP64 for every
// evaluated row and grain, stored as three bf16 pieces: T3[rr][piece][Npad][8]
// (zero for a > d and for padding grains).  For the certified arg-max of a fit
// (M.cert set) also the FP64 values, C[rr][i][a] (a <= d), and, in the blocks of
// the first row, the largest FP64 rounding bound over the grains (block maximum,
// one atomic per block; the fit clears the slot after each evaluation) and per
// 32-grain tile the largest matrix-core bound (btile).
__global__ __launch_bounds__(PD_BLOCK) void k16_prep(const MapDev *__restrict__ maps,
                                                     const int32_t *__restrict__ off, int n_maps) {
  const int m = pd_find_map(off, n_maps, blockIdx.x);
  const MapDev &M = maps[m];
  if (PD_GATED(M)) return;
  const long long e = (long long)(blockIdx.x - off[m]) * PD_BLOCK + threadIdx.x;
  if (M.cert != nullptr && (long long)(blockIdx.x - off[m]) * PD_BLOCK < M.Npad) {
    __shared__ double bred[PD_BLOCK];
    bred[threadIdx.x] = e < M.N ? cert_bound16(M, (int)e) : 0.0;
    // the tile maximum over 32 consecutive grains (lanes of one wave half; N_pad
    // is a multiple of 64)
    float bt = e < M.N ? mfma_bound16(M, (int)e) : 0.f;
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) bt = fmaxf(bt, __shfl_xor(bt, o, PD_WAVE));
    if (e < M.Npad && (e & 31) == 0) M.btile[e / 32] = bt;
    __syncthreads();
    for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        const double o = bred[threadIdx.x + w];
        // NaN wins (it makes every pixel uncertain, and the canonical pass flags it)
        if (!(o <= bred[threadIdx.x])) bred[threadIdx.x] = o;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0)
      atomicMax((unsigned long long *)M.cert, (unsigned long long)__double_as_longlong(bred[0]));
  }
  if (e >= (long long)M.rows * M.Npad) return;
  const int rr = (int)(e / M.Npad), i = (int)(e - (long long)rr * M.Npad);
  double c[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) c[a] = 0.0;
  if (i < M.N) {
    const double *py = M.ty64 + (size_t)(M.row0 + rr) * M.DP;
    const double *th = M.thc + (size_t)i * M.K;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; a + b < 8; ++b)
        if (a + b <= M.d) c[a] = __builtin_fma(th[(a + b) * (a + b + 1) / 2 + b], py[b], c[a]);
  }
  bf16x8 h, md, lo;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double v = c[a];
    h[a] = (__bf16)(float)v;
    const double r1 = v - (double)bf_to_f(h[a]);
    md[a] = (__bf16)(float)r1;
    lo[a] = (__bf16)(float)(r1 - (double)bf_to_f(md[a]));
  }
  bf16x8 *T = (bf16x8 *)M.T3 + (size_t)rr * 3 * M.Npad + i;
  T[0] = h;
  T[(size_t)M.Npad] = md;
  T[(size_t)2 * M.Npad] = lo;
  if (M.cert != nullptr) {
    double *C = (double *)M.C + (size_t)e * M.DP;
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (a <= M.d) C[a] = c[a];
  }
}

// ---------------------------------------------------------------------------
// With CERT, also the hard assignment of every pixel at this theta, certified
// against the canonical FP64 arg-min (Section 2.1): each lane keeps, per pixel,
// its 16-grain chunk with the largest matrix-core maximum and the largest upper
// bound of the other chunks' exact logits (chunk maximum plus the tile's
// matrix-core bound); at the end the best chunk's 16 logits are formed again in
// FP64 from the FP64 row coefficients.  If the best grain leads the runner-up
// (the chunk's second, the other half's best, or that upper bound) by more than
// twice the FP64 rounding bound of cert_bound16, the canonical scores have the
// same strict minimum there; otherwise the pixel is listed for k_assign_list.
// Per-wave counts of certified correct pixels go to part_c.
template <bool CERT>
__device__ inline void lse16_block(const MapDev &M, int blk, bf16x8 *sT) {
  constexpr int TPW = MF_TILES_PER_WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / PD_WAVE);
  const int lane = threadIdx.x % PD_WAVE;
  const int half = lane / 32, col = lane % 32;
  const int tw = (M.W + 31) / 32, segs = (tw + MF_SEG_TILES - 1) / MF_SEG_TILES;
  const int rr = blk / segs, seg = blk - rr * segs;  // evaluated row, segment
  const int r = M.row0 + rr;
  // B operands: P_a(x1) of this wave's tiles (pixel = column); tile t holds
  // columns (seg * 16 + 4 t + wave) * 32 + col
  bf16x8 xa[TPW], xb[TPW];
  float mrun[TPW], S[TPW];
  int lab[TPW];
  // CERT: the two chunks with the largest matrix-core maxima (maximum, upper
  // bound of the exact logits = maximum plus the tile's matrix-core bound, grain
  // base) and the largest such upper bound of the other chunks
  float bv[TPW], bvu[TPW], b2v[TPW], b2u[TPW], sv[TPW];
  int bi[TPW], b2i[TPW];
  int ntile = 0;  // this wave's tiles that start inside the row (wave-uniform)
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int c0 = (seg * MF_SEG_TILES + 4 * t + wave) * 32;
    const int c = c0 + col;
    const bool valid = c < M.W;
    if (c0 < M.W) ntile = t + 1;
    pixel_operands(M, c, valid, half, xa[t], xb[t]);
    // S sums over the grains other than the pixel's label (r = 1 - p_G, below)
    mrun[t] = -INFINITY;
    S[t] = 0.f;
    bv[t] = -INFINITY;
    bvu[t] = -INFINITY;
    b2v[t] = -INFINITY;
    b2u[t] = -INFINITY;
    sv[t] = -INFINITY;
    bi[t] = -1;
    b2i[t] = -1;
    lab[t] = valid ? pd_glb(M.labels)[(size_t)r * M.W + c] : -1;
  }
  const bf16x8 *T = (const bf16x8 *)M.T3 + (size_t)rr * 3 * M.Npad;
  for (int g0 = 0; g0 < M.Npad; g0 += MF_GRAIN_STAGE) {
    const int gcnt = min(MF_GRAIN_STAGE, M.Npad - g0);
    __syncthreads();
    // stage the three pieces of grains [g0, g0 + gcnt): sT[piece][g]
    for (int w = threadIdx.x; w < 3 * gcnt; w += PD_BLOCK) {
      const int piece = w / gcnt, q = w - piece * gcnt;
      sT[piece * MF_GRAIN_STAGE + q] = T[(size_t)piece * M.Npad + g0 + q];
    }
    __syncthreads();
    if (ntile == 0) continue;
    for (int gt = 0; gt < gcnt; gt += 32) {
      const bf16x8 *sg = sT + gt + col;
      const bf16x8 yh = sg[0], ym = sg[MF_GRAIN_STAGE], yl = sg[2 * MF_GRAIN_STAGE];
      const bf16x8 y1 = half ? yh : ym, y2 = half ? yh : yl, y3 = half ? ym : yh;
      const int gbase = g0 + gt;
      const bool partial = gbase + 32 > M.N;
      const float btl = CERT ? pd_uni(M.btile)[gbase / 32] : 0.f;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        if (t >= ntile) break;
        f32x16 acc;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.f;
        acc = mfma3(y1, y2, y3, xa[t], xb[t], acc, true);
        if (partial) {
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const int g = gbase + (j / 4) * 8 + half * 4 + (j % 4);
            if (g >= M.N) acc[j] = -INFINITY;
          }
        }
        float cm = acc[0];
#pragma unroll
        for (int j = 1; j < 16; ++j) cm = fmaxf(cm, acc[j]);
        // rows that are all padding grains (-inf) contribute nothing; skipping them
        // also avoids exp2(-inf - (-inf)) while this lane's maximum is still -inf
        if (cm == -INFINITY) continue;
        if constexpr (CERT) {
          const float cu = cm + btl;
          const bool gt1 = cm > bv[t];
          const bool gt2 = !gt1 && cm > b2v[t];
          sv[t] = fmaxf(sv[t], (gt1 || gt2) ? b2u[t] : cu);
          b2v[t] = gt1 ? bv[t] : (gt2 ? cm : b2v[t]);
          b2u[t] = gt1 ? bvu[t] : (gt2 ? cu : b2u[t]);
          b2i[t] = gt1 ? bi[t] : (gt2 ? gbase : b2i[t]);
          bv[t] = gt1 ? cm : bv[t];
          bvu[t] = gt1 ? cu : bvu[t];
          bi[t] = gt1 ? gbase : bi[t];
        }
        const float mn = fmaxf(mrun[t], cm);
        float s = S[t] * __builtin_amdgcn_exp2f(mrun[t] - mn);
        if (__ballot((unsigned)(lab[t] - gbase) < 32u) != 0) {
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const int g = gbase + (j / 4) * 8 + half * 4 + (j % 4);
            const float e = __builtin_amdgcn_exp2f(acc[j] - mn);
            s += g == lab[t] ? 0.f : e;
          }
        } else {
#pragma unroll
          for (int j = 0; j < 16; ++j) s += __builtin_amdgcn_exp2f(acc[j] - mn);
        }
        S[t] = s;
        mrun[t] = mn;
      }
    }
  }
  // merge the two halves (lanes l and l + 32 hold the same pixel)
  double ell = 0.0;
  long long n_ok = 0;
  const double bound =
      CERT ? __longlong_as_double((long long)*pd_uni((const unsigned long long *)M.cert)) : 0.0;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    if constexpr (CERT) {
      const int c = (seg * MF_SEG_TILES + 4 * t + wave) * 32 + col;
      const bool valid = c < M.W;
      // FP64 logits of this lane's two best chunks: grains base + 8 (j / 4) +
      // 4 half + j % 4; v1 (grain j1) and v2 the largest two of them
      double v1 = -INFINITY, v2 = -INFINITY;
      int j1 = -1;
      if (valid) {
        const double *px = M.tx64 + (size_t)c * M.DP;
        double pa[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) pa[a] = a <= M.d ? px[a] : 0.0;
        const double *C = (const double *)M.C + (size_t)rr * M.Npad * M.DP;
#pragma unroll 1
        for (int q = 0; q < 32; ++q) {
          const int base = q < 16 ? bi[t] : b2i[t];
          const int j = q & 15;
          const int g = base + (j / 4) * 8 + half * 4 + (j % 4);
          if (base < 0 || g >= M.N) continue;
          const double *cp = C + (size_t)g * M.DP;
          double v = cp[0];
#pragma unroll
          for (int a = 1; a < 8; ++a)
            if (a <= M.d) v = __builtin_fma(cp[a], pa[a], v);
          if (v > v1) {
            v2 = v1;
            v1 = v;
            j1 = g;
          } else {
            v2 = fmax(v2, v);
          }
        }
      }
      const double v1o = __shfl_xor(v1, 32, PD_WAVE), v2o = __shfl_xor(v2, 32, PD_WAVE);
      const int j1o = __shfl_xor(j1, 32, PD_WAVE);
      const float svo = __shfl_xor(sv[t], 32, PD_WAVE);
      const bool mine = v1 >= v1o;
      const double top = mine ? v1 : v1o;
      const int jt = mine ? j1 : j1o;
      const double run = fmax(mine ? v2 : v2o, mine ? v1o : v1);
      const double others = (double)fmaxf(sv[t], svo);
      const bool sure = (top - fmax(run, others)) > 2.0 * bound;  // false for NaN
      const bool act = half == 0 && valid;
      n_ok += (act && sure && jt == lab[t]) ? 1 : 0;
      const bool unsure = act && !sure;
      const unsigned long long um = __ballot(unsure);
      if (um != 0) {
        int base = 0;
        if (lane == 0) base = atomicAdd(M.unc_count, __popcll(um));
        base = __shfl(base, 0, PD_WAVE);
        const int pos = base + __popcll(um & ((1ull << lane) - 1ull));
        if (unsure && pos < M.rows * M.W) pd_glb(M.unc_list)[pos] = r * M.W + c;
      }
    }
    const float mo = __shfl_xor(mrun[t], 32, PD_WAVE);
    const float so = __shfl_xor(S[t], 32, PD_WAVE);
    const float mm = fmaxf(mrun[t], mo);
    // the other grains' sum (both halves), then the label's own term
    const float sx = S[t] * __builtin_amdgcn_exp2f(mrun[t] - mm) + so * __builtin_amdgcn_exp2f(mo - mm);
    const int c = (seg * MF_SEG_TILES + 4 * t + wave) * 32 + col;
    if (half == 0 && c < M.W) {
      const size_t p = (size_t)rr * M.W + c;  // index among the evaluated pixels
      float lse, rr_p = 0.f;
      const int g = lab[t];
      if (g >= 0 && g < M.N) {
        // exact FP64 logit of the true grain
        const double *px = M.tx64 + (size_t)c * M.DP, *py = M.ty64 + (size_t)r * M.DP;
        const double *th = M.thc + (size_t)g * M.K;
        double sg = 0.0;
        for (int k = 0; k < M.K; ++k) sg = __builtin_fma(th[k], px[c_fa[k]] * py[c_fb[k]], sg);
        const float tot = sx + __builtin_amdgcn_exp2f((float)(sg - (double)mm));
        lse = mm + __builtin_amdgcn_logf(tot);
        rr_p = sx / tot;
        ell += sg - (double)lse;
      } else {
        lse = mm + __builtin_amdgcn_logf(sx);
        ell = NAN;
      }
      pd_glb(M.lse32)[p] = lse;
      pd_glb((float *)M.rpix)[p] = rr_p;
    }
  }
  const double tot_l = pd_wave_sum(ell);
  if (lane == 0) pd_glb(M.part_l)[blk * 4 + wave] = tot_l;
  if constexpr (CERT) {
    const long long wc = pd_wave_sum_i64(n_ok);
    if (lane == 0) pd_glb(M.part_c)[blk * 4 + wave] = wc;
  }
}

// Occupancy: the objective runs 4 waves per SIMD (128 VGPRs; the few spills are
// loop-invariant values read back once per LDS stage and in the epilogue), the
// gradient 3 (168 VGPRs; the spilled output addresses are read back once per
// row).  Both kernels are latency-bound at the compiler's own choice of 2 waves:
// at c5 (2048^2, 4928 grains, d = 6) the forced occupancy takes the objective
// from 4.6 to 3.4 ms and the gradient from 10.5 to 8.2 ms.
template <bool CERT>
__global__ __launch_bounds__(PD_BLOCK) __attribute__((amdgpu_waves_per_eu(4, 4))) void k16_lse(const MapDev *__restrict__ maps,
                                                    const int32_t *__restrict__ off, int n_maps,
                                                    int total) {
  __shared__ bf16x8 sT[3 * MF_GRAIN_STAGE];
  if ((int)blockIdx.x >= total) return;
  const int m = pd_find_map(off, n_maps, blockIdx.x);
  const MapDev &M = maps[m];
  if (PD_GATED(M)) return;
  lse16_block<CERT>(M, blockIdx.x - off[m], sT);
}

// ---------------------------------------------------------------------------
// k16_grad: block = 4 waves on one pixel chunk, wave w on grain group 4 q + w.
// Per 32-pixel tile the four waves build the shared operands once in LDS (two
// buffers: tile t + 1 is built while tile t's products run):
//   sX  [2][64]      x 16 B : P_a(x1) pieces [h|m], [h|l] (pixel = row) for the
//                             logit product
//   sQ  [2][2][64]   x 16 B : P_a(x1) of the tile's pixels as the B operands of
//                             the gradient product, per 16-pixel block kb2 (inner
//                             index h*8+e = pixel 16 kb2 + 8 (e / 4) + 4 h + e % 4):
//                             columns [P_hi | P_lo | 0 | 0] and [0 | 0 | P_hi | 0]
//                             (8 columns a each, FP16 pieces)
//   sL, sR, sG [32]         : lse - PD_MF_WSHIFT, r = 1 - p_G and label of the
//                             tile's pixels
// The gradient product takes the weight p (other grains) or -r (the pixel's
// own grain: p - 1 without the cancellation near p = 1) as two FP16 pieces
// (hi + lo, about 22 bits), scaled by 2^PD_MF_WSHIFT so that small weights stay
// normal, against the two FP16 pieces of P_a: w_hi P_hi and w_hi P_lo in one
// instruction (columns 0-7 and 8-15), w_lo P_hi in another (columns 16-23); the
// three column groups are added at the end of each row and the scale taken out.
// One FP16 piece (2^-12 relative per weight) put the gradient at a fitted
// iterate, where p - delta cancels most, at the edge of a 2e-3 tolerance.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

#define PD_MF_WSHIFT 12
struct GradLds {
  bf16x8 X[2][64];
  f16x8 Q[2][2][64];
  float L[32];
  float R[32];
  int G[32];
  int lo, hi;
};

__device__ inline void grad16_block(const MapDev &M, int local_blk, GradLds (&sh)[2]) {
  constexpr int GT = PD_MF_GROUP_TILES;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / PD_WAVE);
  const int lane = threadIdx.x % PD_WAVE;
  const int half = lane / 32, col = lane % 32;
  const int qb = (M.ggroups + 3) / 4;  // blocks of 4 grain groups per chunk
  const int chunk = local_blk / qb;
  const int grp = (local_blk - chunk * qb) * 4 + wave;
  const bool active = grp < M.ggroups;
  const int g0 = min(grp, M.ggroups - 1) * (GT * 32);
  const int gtn = min(GT, (M.Npad - g0) / 32);
  const int tw = (M.W + 31) / 32;  // tiles per row
  // row-coefficient operands of this wave's grains, for the row cur_rr
  bf16x8 y1[GT], y2[GT], y3[GT];
  int cur_rr = -1;
  auto load_rowc = [&](int rr) {
    const bf16x8 *T = (const bf16x8 *)M.T3 + (size_t)rr * 3 * M.Npad;
#pragma unroll
    for (int t = 0; t < GT; ++t) {
      const int g = min(g0 + t * 32 + col, M.Npad - 1);
      const bf16x8 yh = T[g], ym = T[(size_t)M.Npad + g], yl = T[(size_t)2 * M.Npad + g];
      y1[t] = half ? yh : ym;
      y2[t] = half ? yh : yl;
      y3[t] = half ? ym : yh;
    }
  };
  f32x16 accg[GT];
#pragma unroll
  for (int t = 0; t < GT; ++t)
#pragma unroll
    for (int j = 0; j < 16; ++j) accg[t][j] = 0.f;
  const int pt0 = chunk * M.chunk_tiles;
  const int pt1 = min(pt0 + M.chunk_tiles, M.tiles32);
  // this lane's column of the gradient product: a = col % 8 in group col / 8
  const int qa = col & 7, qgrp = col >> 3;
  const bool qvalid = qgrp < 3 && qa <= M.d;
  const float *txf = (const float *)M.txT;
  auto compute_tile = [&](const GradLds &S) {
    const bf16x8 xa = S.X[0][lane], xb = S.X[1][lane];
    // the logits exactly as k16_lse formed them (the same products from zero, so
    // that the weights are those of its log-sum-exp); S.L holds lse - PD_MF_WSHIFT
    // (exact in FP32), so exp2 gives the weight p scaled by 2^PD_MF_WSHIFT
    float lrow[16];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) lrow[4 * b + r] = S.L[8 * b + 4 * half + r];
    f32x16 acc[GT];
#pragma unroll
    for (int t = 0; t < GT; ++t) {
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[t][j] = 0.f;
      acc[t] = mfma3(y1[t], y2[t], y3[t], xa, xb, acc[t], false);
    }
#pragma unroll
    for (int t = 0; t < GT; ++t)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[t][j] = __builtin_amdgcn_exp2f(acc[t][j] - lrow[j]);
    if (S.hi >= g0 && S.lo < g0 + GT * 32) {
      constexpr float wscale = (float)(1 << PD_MF_WSHIFT);
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gr = S.G[8 * b + 4 * half + r];
          const float rv = -S.R[8 * b + 4 * half + r] * wscale;
#pragma unroll
          for (int t = 0; t < GT; ++t)
            acc[t][4 * b + r] = (gr == g0 + t * 32 + col) ? rv : acc[t][4 * b + r];
        }
    }
#pragma unroll
    for (int kb2 = 0; kb2 < 2; ++kb2) {
      const f16x8 qa_op = S.Q[kb2][0][lane], qb = S.Q[kb2][1][lane];
      f16x8 x[GT], xl[GT];
#pragma unroll
      for (int t = 0; t < GT; ++t)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          // two FP16 pieces of the FP32 weight: the high one is the weight with
          // its 13 low significand bits cleared (11 bits, exact in FP16 for
          // |q| <= 2^12 down to 2^-14), the low one the exact FP32 remainder
          // rounded to FP16
          const float q = acc[t][8 * kb2 + e];
          const float qh = __uint_as_float(__float_as_uint(q) & 0xffffe000u);
          x[t][e] = (_Float16)qh;
          xl[t][e] = (_Float16)(q - qh);
        }
      // (w_hi + w_lo)(psi_hi + psi_lo) without w_lo psi_lo, small terms first
      // w_lo P_hi (columns 16-23), then w_hi P_hi and w_hi P_lo (columns 0-15)
#pragma unroll
      for (int t = 0; t < GT; ++t) accg[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(xl[t], qb, accg[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < GT; ++t) accg[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(x[t], qa_op, accg[t], 0, 0, 0);
    }
  };
  // Per tile the waves' roles: wave 0 the P_a(x1) pieces, waves 1-2 the psi^T
  // pieces, wave 3 lse and labels.  The global data of tile pt + 1 is loaded
  // before tile pt's products and written to the other LDS buffer after them, so
  // one barrier per tile separates building from use.
  // the loaded values of the next tile, by role: wave 0 P_a(x1) of its pixel,
  // waves 1-2 P_a(x1) of 8 pixels, wave 3 lse, r and label of one pixel
  float pre[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) pre[e] = 0.f;
  auto load_tile = [&](int pt) {
    const int rr = pt / tw;
    const int c0 = (pt - rr * tw) * 32;
    const int r = M.row0 + rr;
    if (wave == 0) {
      const int c = c0 + col;
      const bool ok = c < M.W;
#pragma unroll
      for (int a = 0; a < 8; ++a) pre[a] = (ok && a <= M.d) ? pd_glb(txf)[c * M.DP + a] : 0.f;
    } else if (wave <= 2) {
      const int kb2 = wave - 1;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = c0 + 16 * kb2 + 8 * (e / 4) + 4 * half + (e % 4);
        const bool ok = qvalid && c < M.W;
        pre[e] = ok ? pd_glb(txf)[c * M.DP + qa] : 0.f;
      }
    } else if (lane < 32) {
      const int c = c0 + lane;
      const bool ok = c < M.W;
      const size_t p = (size_t)rr * M.W + c;
      // pixels past the row's end: lse = +inf gives them weight 0
      pre[0] = ok ? pd_glb(M.lse32)[p] : INFINITY;
      pre[1] = ok ? pd_glb((const float *)M.rpix)[p] : 0.f;
      pre[2] = __int_as_float(ok ? pd_glb(M.labels)[(size_t)r * M.W + c] : -1);
    }
  };
  auto build_tile = [&](GradLds &S) {
    if (wave == 0) {
      bf16x8 h, m, l;
      split3(pre, h, m, l);
      S.X[0][lane] = half ? m : h;
      S.X[1][lane] = half ? l : h;
    } else if (wave <= 2) {
      const int kb2 = wave - 1;
      f16x8 qa8, qb8;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        // the two FP16 pieces of the FP32 table value P_a(x1)
        const float v = pre[e];
        const _Float16 h = (_Float16)v;
        const _Float16 l = (_Float16)(v - (float)h);
        const _Float16 z = (_Float16)0.f;
        qa8[e] = qgrp == 0 ? h : (qgrp == 1 ? l : z);
        qb8[e] = qgrp == 2 ? h : z;
      }
      S.Q[kb2][0][lane] = qa8;
      S.Q[kb2][1][lane] = qb8;
    } else {
      int g = -1, lo = 0x7fffffff, hi = -1;
      if (lane < 32) {
        S.L[lane] = pre[0] - (float)PD_MF_WSHIFT;
        S.R[lane] = pre[1];
        g = __float_as_int(pre[2]);
        S.G[lane] = g;
        if (g >= 0) lo = hi = g;
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, PD_WAVE));
        hi = max(hi, __shfl_xor(hi, o, PD_WAVE));
      }
      if (lane == 0) {
        S.lo = lo;
        S.hi = hi;
      }
    }
  };
  if (pt0 < pt1) {
    load_tile(pt0);
    build_tile(sh[0]);
  }
  // G of row rr for this wave's grains: column groups added (lanes col, col + 8,
  // col + 16), the scale taken out, written by the lanes col < 8; then cleared
  auto flush_row = [&](int rr) {
    float *out = M.part_g32 + (size_t)rr * M.Npad * 8;
#pragma unroll
    for (int t = 0; t < GT; ++t) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const float v = accg[t][j];
        const float s1 = __shfl_down(v, 8, PD_WAVE), s2 = __shfl_down(v, 16, PD_WAVE);
        const int g = g0 + t * 32 + (j / 4) * 8 + half * 4 + (j % 4);
        if (col < 8 && t < gtn)
          pd_glb(out)[(size_t)g * 8 + col] = ((v + s1) + s2) * (1.f / (float)(1 << PD_MF_WSHIFT));
        accg[t][j] = 0.f;
      }
    }
  };
  for (int pt = pt0; pt < pt1; ++pt) {
    GradLds &cur = sh[(pt - pt0) & 1];
    const int rr = pt / tw;
    if (active && rr != cur_rr) {
      load_rowc(rr);  // the chunk entered a new row (in flight across the barrier)
      cur_rr = rr;
    }
    if (pt + 1 < pt1) load_tile(pt + 1);
    __syncthreads();  // cur is built; the other buffer's readers (tile pt - 1) are done
    if (active) {
      compute_tile(cur);
      if (pt + 1 == pt1 || (pt + 1) / tw != rr) flush_row(rr);  // the row's last tile
    }
    if (pt + 1 < pt1) build_tile(sh[(pt - pt0 + 1) & 1]);
  }
}

__global__ __launch_bounds__(PD_BLOCK) __attribute__((amdgpu_waves_per_eu(3, 3))) void k16_grad(const MapDev *__restrict__ maps,
                                                     const int32_t *__restrict__ off, int n_maps,
                                                     int total) {
  __shared__ GradLds sh[2];
  if ((int)blockIdx.x >= total) return;
  const int m = pd_find_map(off, n_maps, blockIdx.x);
  const MapDev &M = maps[m];
  if (PD_GATED(M)) return;
  grad16_block(M, blockIdx.x - off[m], sh);
}

// Phi from the per-wave partials; grad_(a, b) of grain i = sum_r P_b(x2_r)
// G_i(r, a) in FP64 from the row partials: block = 8 grains x 32 row phases
// (rows r = phase mod 32 in order, then a fixed butterfly over the phases).
__global__ __launch_bounds__(PD_BLOCK) void k16_reduce(const MapDev *__restrict__ maps,
                                                       const int32_t *__restrict__ off, int n_maps) {
  if ((int)blockIdx.x < n_maps) {
    const MapDev &M = maps[blockIdx.x];
    if (PD_GATED(M)) return;
    __shared__ double red[PD_BLOCK];
    double s = 0.0;
    for (int t = threadIdx.x; t < M.a16_items * 4; t += PD_BLOCK) s += M.part_l[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = PD_BLOCK / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) *M.phi = PD_LN2 * red[0] / ((double)M.H * (double)M.W);
    return;
  }
  const int b = blockIdx.x - n_maps;
  const int m = pd_find_map(off, n_maps, b);
  const MapDev &M = maps[m];
  if (M.grad == nullptr || PD_GATED(M)) return;
  const int i = (b - off[m]) * 8 + (int)threadIdx.x / 32, ph = threadIdx.x % 32;
  double acc[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) acc[k] = 0.0;
  if (i < M.N) {
    for (int rr = ph; rr < M.rows; rr += 32) {
      typedef float f32x4 __attribute__((ext_vector_type(4)));
      const auto gp = pd_glb((const f32x4 *)(M.part_g32 + ((size_t)rr * M.Npad + i) * 8));
      const f32x4 ga = gp[0], gb = gp[1];
      const float gv[8] = {ga[0], ga[1], ga[2], ga[3], gb[0], gb[1], gb[2], gb[3]};
      const double *py = M.ty64 + (size_t)(M.row0 + rr) * M.DP;
#pragma unroll
      for (int a = 0; a < 7; ++a)
#pragma unroll
        for (int bb = 0; a + bb < 7; ++bb)
          if (a + bb <= M.d) {
            const int k = (a + bb) * (a + bb + 1) / 2 + bb;
            acc[k] = __builtin_fma((double)gv[a], py[bb], acc[k]);
          }
    }
  }
#pragma unroll
  for (int k = 0; k < 28; ++k) {
    double v = acc[k];
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, PD_WAVE);
    if (ph == 0 && i < M.N && k < M.K) M.grad[(size_t)i * M.K + k] = v * (M.grad_scale * M.grad_sign);
  }
}

// ---------------------------------------------------------------------------
// Fallback of the certified arg-max of a BF16 fit.  Late in a fit sum |thc| can
// grow so large that the matrix-core bound of k16_lse exceeds the logit gaps at
// most pixels; then every pixel is decided again from the FP64 row coefficients
// alone (d + 1 FMAs per pair, FP64 bound), so that only the few pixels that
// this leaves undecided go to the canonical scan.  The flag (bytes 12..15 of the
// certificate slot) is set by k16_recheck_gate when k16_lse left more than 1/16
// of the map's pixels undecided; the gate also clears the list for the new pass
// and zeroes the count slots that neither pass writes.
__global__ void k16_recheck_gate(const MapDev *__restrict__ maps, int n_maps) {
  const MapDev &M = maps[blockIdx.x];
  if ((int)blockIdx.x >= n_maps || PD_GATED(M) || M.cert == nullptr) return;
  int32_t *flag = (int32_t *)((char *)M.cert + 12);
  const long long n_px = (long long)M.rows * M.W;
  const bool redo = (long long)*M.unc_count > (n_px >> 4);
  __syncthreads();  // every thread has read the count
  const int c_items = max(M.a_items, 4 * M.a16_items);
  for (int t = (redo ? M.a_items : 4 * M.a16_items) + threadIdx.x; t < c_items; t += blockDim.x)
    M.part_c[t] = 0;
  if (threadIdx.x == 0) {
    *flag = redo ? 1 : 0;
    if (redo) *M.unc_count = 0;
  }
}

// One wave per 64-pixel row segment (the FP64 objective's work list), lanes =
// pixels: the logits of grains in chunks of 8 from the FP64 row coefficients
// (wave-uniform loads), the largest chunk maximum, its chunk and the largest of
// the others; then the best chunk again, and the gap to the runner-up against
// twice the FP64 bound of cert_bound16.
template <int D>
__device__ inline void recert_item(const MapDev &M, int local, int lane) {
  constexpr int DP = D + 1;
  if (local >= M.rows * M.segs) {
    if (lane == 0) pd_glb(M.part_c)[local] = 0;
    return;
  }
  const int lr = local / M.segs;
  const int r = M.row0 + lr;
  const int c = (local - lr * M.segs) * PD_WAVE + lane;
  const bool valid = c < M.W;
  const int cc = valid ? c : M.W - 1;
  double px[DP];
#pragma unroll
  for (int a = 0; a < DP; ++a) px[a] = M.tx64[(size_t)cc * DP + a];
  const auto Crow = pd_uni((const double *)M.C + (size_t)lr * M.Npad * DP);
  const int g = valid ? pd_glb(M.labels)[(size_t)r * M.W + c] : -1;
  auto logit = [&](int i) {
    const auto cp = Crow + (size_t)i * DP;
    double v = cp[0];
#pragma unroll
    for (int a = 1; a < DP; ++a) v = __builtin_fma(cp[a], px[a], v);
    return v;
  };
  double bv = -INFINITY, sv = -INFINITY;
  int bi = 0;
  const int nfull = M.N & ~7;
  for (int i0 = 0; i0 < M.N; i0 += 8) {
    double cm = -INFINITY;
    if (i0 < nfull) {
#pragma unroll
      for (int j = 0; j < 8; ++j) cm = fmax(cm, logit(i0 + j));
    } else {
      for (int j = 0; i0 + j < M.N; ++j) cm = fmax(cm, logit(i0 + j));
    }
    const bool gt = cm > bv;
    sv = gt ? bv : fmax(sv, cm);
    bi = gt ? i0 : bi;
    bv = gt ? cm : bv;
  }
  double v1 = -INFINITY, v2 = -INFINITY;
  int j1 = -1;
#pragma unroll 1
  for (int j = 0; j < 8; ++j) {
    if (bi + j >= M.N) break;
    const double v = logit(bi + j);
    if (v > v1) {
      v2 = v1;
      v1 = v;
      j1 = bi + j;
    } else {
      v2 = fmax(v2, v);
    }
  }
  const double bound = __longlong_as_double((long long)*pd_uni((const unsigned long long *)M.cert));
  const bool sure = (v1 - fmax(v2, sv)) > 2.0 * bound;  // false for NaN
  const long long ok = (valid && sure && j1 == g) ? 1 : 0;
  const bool unsure = valid && !sure;
  const unsigned long long um = __ballot(unsure);
  if (um != 0) {
    int base = 0;
    if (lane == 0) base = atomicAdd(M.unc_count, __popcll(um));
    base = __shfl(base, 0, PD_WAVE);
    const int pos = base + __popcll(um & ((1ull << lane) - 1ull));
    if (unsure && pos < M.rows * M.W) pd_glb(M.unc_list)[pos] = r * M.W + c;
  }
  const long long wc = pd_wave_sum_i64(ok);
  if (lane == 0) pd_glb(M.part_c)[local] = wc;
}

template <int DMAX>
__global__ __launch_bounds__(PD_BLOCK) void k16_recert(const MapDev *__restrict__ maps,
                                                       const int32_t *__restrict__ off,
                                                       int n_maps, int total) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / PD_WAVE);
  const int lane = threadIdx.x % PD_WAVE;
  const int item = pd_xcd_block(blockIdx.x, gridDim.x) * PD_WAVES_PER_BLOCK + wave;
  if (item >= total) return;
  const int m = pd_find_map(off, n_maps, item);
  const MapDev &M = maps[m];
  if (PD_GATED(M) || M.cert == nullptr) return;
  if (*pd_uni((const int32_t *)((const char *)M.cert + 12)) == 0) return;
  PD_DISPATCH_UPTO(DMAX, M.d, (recert_item<D>(M, item - off[m], lane)));
}

// ---------------------------------------------------------------------------
// Host side.

void pd_bf16_launch(const EvalPlan &P, int stage, hipStream_t s) {
  if (stage == 0) {
    if (P.off16P[P.n] > 0) k16_prep<<<P.off16P[P.n], PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16P, P.n);
  } else if (stage == 1) {
    const int total = P.off16A[P.n];
    if (total <= 0) return;  // no rows to evaluate (empty row bands)
    if (P.cert) k16_lse<true><<<total, PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16A, P.n, total);
    else k16_lse<false><<<total, PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16A, P.n, total);
  } else if (stage == 2) {
    const int total = P.off16B[P.n];  // blocks: chunks x ceil(grain groups / 4)
    if (total <= 0) return;
    k16_grad<<<total, PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16B, P.n, total);
  } else {
    k16_reduce<<<P.n + P.off16R[P.n], PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16R, P.n);
  }
}

void pd_bf16_plan_eval(pd_ctx *, const EvalPlan &P, hipStream_t s, bool center) {
  if (center) pd_launch_center(P.d_maps, P.n, P.max_k, s);
  for (int st = 0; st < 4; ++st) pd_bf16_launch(P, st, s);
  if (P.cert) {
    // the FP64 fallback where k16_lse left many pixels undecided, then the
    // canonical scan of the pixels still undecided
    k16_recheck_gate<<<P.n, PD_WAVE, 0, s>>>(P.d_maps, P.n);
    const int total = P.offA[P.n];
    if (total > 0)
    {
      const int blocks = (total + PD_WAVES_PER_BLOCK - 1) / PD_WAVES_PER_BLOCK;
      switch (P.dmax) {
        case 2: k16_recert<2><<<blocks, PD_BLOCK, 0, s>>>(P.d_maps, P.d_offA, P.n, total); break;
        case 4: k16_recert<4><<<blocks, PD_BLOCK, 0, s>>>(P.d_maps, P.d_offA, P.n, total); break;
        default: k16_recert<6><<<blocks, PD_BLOCK, 0, s>>>(P.d_maps, P.d_offA, P.n, total); break;
      }
    }
    pd_launch_assign_list(P.dmax, P.d_maps, P.n, s);
  }
}

pd_status pd_bf16_objective_grad(pd_ctx *ctx, const pd_problem *probs, int n,
                                 const int32_t *rows, const double *const *theta,
                                 double *phi_out, double *const *grad_out, hipStream_t s,
                                 const PlanMemory &mem) {
  for (int p = 0; p < n; ++p)
    if (probs[p].degree > 6)
      return pd_fail(ctx, PD_ERR_UNSUPPORTED, "PD_BF16 supports degree <= 6");
  EvalPlan P;
  Arena L;
  P.target_waves = pd_tuned_waves(ctx, probs, n, 2);
  pd_plan_layout(P, L, probs, n, 2, rows);
  pd_status st = pd_plan_place(ctx, P, L, mem, theta, phi_out, grad_out, s);
  if (st != PD_OK) return st;
  pd_plan_tables(P, s);
  pd_bf16_plan_eval(ctx, P, s, true);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pd_fail(ctx, PD_ERR_HIP, hipGetErrorString(e));
  return PD_OK;
}

void pd_bf16_profile_stages(pd_ctx *, const EvalPlan &P, int reps, hipStream_t s, hipEvent_t *ev) {
  for (int r = 0; r < reps; ++r) pd_bf16_launch(P, 0, s);
  (void)hipEventRecord(ev[1], s);
  for (int r = 0; r < reps; ++r) pd_bf16_launch(P, 1, s);
  (void)hipEventRecord(ev[2], s);
  for (int r = 0; r < reps; ++r) pd_bf16_launch(P, 2, s);
  (void)hipEventRecord(ev[3], s);
}
