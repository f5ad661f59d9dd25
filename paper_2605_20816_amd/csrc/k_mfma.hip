// k_mfma.hip -- BF16 matrix-core objective/gradient path (v_mfma_f32_32x32x16_bf16).
//
// Logits in base 2, s_i(x) = thc_i . psi(x) with thc = -(log2 e / eps)(theta -
// mean), are a GEMM with inner dimension K (padded to 16 or 32).  At eps = 1e-3
// the logits reach |s| ~ 1e3..1e4 while the softmax needs them to ~1e-3, i.e.
// about 22 significant bits.  Both operands are therefore split into three
// bf16 pieces (hi + mid + lo, each the rounding of the remainder) and the six
// products of total order <= 2 (hh, hm, mh, hl, lh, mm) are accumulated in FP32;
// the dropped terms are below 2^-26 relative.  The gradient contraction
// sum_x (p_i(x) - delta_{i,G(x)}) psi(x) multiplies values of size <= 1: p - delta
// as two FP16 pieces against the two FP16 pieces of psi, on
// v_mfma_f32_32x32x16_f16.  Log-sum-exp in FP32; Phi and grad Phi are summed in
// FP64 in a fixed order.
//
// Operand/accumulator lane layout of the 32x32x16 instruction (lane l, half
// h = l / 32): A[i][k] at lane i + 32 (k / 8), element k % 8; B[k][j] at lane
// j + 32 (k / 8), element k % 8; D[i][j] at lane j + 32 ((i / 4) % 2),
// register 4 (i / 8) + i % 4.
//
// k16_lse:  block = 4 waves x 4 pixel tiles of 32 pixels; the three pieces of
//           thc for 128 grains at a time are staged in LDS and shared; S = thc
//           psi^T puts one pixel per lane column and 16 grains per lane, so the
//           online max / sum of exp2 stays in-lane (halves merged at the end).
// k16_grad: wave = (pixel chunk, 64 grains); thc pieces and the 2 x 32 x 32
//           gradient accumulators stay in registers across the chunk; S^T = psi
//           thc^T puts one grain per lane column, so p - delta feeds the gradient
//           product directly as its A operand.
#include "pd_host.h"

#include <math.h>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#define MF_TILES_PER_WAVE 4     // pixel tiles per wave in k16_lse
#define MF_GRAIN_STAGE 128      // grains staged in LDS per step of k16_lse

// Exponents (a, b) of feature k in the degree-graded order (degree <= 8).
__constant__ signed char c_fa[45] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0,
                                     5, 4, 3, 2, 1, 0, 6, 5, 4, 3, 2, 1, 0,
                                     7, 6, 5, 4, 3, 2, 1, 0, 8, 7, 6, 5, 4, 3, 2, 1, 0};
__constant__ signed char c_fb[45] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4,
                                     0, 1, 2, 3, 4, 5, 0, 1, 2, 3, 4, 5, 6,
                                     0, 1, 2, 3, 4, 5, 6, 7, 0, 1, 2, 3, 4, 5, 6, 7, 8};

__device__ inline float bf_to_f(__bf16 h) { return (float)h; }

// Exponents of feature k in the graded order, at compile time.
__host__ __device__ constexpr int feat_deg(int k) {
  int d = 0;
  while ((d + 1) * (d + 2) / 2 <= k) ++d;
  return d;
}
__host__ __device__ constexpr int feat_b(int k) { return k - feat_deg(k) * (feat_deg(k) + 1) / 2; }
__host__ __device__ constexpr int feat_a(int k) { return feat_deg(k) - feat_b(k); }

// Row and column of flat pixel pbase + o from those of pbase (o < 32).
__device__ inline void pix_rc(int r0, int c0, int o, int W, int &r, int &c) {
  c = c0 + o;
  r = r0;
  while (c >= W) {
    c -= W;
    ++r;
  }
}

// P_a(x1) and P_b(x2) of one pixel for a, b <= the largest exponent that the
// 16 * NKB features need (zero beyond the degree or outside the map).
template <int NKB>
struct PixTables {
  static constexpr int AM = feat_deg(16 * NKB - 1);
  float px[AM + 1], py[AM + 1];
};
template <int NKB>
__device__ inline void pixel_tables(const MapDev &M, int r, int c, bool valid, PixTables<NKB> &t) {
  // global (not flat) loads: they must not hold up the LDS waits of the
  // products that run while they are in flight
  const auto tx = pd_glb((const float *)M.txT), ty = pd_glb((const float *)M.tyT);
#pragma unroll
  for (int a = 0; a <= PixTables<NKB>::AM; ++a) {
    t.px[a] = (valid && a <= M.d) ? tx[c * M.DP + a] : 0.f;
    t.py[a] = (valid && a <= M.d) ? ty[r * M.DP + a] : 0.f;
  }
}
// The 8 features of block kb for lane half h: v[kb][e] = psi_{16 kb + 8 h + e}
// (zero beyond K).
template <int NKB>
__device__ inline void feats_from_tables(const MapDev &M, const PixTables<NKB> &t, int half,
                                         float (&v)[NKB][8]) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k0 = 16 * kb + e, k1 = 16 * kb + 8 + e;
      const float f0 = t.px[feat_a(k0)] * t.py[feat_b(k0)];
      const float f1 = t.px[feat_a(k1)] * t.py[feat_b(k1)];
      const float f = half ? f1 : f0;
      const int k = half ? k1 : k0;
      v[kb][e] = k < M.K ? f : 0.f;
    }
}
// All 16 * NKB features of one pixel, the 8 of block kb for lane half h.
template <int NKB>
__device__ inline void pixel_feats(const MapDev &M, int r, int c, bool valid, int half,
                                   float (&v)[NKB][8]) {
  PixTables<NKB> t;
  pixel_tables<NKB>(M, r, c, valid, t);
  feats_from_tables<NKB>(M, t, half, v);
}

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

__device__ inline void split2(const float (&v)[8], bf16x8 &h, bf16x8 &l) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 a = (__bf16)v[e];
    h[e] = a;
    l[e] = (__bf16)(v[e] - bf_to_f(a));
  }
}

// acc += (ah + am + al)(bh + bm + bl) up to second-order terms, small first.
__device__ inline f32x16 mfma6(const bf16x8 &ah, const bf16x8 &am, const bf16x8 &al,
                               const bf16x8 &bh, const bf16x8 &bm, const bf16x8 &bl, f32x16 acc) {
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
  return acc;
}

// ---------------------------------------------------------------------------
// thc (FP64, N x K) -> three bf16 pieces [3][Npad][Kp], zero-padded.
__global__ __launch_bounds__(PD_BLOCK) void k16_prep(const MapDev *__restrict__ maps,
                                                     const int32_t *__restrict__ off, int n_maps) {
  const int m = pd_find_map(off, n_maps, blockIdx.x);
  const MapDev &M = maps[m];
  if (PD_GATED(M)) return;
  const long long e = (long long)(blockIdx.x - off[m]) * PD_BLOCK + threadIdx.x;
  const long long tot = (long long)M.Npad * M.Kp;
  if (e >= tot) return;
  const int i = (int)(e / M.Kp), k = (int)(e - (long long)i * M.Kp);
  const double v = (i < M.N && k < M.K) ? M.thc[(size_t)i * M.K + k] : 0.0;
  const __bf16 h = (__bf16)(float)v;
  const double r1 = v - (double)bf_to_f(h);
  const __bf16 md = (__bf16)(float)r1;
  const double r2 = r1 - (double)bf_to_f(md);
  const __bf16 lo = (__bf16)(float)r2;
  __bf16 *T = (__bf16 *)M.T3;
  T[e] = h;
  T[tot + e] = md;
  T[2 * tot + e] = lo;
}

// ---------------------------------------------------------------------------
template <int NKB>
__device__ inline void lse16_block(const MapDev &M, int blk, __bf16 *sT) {
  constexpr int TPW = MF_TILES_PER_WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / PD_WAVE);
  const int lane = threadIdx.x % PD_WAVE;
  const int half = lane / 32, col = lane % 32;
  const int Kp = M.Kp;
  const int tile0 = blk * (4 * TPW) + wave * TPW;
  // B operands: psi^T of this wave's tiles (pixel = column), three pieces
  bf16x8 bh[TPW][NKB], bm[TPW][NKB], bl[TPW][NKB];
  // p: index among the evaluated pixels (rows row0 .. row0 + rows - 1, row-major);
  // q = pix0 + p: index in the whole map
  const int npx = M.rows * M.W, pix0 = M.row0 * M.W;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int p = (tile0 + t) * 32 + col;
    const int q = pix0 + p;
    const int r = q / M.W, c = q - r * M.W;
    float v[NKB][8];
    pixel_feats<NKB>(M, r, c, p < npx, half, v);
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) split3(v[kb], bh[t][kb], bm[t][kb], bl[t][kb]);
  }
  // S sums over the grains other than the pixel's label (r = 1 - p_G, below)
  float mrun[TPW], S[TPW];
  int lab[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    mrun[t] = -INFINITY;
    S[t] = 0.f;
    const int p = (tile0 + t) * 32 + col;
    lab[t] = p < npx ? pd_glb(M.labels)[pix0 + p] : -1;
  }
  const long long tot = (long long)M.Npad * Kp;
  const __bf16 *T = (const __bf16 *)M.T3;
  for (int g0 = 0; g0 < M.Npad; g0 += MF_GRAIN_STAGE) {
    const int gcnt = min(MF_GRAIN_STAGE, M.Npad - g0);
    __syncthreads();
    // stage the three pieces of grains [g0, g0 + gcnt): sT[piece][g][Kp]
    const int words = gcnt * Kp / 8;  // 16-byte units per piece
    for (int w = threadIdx.x; w < 3 * words; w += PD_BLOCK) {
      const int piece = w / words, q = w - piece * words;
      const bf16x8 v = *(const bf16x8 *)(T + piece * tot + (size_t)g0 * Kp + (size_t)q * 8);
      *(bf16x8 *)(sT + (size_t)piece * MF_GRAIN_STAGE * Kp + (size_t)q * 8) = v;
    }
    __syncthreads();
    for (int gt = 0; gt < gcnt; gt += 32) {
      bf16x8 ah[NKB], am[NKB], al[NKB];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        const size_t o = (size_t)(gt + col) * Kp + kb * 16 + half * 8;
        ah[kb] = *(const bf16x8 *)(sT + o);
        am[kb] = *(const bf16x8 *)(sT + (size_t)MF_GRAIN_STAGE * Kp + o);
        al[kb] = *(const bf16x8 *)(sT + (size_t)2 * MF_GRAIN_STAGE * Kp + o);
      }
      const int gbase = g0 + gt;
      const bool partial = gbase + 32 > M.N;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        f32x16 acc;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.f;
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
          acc = mfma6(ah[kb], am[kb], al[kb], bh[t][kb], bm[t][kb], bl[t][kb], acc);
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
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const float mo = __shfl_xor(mrun[t], 32, PD_WAVE);
    const float so = __shfl_xor(S[t], 32, PD_WAVE);
    const float mm = fmaxf(mrun[t], mo);
    // the other grains' sum (both halves), then the label's own term
    const float sx = S[t] * __builtin_amdgcn_exp2f(mrun[t] - mm) + so * __builtin_amdgcn_exp2f(mo - mm);
    const int p = (tile0 + t) * 32 + col;
    if (half == 0 && p < M.n32) {
      float lse = INFINITY, rr = 0.f;
      if (p < npx) {
        const int q = pix0 + p;
        const int g = lab[t];
        if (g >= 0 && g < M.N) {
          // exact FP64 logit of the true grain
          const int r = q / M.W, c = q - r * M.W;
          const double *px = M.tx64 + (size_t)c * M.DP, *py = M.ty64 + (size_t)r * M.DP;
          const double *th = M.thc + (size_t)g * M.K;
          double sg = 0.0;
          for (int k = 0; k < M.K; ++k) sg = __builtin_fma(th[k], px[c_fa[k]] * py[c_fb[k]], sg);
          const float tot = sx + __builtin_amdgcn_exp2f((float)(sg - (double)mm));
          lse = mm + __builtin_amdgcn_logf(tot);
          rr = sx / tot;
          ell += sg - (double)lse;
        } else {
          lse = mm + __builtin_amdgcn_logf(sx);
          ell = NAN;
        }
      }
      pd_glb(M.lse32)[p] = lse;
      pd_glb((float *)M.rpix)[p] = rr;
    }
  }
  const double tot_l = pd_wave_sum(ell);
  if (lane == 0) pd_glb(M.part_l)[blk * 4 + wave] = tot_l;
}

template <int NKB>
__global__ __launch_bounds__(PD_BLOCK) void k16_lse(const MapDev *__restrict__ maps,
                                                    const int32_t *__restrict__ off, int n_maps,
                                                    int total) {
  __shared__ __align__(16) __bf16 sT[3 * MF_GRAIN_STAGE * 16 * NKB];
  if ((int)blockIdx.x >= total) return;
  const int m = pd_find_map(off, n_maps, blockIdx.x);
  const MapDev &M = maps[m];
  if (PD_GATED(M)) return;
  lse16_block<NKB>(M, blockIdx.x - off[m], sT);
}

// ---------------------------------------------------------------------------
// k16_grad: block = 4 waves on one pixel chunk, wave w on grain group 4 q + w.
// Per 32-pixel tile the four waves build the shared operands once in LDS (two
// buffers: tile t + 1 is built while tile t's products run):
//   sA  [3][NKB][64] x 16 B : psi rows (pixel = row) for the logit product
//   sQ  [2][2][64]   x 16 B : psi^T (feature = column) in FP16 hi/lo for the
//                             gradient product, inner index h*8+e of block kb2
//                             = pixel 16 kb2 + 8 (e / 4) + 4 h + e % 4
//   sL, sR, sG [32]         : lse, r = 1 - p_G and label of the tile's pixels
// The gradient product takes the weight p (other grains) or -r (the pixel's
// own grain: p - 1 without the cancellation near p = 1) as two FP16 pieces
// (hi + lo, about 22 bits), scaled by 2^PD_MF_WSHIFT so that small weights stay
// normal, against the two FP16 pieces of psi (three products: the lo x lo term is
// below 2^-22); the scale is taken out of the FP32 partial sums.  One FP16 piece
// (2^-12 relative per weight) put the gradient at a fitted iterate, where p - delta
// cancels most, at the edge of a 2e-3 tolerance.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

#define PD_MF_WSHIFT 12
struct GradLds {
  bf16x8 A[3][2][64];
  f16x8 Q[2][2][64];
  float L[32];
  float R[32];
  int G[32];
  int lo, hi;
};

template <int NKB>
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
  const int Kp = M.Kp;
  const long long tot = (long long)M.Npad * Kp;
  const __bf16 *T = (const __bf16 *)M.T3;
  bf16x8 th[GT][NKB], tm[GT][NKB], tl[GT][NKB];
#pragma unroll
  for (int t = 0; t < GT; ++t) {
    const int g = min(g0 + t * 32 + col, M.Npad - 1);
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      const size_t o = (size_t)g * Kp + kb * 16 + half * 8;
      th[t][kb] = *(const bf16x8 *)(T + o);
      tm[t][kb] = *(const bf16x8 *)(T + tot + o);
      tl[t][kb] = *(const bf16x8 *)(T + 2 * tot + o);
    }
  }
  f32x16 accg[GT];
#pragma unroll
  for (int t = 0; t < GT; ++t)
#pragma unroll
    for (int j = 0; j < 16; ++j) accg[t][j] = 0.f;
  const int npx = M.rows * M.W, pix0 = M.row0 * M.W;  // evaluated pixels, first one
  const int pt0 = chunk * M.chunk_tiles;
  const int pt1 = min(pt0 + M.chunk_tiles, M.tiles32);
  const int fcol = col < M.K ? col : 0;
  const int fa = c_fa[fcol], fb = c_fb[fcol];
  const bool fvalid = col < M.K;
  const float *txf = (const float *)M.txT, *tyf = (const float *)M.tyT;
  auto compute_tile = [&](const GradLds &S) {
    bf16x8 ph[NKB], pm[NKB], pl[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      ph[kb] = S.A[0][kb][lane];
      pm[kb] = S.A[1][kb][lane];
      pl[kb] = S.A[2][kb][lane];
    }
    float lrow[16];
    int grow[16];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        lrow[4 * b + r] = S.L[8 * b + 4 * half + r];
        grow[4 * b + r] = S.G[8 * b + 4 * half + r];
      }
    constexpr float wscale = (float)(1 << PD_MF_WSHIFT);
    f32x16 acc[GT];
#pragma unroll
    for (int t = 0; t < GT; ++t)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[t][j] = 0.f;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
#pragma unroll
      for (int t = 0; t < GT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pm[kb], tm[t][kb], acc[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < GT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl[kb], th[t][kb], acc[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < GT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph[kb], tl[t][kb], acc[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < GT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pm[kb], th[t][kb], acc[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < GT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph[kb], tm[t][kb], acc[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < GT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph[kb], th[t][kb], acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < GT; ++t)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[t][j] = __builtin_amdgcn_exp2f(acc[t][j] - lrow[j]) * wscale;
    if (S.hi >= g0 && S.lo < g0 + GT * 32) {
      float rrow[16];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) rrow[4 * b + r] = S.R[8 * b + 4 * half + r];
#pragma unroll
      for (int t = 0; t < GT; ++t) {
        const int grain = g0 + t * 32 + col;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[t][j] = (grow[j] == grain) ? -rrow[j] * wscale : acc[t][j];
      }
    }
#pragma unroll
    for (int kb2 = 0; kb2 < 2; ++kb2) {
      const f16x8 qh = S.Q[kb2][0][lane], ql = S.Q[kb2][1][lane];
      f16x8 x[GT], xl[GT];
#pragma unroll
      for (int t = 0; t < GT; ++t)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          // the weight rounded to FP32, then split into two FP16 pieces (as above,
          // no fused form)
          float q = acc[t][8 * kb2 + e];
          asm volatile("" : "+v"(q));
          const _Float16 h = (_Float16)q;
          x[t][e] = h;
          xl[t][e] = (_Float16)(q - (float)h);
        }
      // (w_hi + w_lo)(psi_hi + psi_lo) without w_lo psi_lo, small terms first
#pragma unroll
      for (int t = 0; t < GT; ++t) accg[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(xl[t], qh, accg[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < GT; ++t) accg[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(x[t], ql, accg[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < GT; ++t) accg[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(x[t], qh, accg[t], 0, 0, 0);
    }
  };
  // Per tile the waves' roles: wave 0 the psi rows, waves 1-2 the psi^T pieces,
  // wave 3 lse and labels.  The global data of tile pt + 1 is loaded before tile
  // pt's products and written to the other LDS buffer after them, so one
  // barrier per tile separates building from use.
  PixTables<NKB> tab;     // wave 0
  float qx[8], qy[8];     // waves 1-2
  float lse_l = 0.f;      // wave 3 (lanes < 32)
  float r_l = 0.f;
  int lab_l = -1;
  auto load_tile = [&](int pt) {
    const int pbase = pt * 32;
    const int r0 = (pix0 + pbase) / M.W, c0 = pix0 + pbase - r0 * M.W;
    if (wave == 0) {
      int r, c;
      pix_rc(r0, c0, col, M.W, r, c);
      pixel_tables<NKB>(M, r, c, pbase + col < npx, tab);
    } else if (wave <= 2) {
      const int kb2 = wave - 1;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int o = 16 * kb2 + 8 * (e / 4) + 4 * half + (e % 4);
        int r, c;
        pix_rc(r0, c0, o, M.W, r, c);
        const bool ok = fvalid && pbase + o < npx;
        qx[e] = ok ? pd_glb(txf)[c * M.DP + fa] : 0.f;
        qy[e] = ok ? pd_glb(tyf)[r * M.DP + fb] : 0.f;
      }
    } else if (lane < 32) {
      const int p = pbase + lane;
      lse_l = pd_glb(M.lse32)[p];
      r_l = pd_glb((const float *)M.rpix)[p];
      lab_l = p < npx ? pd_glb(M.labels)[pix0 + p] : -1;
    }
  };
  auto build_tile = [&](GradLds &S) {
    if (wave == 0) {
      float v[NKB][8];
      feats_from_tables<NKB>(M, tab, half, v);
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) split3(v[kb], S.A[0][kb][lane], S.A[1][kb][lane], S.A[2][kb][lane]);
    } else if (wave <= 2) {
      const int kb2 = wave - 1;
      f16x8 qh, ql;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        // psi in FP32 first, then its two FP16 pieces (the empty asm keeps the
        // product from being folded into a mixed-precision FMA that would round
        // it to FP16 once, without the FP32 step)
        float v = qx[e] * qy[e];
        asm volatile("" : "+v"(v));
        const _Float16 h = (_Float16)v;
        qh[e] = h;
        ql[e] = (_Float16)(v - (float)h);
      }
      S.Q[kb2][0][lane] = qh;
      S.Q[kb2][1][lane] = ql;
    } else {
      int g = -1, lo = 0x7fffffff, hi = -1;
      if (lane < 32) {
        S.L[lane] = lse_l;
        S.R[lane] = r_l;
        g = lab_l;
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
  for (int pt = pt0; pt < pt1; ++pt) {
    GradLds &cur = sh[(pt - pt0) & 1];
    if (pt + 1 < pt1) load_tile(pt + 1);
    __syncthreads();  // cur is built; the other buffer's readers (tile pt - 1) are done
    if (active) {
      compute_tile(cur);
    }
    if (pt + 1 < pt1) build_tile(sh[(pt - pt0 + 1) & 1]);
  }
  if (!active) return;
  // accg[t]: rows = grains g0 + 32 t + (8 b + 4 h + r), column = feature col
  const int FW = 32;
  float *out = M.part_g32 + (size_t)chunk * M.Npad * FW;
#pragma unroll
  for (int t = 0; t < GT; ++t) {
    if (t >= gtn) break;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int g = g0 + t * 32 + (j / 4) * 8 + half * 4 + (j % 4);
      pd_glb(out)[(size_t)g * FW + col] = accg[t][j] * (1.f / (float)(1 << PD_MF_WSHIFT));
    }
  }
}

template <int NKB>
__global__ __launch_bounds__(PD_BLOCK) void k16_grad(const MapDev *__restrict__ maps,
                                                     const int32_t *__restrict__ off, int n_maps,
                                                     int total) {
  __shared__ GradLds sh[2];
  if ((int)blockIdx.x >= total) return;
  const int m = pd_find_map(off, n_maps, blockIdx.x);
  const MapDev &M = maps[m];
  if (PD_GATED(M)) return;
  grad16_block<NKB>(M, blockIdx.x - off[m], sh);
}

// Phi from the per-wave partials, grad from the chunk partials (fixed order).
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
  // 16 consecutive outputs x 16 chunk phases; phase sums added by a fixed tree
  __shared__ double red[16][17];
  const int ol = threadIdx.x % 16, ph = threadIdx.x / 16;
  const int o = (b - off[m]) * 16 + ol;
  double s = 0.0;
  if (o < M.N * M.K) {
    const int i = o / M.K, k = o - i * M.K;
    const size_t stride = (size_t)M.Npad * 32;
    const auto src = pd_glb(M.part_g32 + (size_t)i * 32 + k);
    for (int c = ph; c < M.chunks; c += 16) s += (double)src[(size_t)c * stride];
  }
  red[ph][ol] = s;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (ph < w) red[ph][ol] += red[ph + w][ol];
    __syncthreads();
  }
  if (ph == 0 && o < M.N * M.K) M.grad[o] = red[0][ol] * (M.grad_scale * M.grad_sign);
}

// ---------------------------------------------------------------------------
// Host side.

static int nkb_for(int dmax) { return dmax <= 4 ? 1 : 2; }

void pd_bf16_launch(const EvalPlan &P, int stage, hipStream_t s) {
  const int nkb = nkb_for(P.dmax);
  if (stage == 0) {
    k16_prep<<<P.off16P[P.n], PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16P, P.n);
  } else if (stage == 1) {
    const int total = P.off16A[P.n];
    if (total <= 0) return;  // no rows to evaluate (empty row bands)
    if (nkb == 1) k16_lse<1><<<total, PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16A, P.n, total);
    else k16_lse<2><<<total, PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16A, P.n, total);
  } else if (stage == 2) {
    const int total = P.off16B[P.n];  // blocks: chunks x ceil(grain groups / 4)
    if (total <= 0) return;
    if (nkb == 1) k16_grad<1><<<total, PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16B, P.n, total);
    else k16_grad<2><<<total, PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16B, P.n, total);
  } else {
    k16_reduce<<<P.n + P.off16R[P.n], PD_BLOCK, 0, s>>>(P.d_maps, P.d_off16R, P.n);
  }
}

void pd_bf16_plan_eval(pd_ctx *, const EvalPlan &P, hipStream_t s, bool center) {
  if (center) pd_launch_center(P.d_maps, P.n, P.max_k, s);
  for (int st = 0; st < 4; ++st) pd_bf16_launch(P, st, s);
  if (P.cert) {
    // the certified arg-max of every pixel (FP64 row coefficients), as in the
    // FP64 evaluation of a fit
    pd_launch_prep(0, P.d_maps, P.d_offP, P.n, P.offP[P.n], s);
    pd_launch_cert_argmax(P.dmax, P.d_maps, P.d_offA, P.n, P.offA[P.n], s);
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
