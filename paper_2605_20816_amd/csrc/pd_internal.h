// pd_internal.h -- device-side data layout shared by the HIP sources of libpd.
//
// One "map" is one grain map with its parameters.  Every kernel takes an array
// of MapDev records (one per map of the batch) plus prefix offsets of the work
// items each map contributes, so a single launch serves one map or a batch of
// maps of different sizes, grain counts and degrees.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PD_WAVE 64
#define PD_BLOCK 256
#define PD_WAVES_PER_BLOCK (PD_BLOCK / PD_WAVE)
#define PD_DMAX 8
// 32-grain tiles per wave of the matrix-core gradient kernel
#define PD_MF_GROUP_TILES 2

// log2(e) and ln(2) as the nearest doubles.
#define PD_LOG2E 1.4426950408889634074
// Far-field threshold (base-2 logit below the reference): terms 2^s with
// s <= -PD_SKIP_F64 (FP64) or -PD_SKIP_F32 (FP32 exponentials) are left out of
// the sums when a whole chunk of a wave is below it.  A pixel then loses at most
// N 2^-96 (FP64) or N 2^-48 (FP32) of probability mass, below the rounding of
// its sums for any grain count this library takes.
#define PD_SKIP_F64 96.0
#define PD_SKIP_F32 48.0
// Largest grain count whose spatial order is computed (one block's LDS sort).
#define PD_ORDER_MAX 8192
// Logit of the padded grains N .. Npad-1 (their row coefficients are
// (PD_LOGIT_FLOOR, 0, ..., 0)): finite, so that 2^(s - ref) is an ordinary
// argument of the FP64 2^x (which takes no infinities) and gives 0; it converts
// to -inf in FP32.
#define PD_LOGIT_FLOOR (-0x1p1000)
// The FP64 log-sum-exp raises its running reference only when a chunk's largest
// logit exceeds it by more than this (base 2): the terms stay below 2^PD_LAZY_F64
// and the rescaling 2^x runs on the few chunks that move the reference.
#define PD_LAZY_F64 32.0
#define PD_LN2 0.69314718055994530942
// The per-item bodies of the evaluation kernels are always inlined into their
// kernels: a call would pass the map descriptor through the call ABI and lose the
// scalar loads of its wave-uniform data.
#define PD_HOT_INLINE __device__ __attribute__((always_inline)) inline

struct MapDev {
  // problem
  int32_t H, W, N, d, K, DP, Npad;  // DP = d + 1; Npad = N rounded up to 64
  int32_t segs;                     // ceil(W / 64): 64-pixel row segments
  // evaluated rows [row0, row0 + rows): the whole map (0, H), or one slab of it
  // (the share of one device when a map is split by pixel rows).  Coordinates,
  // tables and the 1/n of Phi and grad Phi always refer to the whole H x W map.
  int32_t row0, rows;
  double eps;
  double grad_scale;                // 1 / (eps * n)
  double grad_sign;                 // +1: grad = dPhi/dtheta; -1: its negative (the fit's f = -Phi)
  const int32_t *labels;            // n
  const double *theta;              // N x K
  double *grad;                     // N x K or null
  double *phi;                      // -> phi_out[map]
  // per-evaluation workspace (device)
  double *tx64;                     // [W][DP]  P_a(x1) at each column, FP64
  double *ty64;                     // [H][DP]  P_b(x2) at each row, FP64
  void *txT;                        // [W][DP]  the same in the evaluation type
  double *thc;                      // [N][K]   -log2(e)/eps * (theta_i - mean_j theta_j)
  void *C;                          // [rows][Npad][DP] row coefficients, evaluation type
  void *lse;                        // [rows * W] base-2 log-sum-exp per pixel, evaluation type
  void *rpix;                       // [rows * W] 1 - p_G(x) per pixel (the sum of the other
                                    // grains' probabilities), evaluation type
  double *part_l;                   // [a_items] per-wave partial sums of log2 p_G
  double *part_g;                   // [stiles][Npad][K] partial sums of (p - delta) psi, or of
                                    // p psi when onehot is set
  double *onehot;                   // [N][K] sum of psi over each grain's pixels (FP64), or
                                    // null when the gradient kernel applies the one-hot term
  // gradient tiling: tiles of tile_rows x tile_cols pixels, 64 grains per wave
  int32_t tile_rows, tile_cols, tiles_r, tiles_c;
  // work-item counts and offsets inside the batched launches
  int32_t a_items, a_off;           // row-segment items (objective, assignment)
  int32_t b_items, b_off;           // gradient items: st_size * stiles * (Npad / 64)
  int32_t st_size, stiles;          // tiles per super-tile (4 for degree <= 4, else 1); super-tiles
  int32_t r_items, r_off;           // reduction items: ceil(N*K / 256) blocks
  // assignment
  int32_t *labels_out;              // n or null
  int64_t *n_correct;               // -> n_correct_out[map] or null
  int64_t *part_c;                  // [a_items] per-block (k_assign) or per-wave (certified
                                    // objective launch) correct counts
  // certified accuracy inside the objective launch (the fit; null elsewhere):
  // cert = the largest rounding bound of a logit against the canonical scores
  // (u64 atomic maximum of non-negative doubles, k_prep); pixels whose top two
  // logits are closer than twice that go to unc_list for the canonical arg-min
  // (k_assign_list), whose correct ones are counted in fb_count
  double *cert;
  int32_t *unc_list, *unc_count;    // [rows * W] pixel indices; their number
  float *btile;                     // BF16 fits: per 32-grain tile, the largest error
                                    // bound of its grains' matrix-core logits
  int64_t *fb_count;
  // optional gate: when non-null and zero, every kernel skips this map
  const int32_t *gate;
  // FP32 row table and the BF16 matrix-core path
  void *tyT;                        // [H][DP] P_b(x2) in the evaluation type
  void *T3;                         // [rows][3][Npad][8] bf16 pieces of the row
                                    // coefficients C_a (a <= d, zero beyond)
  float *lse32;                     // [rows * W] base-2 log-sum-exp of the evaluated pixels
  float *part_g32;                  // [rows][Npad][8] per-row gradient moments
                                    // sum_c w_i(r, c) P_a(x1_c) of the BF16 path
  int32_t n32, tiles32;             // evaluated pixels rounded up to 32; 32-pixel
                                    // tiles (ceil(W / 32) per row)
  int32_t a16_items, b16_items;     // blocks of k16_lse; waves of k16_grad
  int32_t chunk_tiles, chunks, ggroups;
  // Hessian diagonal sum_x p_i (1 - p_i) psi_k^2 / (eps^2 n) of -Phi (eq. hess),
  // computed by the gradient kernels when want_diag is non-null and set
  const int32_t *want_diag;
  double *diag;                     // N x K or null
  double *part_d;                   // [stiles][Npad][K] partial sums (FP64/FP32 paths)
  // Hessian-vector product (pd_hessian_vec): the direction v (N x K), its row
  // coefficients Cv (as C), and the per-pixel mean ubar(x) = sum_k p_k(x) v_k . psi(x)
  const double *hv_in;
  void *Cv;
  double *ubar;
  // spatial grain order of the row coefficients (fit-form plans; null = identity):
  // C row j holds grain order[j]; pos is the inverse (labels -> C rows)
  const int32_t *order;
  const int32_t *pos;
  void *order_sums;                 // [3][N] int64 column, row and pixel sums per grain
  // far-field mask of the objective kernel (FP64/FP32 plans): per row segment,
  // mask_words words of one bit per 64-grain group (see row_near)
  uint32_t *nearmask;
  int32_t mask_words;
};


// Run CALL with the compile-time degree D = dval (1..PD_DMAX).
#define PD_DISPATCH_D(dval, CALL)                 \
  switch (dval) {                                 \
    case 1: { constexpr int D = 1; CALL; } break; \
    case 2: { constexpr int D = 2; CALL; } break; \
    case 3: { constexpr int D = 3; CALL; } break; \
    case 4: { constexpr int D = 4; CALL; } break; \
    case 5: { constexpr int D = 5; CALL; } break; \
    case 6: { constexpr int D = 6; CALL; } break; \
    case 7: { constexpr int D = 7; CALL; } break; \
    case 8: { constexpr int D = 8; CALL; } break; \
    default: break;                               \
  }

// The same, restricted to D <= DMAX (a compile-time bound chosen per launch so
// registers are sized for the largest degree actually present).
#define PD_DISPATCH_UPTO(DMAX, dval, CALL)                          \
  switch (dval) {                                                   \
    case 1: if constexpr (DMAX >= 1) { constexpr int D = 1; CALL; } break; \
    case 2: if constexpr (DMAX >= 2) { constexpr int D = 2; CALL; } break; \
    case 3: if constexpr (DMAX >= 3) { constexpr int D = 3; CALL; } break; \
    case 4: if constexpr (DMAX >= 4) { constexpr int D = 4; CALL; } break; \
    case 5: if constexpr (DMAX >= 5) { constexpr int D = 5; CALL; } break; \
    case 6: if constexpr (DMAX >= 6) { constexpr int D = 6; CALL; } break; \
    case 7: if constexpr (DMAX >= 7) { constexpr int D = 7; CALL; } break; \
    case 8: if constexpr (DMAX >= 8) { constexpr int D = 8; CALL; } break; \
    default: break;                                                 \
  }

// Smallest compiled degree bound (2, 4, 6 or 8) covering max_degree.
inline int pd_dmax_bucket(int max_degree) {
  return max_degree <= 2 ? 2 : max_degree <= 4 ? 4 : max_degree <= 6 ? 6 : 8;
}

// XCD-aware block order.  The hardware hands block b of a launch to XCD b % 8
// (each XCD has its own L2).  Within every group of 64 blocks the numbering is
// transposed so that XCD x runs the 8 consecutive logical blocks 64 g + 8 x ..
// 64 g + 8 x + 7: neighbouring work items -- the row segments of one pixel row
// -- share one L2, which then fetches their row coefficients once instead of
// once per XCD, while every XCD still gets its share of each stretch of the
// work list (a batch whose maps cost differently per block stays balanced).
// The last nb % 64 blocks keep their order.  A bijection of [0, nb).
__device__ inline int pd_xcd_block(int b, int nb) {
  if (b >= nb - nb % 64) return b;
  return (b & ~63) + 8 * (b & 7) + ((b >> 3) & 7);
}

// Wave-uniform map lookup: largest m with off[m] <= item (off has n+1 entries).
__device__ inline int pd_find_map(const int32_t *__restrict__ off, int n, int item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Address-space views.  pd_uni: data that is read-only for the whole kernel and
// read at wave-uniform addresses -> scalar loads through the scalar cache.
// pd_glb: per-lane reads and writes -> global (not flat) memory instructions.
#define PD_AS_CONST __attribute__((address_space(4)))
#define PD_AS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ inline const PD_AS_CONST T *pd_uni(const T *p) {
  return (const PD_AS_CONST T *)(p);
}
template <typename T>
__device__ inline PD_AS_GLOBAL T *pd_glb(T *p) {
  return (PD_AS_GLOBAL T *)(p);
}
template <typename T>
__device__ inline const PD_AS_GLOBAL T *pd_glb(const T *p) {
  return (const PD_AS_GLOBAL T *)(p);
}

// True when the map's gate is closed (the map is skipped by every kernel).
#define PD_GATED(M) ((M).gate != nullptr && *pd_uni((M).gate) == 0)

// Index of multi-index alpha = (a, b) in the degree-graded order.
__host__ __device__ constexpr int pd_alpha_index(int a, int b) {
  return (a + b) * (a + b + 1) / 2 + b;
}

// Wave-wide sums through DPP lane moves (no LDS round trips).  Inclusive scans
// over each row of 16 lanes (row_shr 1, 2, 4, 8), then row 1 and 3 add the last
// lane of the row before them (row_bcast:15) and rows 2, 3 add lane 31
// (row_bcast:31): lane 63 holds the total, in a fixed order.
template <int CTRL, int ROW_MASK>
__device__ inline double pd_dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ inline double pd_wave_sum(double v) {
  v += pd_dpp_f64<0x111, 0xf>(v);
  v += pd_dpp_f64<0x112, 0xf>(v);
  v += pd_dpp_f64<0x114, 0xf>(v);
  v += pd_dpp_f64<0x118, 0xf>(v);
  v += pd_dpp_f64<0x142, 0xa>(v);
  v += pd_dpp_f64<0x143, 0xc>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ inline long long pd_wave_sum_i64(long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, PD_WAVE);
  return v;
}

// Host launchers (defined beside their kernels).  prec: 0 = FP64, 1 = FP32.
void pd_launch_tables(int prec, const MapDev *maps, int n_maps, int max_hw, hipStream_t s);
void pd_launch_center(const MapDev *maps, int n_maps, int max_k, hipStream_t s);
void pd_launch_prep(int prec, const MapDev *maps, const int32_t *off, int n_maps, int blocks,
                    hipStream_t s);
void pd_launch_lse(int prec, int dmax, const MapDev *maps, const int32_t *off, int n_maps,
                   int total, hipStream_t s);
// k_lse plus, in as many more blocks, the assignment of amaps (same work list);
// for dmax > 4, k_assign then k_lse.
void pd_launch_lse_assign(int prec, int dmax, const MapDev *maps, const int32_t *off, int n_maps,
                          int total, const MapDev *amaps, hipStream_t s);
// hot: apply the one-hot term in the kernel; otherwise MapDev::onehot must hold
// the indicator moments (pd_launch_onehot) and the reduction subtracts them.
void pd_launch_grad(int prec, int dmax, const MapDev *maps, const int32_t *off, int n_maps,
                    int total, bool diag, bool hot, hipStream_t s);
// k_onehot over the gradient work list, then its fixed-order tile reduction
// into MapDev::onehot (part_g is the scratch).
void pd_launch_onehot(int dmax, const MapDev *maps, const int32_t *off_b, int n_maps, int total,
                      const int32_t *off_r, int blocks_r, hipStream_t s);
void pd_launch_reduce(const MapDev *maps, const int32_t *off_r, int n_maps, int blocks_r,
                      bool grad, bool diag, hipStream_t s);
void pd_launch_features_out(const MapDev *maps, int prec, void *out, long long n, hipStream_t s);
// count: also sum the per-block counts into n_correct (k_reduce_count); the
// fit's decision kernel sums them itself.
void pd_launch_assign(int dmax, const MapDev *maps, const int32_t *off, int n_maps, int total,
                      bool count, hipStream_t s);
// k_lse with the certified arg-max of every pixel (per-wave correct counts in
// part_c, uncertain pixels to unc_list), then k_assign_list on those pixels.
void pd_launch_lse_cert(int prec, int dmax, const MapDev *maps, const int32_t *off, int n_maps,
                        int total, hipStream_t s);
void pd_launch_assign_list(int dmax, const MapDev *maps, int n_maps, hipStream_t s);
// Spatial grain order of maps with non-null order (fit-form plans): per-grain
// centroid sums, then the Morton-order sort (max_px, max_n: the batch's largest
// pixel and grain counts).
void pd_launch_order(const MapDev *maps, int n_maps, long long max_px, int max_n, hipStream_t s);
// Hessian-vector product stages (after the evaluation's tables, thc, C and lse):
// row coefficients of v, the per-pixel means ubar, the per-tile partials of
// sum_x p_i (u_i - ubar) psi into part_g (then the gradient reduction).
void pd_launch_hvp(int prec, int dmax, const MapDev *maps, const int32_t *off_p,
                   const int32_t *off_a, const int32_t *off_b, int n_maps, int blocks_p,
                   int total_a, int total_b, hipStream_t s);
// The certified arg-max pass alone (FP64 row coefficients from k_prep).
void pd_launch_validate(const MapDev *maps, int n_maps, int32_t *bad, hipStream_t s);
